// lks_device.h -- device-side building blocks shared by the gfx950 kernels:
// velocity sets, grid/boundary geometry, the mapping weight, the rigid-body pose.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lks {

enum { BC_PERIODIC = 0, BC_VELOCITY = 1, BC_PRESSURE = 2, BC_WALL = 3 };

// Body record layout (12 doubles). The first 8 entries are the ABI body state; the
// library keeps cos(theta), sin(theta) of the same record in slots 8, 9.
enum { B_XG = 0, B_UG = 3, B_TH = 6, B_OM = 7, B_COS = 8, B_SIN = 9, B_REC = 12 };

// ------------------------------------------------------------ velocity sets
// D2Q9 / D3Q15 (Sec. 2.2): rest, axis directions, diagonals / cube corners.
template <int DIM> struct Lat;

template <> struct Lat<2> {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};

template <> struct Lat<3> {
    static constexpr int Q = 15;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[15][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},   {0, 0, -1},  {1, 1, 1},   {1, 1, -1}, {1, -1, 1},
                                  {1, -1, -1}, {-1, 1, 1},  {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 2.0 / 9.0 : (i < 7 ? 1.0 / 9.0 : 1.0 / 72.0);
    }
};

// ------------------------------------------------------------ geometry
// The velocity field is held as its deviation v = u - U from a constant reference
// velocity U (the velocity prescribed on the first VELOCITY face, else zero): every
// kernel that needs the velocity itself adds U back. The equilibrium of a uniform flow
// U streams into itself (p* = 0, u* = U), so the LKS update of v involves only small
// quantities; in FP32 the fields then keep their relative precision on the small
// transverse velocities and pressure that drive the body, instead of rounding them
// against |U|.
struct Grid {
    int n[3];
    int per[3];      // axis is periodic (2D: z counts as periodic)
    long long N;
    double U[3];     // reference velocity of the stored deviation
    float Uf[3];     // the same rounded to float (kernel arguments, no conversion on the device)
};

// U_a in the arithmetic type of a kernel.
template <typename T> __device__ __forceinline__ T gU(const Grid &g, int a);
template <> __device__ __forceinline__ float gU<float>(const Grid &g, int a) { return g.Uf[a]; }
template <> __device__ __forceinline__ double gU<double>(const Grid &g, int a) { return g.U[a]; }

struct Bc {
    int kind[6];
    double p[6];
    double u[6][3];
};

__device__ __forceinline__ long long node_id(const Grid &g, int x, int y, int z) {
    return (long long)x + (long long)g.n[0] * ((long long)y + (long long)g.n[1] * z);
}

// Wrap a coordinate on a periodic axis; report whether it lies on the grid.
__device__ __forceinline__ bool wrap_coord(int &v, int n, int per) {
    if (per) {
        if (v < 0) v += n;
        else if (v >= n) v -= n;
        return v >= 0 && v < n;
    }
    return v >= 0 && v < n;
}

// Raw buffer access (gfx9 buffer resource, untyped dword access): a load at a byte
// offset at or past the resource's size returns 0 and such a store is dropped, so a lane
// is switched off by giving it the offset BOFF_NONE (the resource sizes used stay below
// it). Offsets are 32-bit and the base is wave-uniform, so the per-lane address needs
// no 64-bit arithmetic.
constexpr unsigned BOFF_NONE = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0);
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, (int)soff, 0);
}

// Span of a sampled launch on the constant-rate wall clock: ts[0] keeps the earliest
// block start, ts[1] the latest block end (preset to all-ones and zero on the host
// side). Blocks are dispatched in index order and do equal work here, so the first 64
// blocks stamp the start and the last 64 the end (a bounded number of atomics on the
// two slots, whatever the grid). span_end waits for the whole block; every thread
// calls both, and the kernels that use them have no early returns.
__device__ __forceinline__ unsigned span_block() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ void span_begin(unsigned long long *ts) {
    if (ts && threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0 && span_block() < 64)
        atomicMin(&ts[0], (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void span_end(unsigned long long *ts) {
    if (ts) {
        __syncthreads();
        const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0 && span_block() + 64 >= nb)
            atomicMax(&ts[1], (unsigned long long)wall_clock64());
    }
}

// Workgroups are handed out round-robin over the eight XCDs (workgroup b, counted x
// fastest, runs on XCD b mod 8), and each XCD has its own L2. Renumber the tiles so
// that XCD j gets the j-th contiguous run of them (x fastest): neighbouring tiles then
// share their halo lines in one L2 instead of fetching them twice.
__device__ __forceinline__ uint3 xcd_tile() {
    const unsigned gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
    const unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned per = nb >> 3, rem = nb & 7, x = b & 7;
    const unsigned t = x * per + min(x, rem) + (b >> 3);
    return make_uint3(t % gx, (t / gx) % gy, t / (gx * gy));
}

// The same renumbering for grids of independent work items (design points, box rows):
// the logical block of this workgroup, so that XCD j runs the j-th contiguous run of
// logical blocks and the footprint fields a run touches stay in one L2. Over a 2D grid
// (blockIdx.y a second index) the linear order x fastest is renumbered and split again.
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned nb = gridDim.x * gridDim.y, b = blockIdx.x + gridDim.x * blockIdx.y;
    const unsigned per = nb >> 3, rem = nb & 7, x = b & 7;
    return x * per + min(x, rem) + (b >> 3);
}

template <int DIM>
__device__ __forceinline__ bool is_interior(const Grid &g, const int x[3]) {
#pragma unroll
    for (int a = 0; a < DIM; a++)
        if (!g.per[a] && (x[a] == 0 || x[a] == g.n[a] - 1)) return false;
    return true;
}

// Resolution of a boundary (non-interior) node: prescribed p and/or u and the
// nearest interior node that supplies what is not prescribed. WALL beats VELOCITY.
struct BcNode {
    bool p_fixed, u_fixed;
    double p, u[3];
    int in[3];
};

template <int DIM>
__device__ __forceinline__ void bc_resolve(const Grid &g, const Bc &bc, const int x[3], BcNode &r) {
    bool wall = false;
    int vel = -1, pres = -1;
    r.in[0] = x[0];
    r.in[1] = x[1];
    r.in[2] = x[2];
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        if (g.per[a]) continue;
        int f = -1;
        if (x[a] == 0) {
            f = 2 * a;
            r.in[a] = 1;
        } else if (x[a] == g.n[a] - 1) {
            f = 2 * a + 1;
            r.in[a] = g.n[a] - 2;
        }
        if (f < 0) continue;
        const int k = bc.kind[f];
        if (k == BC_WALL) wall = true;
        if (k == BC_VELOCITY && vel < 0) vel = f;
        if (k == BC_PRESSURE && pres < 0) pres = f;
    }
    r.p_fixed = pres >= 0;
    r.p = pres >= 0 ? bc.p[pres] : 0.0;
    r.u_fixed = wall || vel >= 0;
#pragma unroll
    for (int a = 0; a < 3; a++) r.u[a] = wall ? 0.0 : (vel >= 0 ? bc.u[vel][a] : 0.0);
}

// ------------------------------------------------------------ mapping weight
// Eq. weight_function read as the cosine kernel w(r) = (1 + cos(pi r / 2)) / 4 on
// |r| < 2, and its derivative -(pi/8) sin(pi r / 2).
//
//
// FP32 uses the hardware sine and cosine (v_sin_f32 / v_cos_f32, argument in
// revolutions); FP64 uses cospi / sinpi.
__device__ __forceinline__ float wk(float r) {
    // the hardware cosine takes revolutions: cos(pi r / 2) = cos(2 pi (r / 4))
    const float c = __builtin_amdgcn_cosf(0.25f * r);
    return fabsf(r) < 2.0f ? fmaf(0.25f, c, 0.25f) : 0.0f;
}
__device__ __forceinline__ float dwk(float r) {
    const float s = __builtin_amdgcn_sinf(0.25f * r);
    return fabsf(r) < 2.0f ? -0.39269908169872414f * s : 0.0f;
}
__device__ __forceinline__ double wk(double r) {
    return fabs(r) < 2.0 ? 0.25 * (1.0 + cospi(0.5 * r)) : 0.0;
}
__device__ __forceinline__ double dwk(double r) {
    return fabs(r) < 2.0 ? -0.39269908169872414 * sinpi(0.5 * r) : 0.0;
}

// ------------------------------------------------------------ design grid and pose
struct Design {
    int nd[3];
    long long ND;
    double half[3];   // (nd - 1) / 2: index of the rotation centre
    int axis, pi, pj; // rotation axis and its (right-handed) plane
    int H[3];         // footprint box: origin floor(x^G) - H, size L
    int L[3];
    long long boxN;
    int margin;       // allowed drift of x^G within a step
};

// Eqs. rigid_body_position / rigid_body_velocity (rotation about `axis` through x^G):
// r = R(theta) xi, x^ref = x^G + r, u^S,ref = u^G + omega (a x r). FP64.
struct Pose {
    double X[3], US[3], r[3], axr[3];
};

template <int DIM>
__device__ __forceinline__ void design_xi(const Design &D, long long m, double xi[3]) {
    // ND < 2^31 (checked on the host): 32-bit division
    const unsigned mu = (unsigned)m, n0 = (unsigned)D.nd[0], n1 = (unsigned)D.nd[1];
    const unsigned r = mu / n0;
    const unsigned i = mu - r * n0, j = r % n1, k = r / n1;
    xi[0] = (double)i - D.half[0];
    xi[1] = (double)j - D.half[1];
    xi[2] = DIM == 3 ? (double)k - D.half[2] : 0.0;
}

// Select-based access to 3-vectors by a runtime axis index (keeps them in registers).
template <typename T> __device__ __forceinline__ T pick3(const T v[3], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

__device__ __forceinline__ void pose_point(const Design &D, const double *B, const double xi[3],
                                           Pose &o) {
    // No contraction: the spread (gather form) and the interpolation evaluate the
    // same positions in different kernels and must agree bit for bit.
#pragma clang fp contract(off)
    const double c = B[B_COS], s = B[B_SIN], om = B[B_OM];
    const double xa = pick3(xi, D.axis), xp = pick3(xi, D.pi), xq = pick3(xi, D.pj);
    const double ra = xa, rp = c * xp - s * xq, rq = s * xp + c * xq;
#pragma unroll
    for (int b = 0; b < 3; b++) {
        o.r[b] = b == D.axis ? ra : (b == D.pi ? rp : rq);
        o.axr[b] = b == D.axis ? 0.0 : (b == D.pi ? -rq : rp);
        o.X[b] = B[B_XG + b] + o.r[b];
        o.US[b] = B[B_UG + b] + om * o.axr[b];
    }
}

// Footprint box of a step from the body state at t-1.
template <int DIM>
__device__ __forceinline__ void box_origin(const Design &D, const double *Bprev, int o[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++)
        o[a] = (a < DIM) ? (int)floor(Bprev[B_XG + a]) - D.H[a] : 0;
}

// Brinkman interpolation, Eq. brinkman_coefficient, and its derivative.
__host__ __device__ __forceinline__ double kappa_of(double kmax, double q, double g) {
    return kmax * q * g / ((1.0 - g) + q);
}
__host__ __device__ __forceinline__ double dkappa_of(double kmax, double q, double g) {
    const double den = (1.0 - g) + q;
    return kmax * q * (1.0 + q) / (den * den);
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Neumaier-compensated running sum.
struct Kahan {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x) {
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

}  // namespace lks
