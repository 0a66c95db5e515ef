// filter.h -- density filter and Heaviside projection of the design field (Sec. 3.2,
// Eqs. filter and projection) and their reverse, on the design grid (spacing one).
//
//   gt_i = sum_j w_ij g_j / W_i,  w_ij = (R - |x_i - x_j|) / R on |x_i - x_j| <= R,
//          W_i = sum_j w_ij, j over the design grid (the cone is cut at the grid's edge);
//   gh_i = (tanh(beta eta) + tanh(beta (gt_i - eta))) / (tanh(beta eta) + tanh(beta (1 - eta))).
// Reverse: gb_j = sum_i w_ij t_i with t_i = gbh_i (d gh / d gt)_i / W_i (w is symmetric).
//
// The sums over the ball are one tile kernel used both ways: a block owns a tile of
// design points and stages the tile plus a halo of r = floor(R) in LDS (zero off the
// grid), with the weights by offset (zero outside the ball). The kernels are compiled per
// r and per tap set: every tap is unrolled, and the set keeps the offsets with
// |d|^2 <= K2, K2 the smallest compiled bound >= floor(R^2) (so all taps of the ball,
// plus taps of weight zero when R^2 falls between bounds); rows of the cube that miss
// the ball are skipped at run time. Each thread computes XT consecutive points in x: a
// row's window of staged values is read once into registers and feeds XT independent
// accumulations. Sums run in a fixed order (taps by increasing dz, dy, dx).
//
// W_i is one box sum (8 entries in 3D) of the summed-area table of the weights, built
// per block in FP64, over the offsets that stay on the grid. The reverse first forms t_i
// once per point (elementwise, into the caller's scratch), then runs the tile kernel on t.
#pragma once
#include "lks_device.h"

namespace lks {

struct FltArgs {
    int n[3];
    int r;  // floor(R)
    double R, beta, eta;
};

// Points per block and per thread; A is the type staged in LDS.
// Staging loads a thread keeps in flight.
constexpr int FLT_CHUNK = 8;

// Tap sets compiled for radius r: set b keeps the offsets with |d|^2 <= r^2 + b r, b = 0,
// 1, 2 in 3D (b = 2 covers every R < r + 1); 2D compiles b = 2 only.
template <int RR, int B> constexpr int FLT_K2 = RR * RR + B * RR;

template <int DIM, typename A> struct FltShape {
    static constexpr int XT = DIM == 2 ? 2 : 4;
    static constexpr int TX = DIM == 2 ? 32 : (sizeof(A) == 4 ? 32 : 16);
    static constexpr int TY = 8, TZ = DIM == 2 ? 1 : 4;
    static constexpr int NT = (TX / XT) * TY * TZ;
    static constexpr int RMAX = DIM == 2 ? 8 : 4;  // largest floor(R)
};

// Sizes for the radius floor(R) = RR, known at compile time.
template <int DIM, typename A, int RR> struct FltCfg {
    using F = FltShape<DIM, A>;
    static constexpr int E = 2 * RR + 1, EZ = DIM == 2 ? 1 : E, RZ = DIM == 2 ? 0 : RR;
    static constexpr int HX = F::TX + 2 * RR, HY = F::TY + 2 * RR, HZ = DIM == 2 ? 1 : F::TZ + 2 * RR;
    static constexpr int NW = E * E * EZ;
    static constexpr int SA = E + 1, SB = E + 1, SC = EZ + 1;
};

// Weight of the offset (dx, dy, dz).
__device__ __forceinline__ double flt_w(double R, int dx, int dy, int dz) {
    const double d = sqrt((double)(dx * dx + dy * dy + dz * dz));
    return d <= R ? (R - d) / R : 0.0;
}

template <int DIM, typename A, int RR> __device__ __forceinline__ void flt_weights(const FltArgs &p, A *wl) {
    using C = FltCfg<DIM, A, RR>;
    for (int l = threadIdx.x; l < C::NW; l += blockDim.x)
        wl[l] = A(flt_w(p.R, l % C::E - RR, (l / C::E) % C::E - RR, l / (C::E * C::E) - C::RZ));
}

// Summed-area table of the weights (FP64; ends with a barrier): S(a, b, c) is the sum
// over the cube offsets with dx + RR < a, dy + RR < b, dz + RZ < c.
template <int DIM, int RR> __device__ void flt_sat(const FltArgs &p, double *S) {
    using C = FltCfg<DIM, double, RR>;
    for (int l = threadIdx.x; l < C::SA * C::SB * C::SC; l += blockDim.x) {
        const int ia = l % C::SA, ib = (l / C::SA) % C::SB, ic = l / (C::SA * C::SB);
        S[l] = (ia && ib && ic) ? flt_w(p.R, ia - 1 - RR, ib - 1 - RR, ic - 1 - C::RZ) : 0.0;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < C::SB * C::SC; l += blockDim.x) {
        double *q = S + C::SA * l;
        for (int i = 1; i < C::SA; i++) q[i] += q[i - 1];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < C::SA * C::SC; l += blockDim.x) {
        double *q = S + (l % C::SA) + C::SA * C::SB * (l / C::SA);
        for (int i = 1; i < C::SB; i++) q[C::SA * i] += q[C::SA * (i - 1)];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < C::SA * C::SB; l += blockDim.x) {
        double *q = S + l;
        for (int i = 1; i < C::SC; i++) q[C::SA * C::SB * i] += q[C::SA * C::SB * (i - 1)];
    }
    __syncthreads();
}

// W_i: the weights of the offsets that keep x + d on the grid (a box of the cube).
template <int DIM, int RR>
__device__ __forceinline__ double flt_wsum(const FltArgs &p, const double *S, int x, int y, int z) {
    using C = FltCfg<DIM, double, RR>;
    const int a0 = max(-RR, -x) + RR, a1 = min(RR, p.n[0] - 1 - x) + RR + 1;
    const int b0 = max(-RR, -y) + RR, b1 = min(RR, p.n[1] - 1 - y) + RR + 1;
    const int c0 = max(-C::RZ, -z) + C::RZ, c1 = min(C::RZ, p.n[2] - 1 - z) + C::RZ + 1;
    auto at = [&](int i, int j, int k) { return S[i + C::SA * (j + C::SB * k)]; };
    const double top = (at(a1, b1, c1) - at(a0, b1, c1)) - (at(a1, b0, c1) - at(a0, b0, c1));
    const double bot = (at(a1, b1, c0) - at(a0, b1, c0)) - (at(a1, b0, c0) - at(a0, b0, c0));
    return top - bot;
}

// The XT sums over the taps with |d|^2 <= K2 around the thread's points; `base` is the
// staged offset of its first point.
template <int DIM, typename A, int RR, int K2>
__device__ __forceinline__ void flt_gather(const A *tile, const A *wl, int base, double R2,
                                           A acc[FltShape<DIM, A>::XT]) {
    using C = FltCfg<DIM, A, RR>;
    constexpr int XT = FltShape<DIM, A>::XT, NWIN = 2 * RR + XT;
#pragma unroll
    for (int k = 0; k < XT; k++) acc[k] = A(0);
#pragma unroll
    for (int dz = -C::RZ; dz <= C::RZ; dz++) {
#pragma unroll
        for (int dy = -RR; dy <= RR; dy++) {
            if (dy * dy + dz * dz > K2) continue;
            if ((double)(dy * dy + dz * dz) > R2) continue;  // the whole row is off the ball
            const A *t = tile + base - RR + C::HX * (dy + C::HY * dz);
            const A *w = wl + RR + C::E * ((dy + RR) + C::E * (dz + C::RZ));
            A win[NWIN];
#pragma unroll
            for (int i = 0; i < NWIN; i++) win[i] = t[i];
#pragma unroll
            for (int dx = -RR; dx <= RR; dx++) {
                if (dx * dx + dy * dy + dz * dz > K2) continue;
                const A wd = w[dx];
#pragma unroll
                for (int k = 0; k < XT; k++) acc[k] += wd * win[dx + RR + k];
            }
        }
    }
}

template <int DIM, typename A> struct FltThread {
    using F = FltShape<DIM, A>;
    int o[3], lx, ty, tz;  // tile origin; the thread's first point within the tile
    __device__ FltThread() {
        o[0] = blockIdx.x * F::TX;
        o[1] = blockIdx.y * F::TY;
        o[2] = blockIdx.z * F::TZ;
        constexpr int NX = F::TX / F::XT;
        lx = (threadIdx.x % NX) * F::XT;
        ty = (threadIdx.x / NX) % F::TY;
        tz = threadIdx.x / (NX * F::TY);
    }
};

// Grid point of entry l of the staged tile; false off the grid.
template <int DIM, typename A, int RR>
__device__ __forceinline__ bool flt_halo_point(const FltArgs &p, const int o[3], int l, int &x, int &y, int &z) {
    using C = FltCfg<DIM, A, RR>;
    x = o[0] - RR + l % C::HX;
    y = o[1] - RR + (l / C::HX) % C::HY;
    z = o[2] - C::RZ + l / (C::HX * C::HY);
    return x >= 0 && x < p.n[0] && y >= 0 && y < p.n[1] && z >= 0 && z < p.n[2];
}

// Tile kernel. FWD: src = gamma (T = A), out0 = gamma_tilde, out1 = gamma_hat (the sum
// divided by W_i, then projected). Reverse: src = t (A = double), out0 = dJ/dgamma.
template <int DIM, typename A, int RR, int K2, bool FWD>
__global__ __launch_bounds__((FltShape<DIM, A>::NT)) void k_filter_tile(FltArgs p, const A *__restrict__ src,
                                                                       A *__restrict__ out0,
                                                                       A *__restrict__ out1) {
    using F = FltShape<DIM, A>;
    using C = FltCfg<DIM, A, RR>;
    __shared__ double S[FWD ? C::SA * C::SB * C::SC : 1];
    __shared__ A tile[C::HX * C::HY * C::HZ];
    __shared__ A wl[C::NW];
    const FltThread<DIM, A> th;
    // stage the tile: FLT_CHUNK loads in flight per thread, then their LDS stores
    constexpr int NH = C::HX * C::HY * C::HZ;
    for (int l0 = 0; l0 < NH; l0 += FLT_CHUNK * F::NT) {
        A v[FLT_CHUNK];
#pragma unroll
        for (int u = 0; u < FLT_CHUNK; u++) {
            const int l = l0 + u * F::NT + threadIdx.x;
            int x, y, z;
            v[u] = (l < NH && flt_halo_point<DIM, A, RR>(p, th.o, l, x, y, z))
                       ? src[x + (long long)p.n[0] * (y + (long long)p.n[1] * z)]
                       : A(0);
        }
#pragma unroll
        for (int u = 0; u < FLT_CHUNK; u++) {
            const int l = l0 + u * F::NT + threadIdx.x;
            if (l < NH) tile[l] = v[u];
        }
    }
    flt_weights<DIM, A, RR>(p, wl);
    if (FWD) flt_sat<DIM, RR>(p, S);  // ends with a barrier
    else __syncthreads();
    A acc[F::XT];
    const int base = (th.lx + RR) + C::HX * ((th.ty + RR) + C::HY * (th.tz + C::RZ));
    flt_gather<DIM, A, RR, K2>(tile, wl, base, p.R * p.R, acc);
    const int y = th.o[1] + th.ty, z = th.o[2] + th.tz;
    if (y >= p.n[1] || z >= p.n[2]) return;
    const A be = A(p.beta), et = A(p.eta);
    const A t0 = tanh(be * et), den = t0 + tanh(be * (A(1) - et));
#pragma unroll
    for (int k = 0; k < F::XT; k++) {
        const int x = th.o[0] + th.lx + k;
        if (x >= p.n[0]) break;
        const long long id = x + (long long)p.n[0] * (y + (long long)p.n[1] * z);
        if (FWD) {
            const A v = acc[k] / A(flt_wsum<DIM, RR>(p, S, x, y, z));
            out0[id] = v;
            out1[id] = (t0 + tanh(be * (v - et))) / den;
        } else {
            out0[id] = acc[k];
        }
    }
}

// Reverse, first step (FP64): t_i = gbh_i (d gh / d gt)_i / W_i at every design point.
constexpr int FLT_SCALE_NT = 256, FLT_SCALE_PT = 4;  // threads, points per thread
template <int DIM, typename T, int RR>
__global__ __launch_bounds__(FLT_SCALE_NT) void k_filter_scale(FltArgs p, long long nd, const T *__restrict__ gt,
                                                              const double *__restrict__ gbh,
                                                              double *__restrict__ t) {
    using C = FltCfg<DIM, double, RR>;
    __shared__ double S[C::SA * C::SB * C::SC];
    const long long i0 = (long long)blockIdx.x * (FLT_SCALE_NT * FLT_SCALE_PT) + threadIdx.x;
    double vg[FLT_SCALE_PT], vb[FLT_SCALE_PT];
#pragma unroll
    for (int u = 0; u < FLT_SCALE_PT; u++) {
        const long long i = i0 + (long long)u * FLT_SCALE_NT;
        vg[u] = i < nd ? (double)gt[i] : 0.0;
        vb[u] = i < nd ? gbh[i] : 0.0;
    }
    flt_sat<DIM, RR>(p, S);
    const double den = tanh(p.beta * p.eta) + tanh(p.beta * (1.0 - p.eta));
#pragma unroll
    for (int u = 0; u < FLT_SCALE_PT; u++) {
        const long long i = i0 + (long long)u * FLT_SCALE_NT;
        if (i >= nd) break;
        const int x = (int)(i % p.n[0]), y = (int)((i / p.n[0]) % p.n[1]), z = (int)(i / ((long long)p.n[0] * p.n[1]));
        const double s = tanh(p.beta * (vg[u] - p.eta));
        t[i] = vb[u] * (p.beta * (1.0 - s * s) / den) / flt_wsum<DIM, RR>(p, S, x, y, z);
    }
}

}  // namespace lks
