// lks.hip -- host runtime and C ABI of the gfx950 library (declared in include/lks.h).
//
// The time loop lives on the host but every value it needs stays on the device: the
// body state and its iterates, the force/torque, the footprint box origin and the
// error flag never cross PCIe during a run. One call = one stream, kernels enqueued
// back to back; lks_forward / lks_adjoint synchronise once at the end to read the
// error flag (skipped with LKS_FLAG_ASYNC).
//
// Adjoint memory: checkpoints every ckpt_every steps (state + body record); the reverse
// sweep recomputes one segment into the workspace (states, the u* footprint of every
// step and every fluid <-> body iterate), then walks it backwards.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "../../include/lks.h"
#include "body.h"
#include "cyclic.h"
#include "f2.h"
#include "filter.h"
#include "mma.h"

using namespace lks;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LKS_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                      \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
inline unsigned blocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ live kernel timing
// Kernel begin/end timestamps on sampled steps (LKS_FLAG_PROFILE); durations are read
// after the call's final synchronisation and added to process-wide totals.
std::vector<hipEvent_t> g_events;
double g_prof_ms[LKS_K_COUNT];
long long g_prof_n[LKS_K_COUNT];

constexpr int NSPAN = 256;  // stamped launches per call (at most)
__global__ void k_span_init(unsigned long long *s, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        s[2 * i] = ~0ull;
        s[2 * i + 1] = 0ull;
    }
}

// v = u - U on entry (sign -1) and u = v + U on exit (sign +1), velocity components of
// a state in place.
template <typename T>
__global__ __launch_bounds__(256) void k_shift(T *__restrict__ s, long long N, int dim, double U0, double U1,
                                               double U2, double sign) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double U[3] = {U0, U1, U2};
    for (int a = 0; a < dim; a++)
        if (U[a] != 0.0) s[(1 + a) * N + i] = T((double)s[(1 + a) * N + i] + sign * U[a]);
}

// Clears n 32-bit words (a fill kernel rather than hipMemsetAsync, so that a caller
// may capture the enqueued work in a graph).
__global__ void k_zero32(unsigned *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

struct Prof {
    bool on = false;
    bool sample = false;
    hipStream_t st = nullptr;
    std::vector<int> ids;

    // `launch(start, stop)` passes the events to hipExtLaunchKernelGGL, which stamps them
    // with the kernel's own begin and end times (no marker packets in between), so the
    // sampled durations are the kernels' execution times; null events record nothing.
    template <typename F> void run(int id, F &&launch) {
        if (!on || !sample) {
            launch(nullptr, nullptr);
            return;
        }
        const size_t i = ids.size();
        while (g_events.size() < 2 * (i + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                launch(nullptr, nullptr);
                return;
            }
            g_events.push_back(e);
        }
        launch(g_events[2 * i], g_events[2 * i + 1]);
        ids.push_back(id);
    }
    // Stencil kernels stamp their own span (first block start, last block end) into a
    // slot pair of a small workspace area instead; `launch(ts)` passes the slot (null:
    // not sampled).
    unsigned long long *span = nullptr;
    int nspan = 0;
    std::vector<int> span_ids;
    // Stencil kernels: sampled launches alternate between launch-attached events
    // (dispatch to completion, as a profiler counts a launch; recorded under `id`) and
    // the kernel's own span (under `span_id`), so that neither perturbs the other.
    bool next_span = false;
    template <typename F> void run_span(int id, int span_id, F &&launch) {
        if (!on || !sample) {
            launch(nullptr, nullptr, nullptr);
            return;
        }
        next_span = !next_span;
        if (span_id < 0 || !next_span || !span || (int)span_ids.size() >= nspan) {
            run(id, [&](hipEvent_t e0, hipEvent_t e1) { launch(e0, e1, nullptr); });
            return;
        }
        unsigned long long *ts = span + 2 * span_ids.size();
        span_ids.push_back(span_id);
        launch(nullptr, nullptr, ts);
    }
    void finish() {
        for (size_t i = 0; i < ids.size(); i++) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, g_events[2 * i], g_events[2 * i + 1]) == hipSuccess) {
                g_prof_ms[ids[i]] += ms;
                g_prof_n[ids[i]] += 1;
            }
        }
        ids.clear();
        if (!span_ids.empty()) {
            std::vector<unsigned long long> h(2 * span_ids.size());
            int dev = 0, khz = 0;
            if (hipMemcpy(h.data(), span, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) ==
                    hipSuccess &&
                hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0) {
                for (size_t i = 0; i < span_ids.size(); i++)
                    if (h[2 * i + 1] > h[2 * i]) {
                        g_prof_ms[span_ids[i]] += (double)(h[2 * i + 1] - h[2 * i]) / khz;
                        g_prof_n[span_ids[i]] += 1;
                    }
            }
            span_ids.clear();
        }
    }
    // preset the slots (all-ones start, zero end) on stream s
    void arm(unsigned long long *slots, int n, hipStream_t s) {
        span = slots;
        nspan = n;
        if (on) hipLaunchKernelGGL(k_span_init, dim3(1), dim3(256), 0, s, slots, n);
    }
};

struct Ctx {
    int dim = 0, prec = 0;
    size_t elt = 4;
    Grid g{};
    Bc bc{};
    Design D{};
    BodyParams bp{};
    double A = 0;
    int K = 1, NT = 0, Kc = 1;
    bool has_body = false;
    bool rot = true;  // the pose may rotate (wider gather window)
    int face_axes = 0;
    long long face_total = 0;
    long long S = 0;  // elements of a state
    unsigned nblk = 1;
    int dblk = 128;      // threads per block of the design-point kernels
    int tt2 = 0;         // 2D fused iteration: design tile edge (0: separate kernels)
    unsigned ntile = 0;  // its number of tiles
    bool tile3 = false;  // 3D R1 over 8^3 design tiles (nblk = tiles)
    bool paper = false;  // lks_adjoint computes the paper's adjoint variant (f2.h)
    // 2D LKS / adjoint LKS kernels: the column march (large grids) or the tiles
    bool march_fwd = false, march_adj = false;
    bool plane3d = false;  // 3D: LKS kernels address the fields one plane at a time
};

// Grids from which the 2D column-march kernels are faster than the tile kernels
// (measured: the tile forward is faster up to 2M nodes, the march from 8M; the march
// adjoint from 2M, the tile adjoint up to 0.5M).
constexpr long long MARCH_FWD_NODES = 1LL << 22, MARCH_ADJ_NODES = 1LL << 20;

constexpr int MARGIN = 2;
constexpr unsigned CPL_BLOCKS = 1024;  // blocks of the coupling-constant kernel (at most)

// Footprint box: half-extents H from the largest distance of a design point from the
// rotation centre (any angle if `rot_any`, else at angle theta0), plus the mapping
// support (2) and the drift margin.
void box_params(Ctx &c, const lks_problem_t *P, bool rot_any, double theta0) {
    Design &D = c.D;
    double rho[3] = {0, 0, 0};
    const double hp = D.half[D.pi], hq = D.half[D.pj];
    if (rot_any) {
        const double r = std::sqrt(hp * hp + hq * hq);
        rho[D.pi] = r;
        rho[D.pj] = r;
    } else {
        const double cs = std::fabs(std::cos(theta0)), sn = std::fabs(std::sin(theta0));
        rho[D.pi] = cs * hp + sn * hq;
        rho[D.pj] = sn * hp + cs * hq;
    }
    rho[D.axis] = D.half[D.axis];
    D.boxN = 1;
    for (int a = 0; a < 3; a++) {
        if (a < c.dim) {
            D.H[a] = (int)std::ceil(rho[a] - 1e-12) + 2 + MARGIN;
            D.L[a] = 2 * D.H[a] + 2;
        } else {
            D.H[a] = 0;
            D.L[a] = 1;
        }
        D.boxN *= D.L[a];
    }
    D.margin = MARGIN;
    const double sn = std::fabs(std::sin(theta0)), cs = std::fabs(std::cos(theta0));
    c.rot = rot_any || std::min(sn, cs) > 1e-12;
    (void)P;
}

int make_ctx(const lks_problem_t *P, Ctx &c) {
    if (!P) return fail(LKS_EINVAL, "null problem");
    if (P->dim != 2 && P->dim != 3) return fail(LKS_EINVAL, "dim must be 2 or 3 (got %d)", P->dim);
    if (P->precision != LKS_FP32 && P->precision != LKS_FP64)
        return fail(LKS_EINVAL, "precision must be LKS_FP32 or LKS_FP64");
    c.dim = P->dim;
    c.prec = P->precision;
    c.elt = c.prec == LKS_FP32 ? 4 : 8;
    if (c.dim == 2 && P->n[2] != 1) return fail(LKS_EINVAL, "2D problems need n[2] == 1");
    c.g.N = 1;
    for (int a = 0; a < 3; a++) {
        if (P->n[a] < 1) return fail(LKS_EINVAL, "n[%d] < 1", a);
        c.g.n[a] = P->n[a];
        c.g.N *= P->n[a];
    }
    if (c.g.N > (1LL << 31)) return fail(LKS_EINVAL, "grid too large");
    for (int a = 0; a < 3; a++) {
        if (a >= c.dim) {
            c.g.per[a] = 1;
            continue;
        }
        const int lo = P->bc[2 * a], hi = P->bc[2 * a + 1];
        for (int f : {lo, hi})
            if (f < LKS_PERIODIC || f > LKS_WALL) return fail(LKS_EINVAL, "bad boundary kind %d", f);
        if ((lo == LKS_PERIODIC) != (hi == LKS_PERIODIC))
            return fail(LKS_EINVAL, "axis %d: PERIODIC must be set on both faces", a);
        c.g.per[a] = lo == LKS_PERIODIC;
        if (c.g.n[a] < 3) return fail(LKS_EINVAL, "n[%d] must be >= 3", a);
        if (!c.g.per[a]) {
            c.face_axes |= 1 << a;
            c.face_total += 2 * (c.g.N / c.g.n[a]);
        }
    }
    for (int f = 0; f < 6; f++) {
        c.bc.kind[f] = f < 2 * c.dim ? P->bc[f] : LKS_PERIODIC;
        c.bc.p[f] = P->bc_p[f];
        for (int a = 0; a < 3; a++) c.bc.u[f][a] = P->bc_u[f][a];
    }
    // reference velocity of the stored deviation v = u - U: the first VELOCITY face's,
    // rounded to FP32, so that U and -U (the deviation of a wall or of a fluid at rest)
    // are exact in FP32 fields; the inflow's own deviation is then a tiny number that
    // FP32 holds to its full relative precision
    for (int a = 0; a < 3; a++) c.g.U[a] = 0.0;
    for (int f = 0; f < 2 * c.dim; f++)
        if (c.bc.kind[f] == LKS_VELOCITY) {
            for (int a = 0; a < c.dim; a++) {
                if (!std::isfinite(c.bc.u[f][a])) return fail(LKS_EINVAL, "bc_u not finite");
                c.g.U[a] = (double)(float)c.bc.u[f][a];
            }
            break;
        }
    for (int a = 0; a < 3; a++) c.g.Uf[a] = (float)c.g.U[a];
    if (!std::isfinite(P->nu)) return fail(LKS_EINVAL, "nu not finite");
    c.A = 4.5 * (1.0 / 6.0 - P->nu);
    c.S = (long long)(c.dim + 1) * c.g.N;
    // design
    Design &D = c.D;
    D.ND = 1;
    int zero = 0;
    for (int a = 0; a < 3; a++) {
        if (P->nd[a] < 0) return fail(LKS_EINVAL, "nd[%d] < 0", a);
        zero += P->nd[a] == 0;
        D.nd[a] = P->nd[a];
        D.ND *= P->nd[a];
    }
    c.has_body = D.ND > 0;
    if (!c.has_body && zero != 3 && !(c.dim == 2 && P->nd[0] == 0 && P->nd[1] == 0))
        return fail(LKS_EINVAL, "nd must be all positive or all zero");
    if (c.has_body) {
        if (c.dim == 2 && P->nd[2] != 1) return fail(LKS_EINVAL, "2D designs need nd[2] == 1");
        if (P->n_itr < 1) return fail(LKS_EINVAL, "n_itr must be >= 1");
        if (!(P->mass > 0) || !(P->inertia > 0)) return fail(LKS_EINVAL, "mass and inertia must be > 0");
        if (!std::isfinite(P->kappa_max) || !std::isfinite(P->q))
            return fail(LKS_EINVAL, "kappa_max, q must be finite");
    }
    D.axis = c.dim == 2 ? 2 : P->axis;
    if (D.axis < 0 || D.axis > 2) return fail(LKS_EINVAL, "axis must be 0, 1 or 2");
    D.pi = (D.axis + 1) % 3;
    D.pj = (D.axis + 2) % 3;
    for (int a = 0; a < 3; a++) D.half[a] = D.nd[a] > 0 ? 0.5 * (D.nd[a] - 1) : 0.0;
    if (c.dim == 2) D.half[2] = 0.0;
    box_params(c, P, true, 0.0);
    c.bp.kmax = P->kappa_max;
    c.bp.q = P->q;
    c.bp.mass = P->mass;
    c.bp.inertia = P->inertia;
    c.bp.dof = P->dof_mask & (c.dim == 2 ? (LKS_DOF_TX | LKS_DOF_TY | LKS_DOF_ROT) : 15);
    c.K = c.has_body ? P->n_itr : 1;
    c.paper = (P->flags & LKS_FLAG_PAPER_ADJOINT) != 0;
    {
        const bool force = (P->flags & LKS_FLAG_MARCH2D) != 0;
        c.march_fwd = c.dim == 2 && (force || c.g.N >= MARCH_FWD_NODES);
        c.march_adj = c.dim == 2 && (force || c.g.N >= MARCH_ADJ_NODES);
        c.plane3d = c.dim == 3 && ((P->flags & LKS_FLAG_PLANE3D) != 0 ||
                                   4ULL * (unsigned long long)c.g.N * (P->precision == LKS_FP64 ? 8 : 4) >=
                                       (unsigned long long)BOFF_NONE);
    }
    if (P->n_steps < 0) return fail(LKS_EINVAL, "n_steps < 0");
    c.NT = P->n_steps;
    c.Kc = P->ckpt_every;
    if (P->objective < 0 || P->objective > 3) return fail(LKS_EINVAL, "bad objective");
    if (P->objective < 3 && P->objective >= c.dim) return fail(LKS_EINVAL, "objective axis >= dim");
    if (c.has_body && D.boxN > 0x7fffffffLL) return fail(LKS_EINVAL, "design footprint box too large");
    if (c.has_body && D.ND > 0x7fffffffLL) return fail(LKS_EINVAL, "design grid too large");
    if (c.dim == 3 && layer_count(c.g.n, c.g.per) > 0x7fffffffLL) return fail(LKS_EINVAL, "grid faces too large");
    // the 3D LKS kernels address one plane of a field with 32-bit byte offsets
    if (c.dim == 3 && (long long)c.g.n[0] * c.g.n[1] * 8 >= (1LL << 31)) return fail(LKS_EINVAL, "grid plane too large");
    if (c.has_body && c.dim == 3 && (long long)(D.nd[D.axis] + 4) * D.nd[D.pi] * D.nd[D.pj] > 0x7fffffffLL)
        return fail(LKS_EINVAL, "design grid too large");
    c.dblk = c.dim == 3 ? Dblk<3>::v : Dblk<2>::v;
    c.nblk = c.has_body ? blocks(D.ND, c.dblk) : 1;
    // 3D FP32: the interpolation reverse (R1) runs over 8^3 design tiles with the stencil
    // patch staged in LDS; the other design-point kernels keep the linear point order on
    // as many blocks (nblk * 512 >= ND), so that R1's and R3's partials pair up
    c.tile3 = c.has_body && c.dim == 3 && c.prec == LKS_FP32;
    if (c.tile3) c.nblk = blocks(D.nd[0], Tile3::E) * blocks(D.nd[1], Tile3::E) * blocks(D.nd[2], Tile3::E);
    // fused 2D iterations while every block can afford to read all partials (<= 256)
    if (c.has_body && c.dim == 2) {
        for (int tt : {8, 16}) {
            const unsigned nt = blocks(D.nd[0], tt) * blocks(D.nd[1], tt);
            if (nt <= 256) {
                c.tt2 = tt;
                c.ntile = nt;
                break;
            }
        }
    }
    return LKS_OK;
}

// ------------------------------------------------------------------ layout
struct Layout {
    size_t krT, krD, st1, ustar, Bf, Binit, part, counter, flag, span, cpl;
    // adjoint: two segment buffers (recompute of one segment overlaps the reverse sweep
    // of the other), each of seg_n / ustar_seg_n / Bseg_n bytes
    size_t seg, ustar_seg, Bseg, seg_n, ustar_seg_n, Bseg_n;
    size_t ab, kapk, usk, uk, ustb, kb, usb, URb, krb, part1, part3, rec;
    size_t K1f, K1r;  // 3D axial sums of kappa_ref: forward (one pose), reverse (n_itr poses)
    size_t AU;        // 3D axial sums of the u^ref cotangents (one pose, 3 components)
    // 2D adjoint: kappa^(k), u^S^(k), u^(k) on the box for every step of a segment (two
    // buffers like the segments), pre_n bytes each; 0 in 3D
    size_t pre, pre_n;
    // the paper's adjoint variant: box fields, h/q, u~* of two levels, partials, record
    size_t f2F, f2hq, f2ups, f2pn, f2pd, f2rec;
    size_t total;
};

// Rows of the footprint box along the rotation axis (3D row kernels: one wave each).
long long box_rows(const Ctx &c) { return (long long)c.D.L[c.D.pi] * c.D.L[c.D.pj]; }

// Elements of one pose's axial sums (3D bodies; see k_axial).
size_t axial_elems(const Ctx &c) {
    if (!c.has_body || c.dim != 3) return 1;
    return (size_t)(c.D.nd[c.D.axis] + 4) * c.D.nd[c.D.pi] * c.D.nd[c.D.pj];
}

// Elements of one step's footprint fields for the reverse sweep: kappa^(k), u^S^(k),
// u^(k) for the n_itr iterations, in that order.
size_t pre_elems(const Ctx &c) { return (size_t)c.K * (size_t)(1 + 2 * c.dim) * (size_t)c.D.boxN; }

Layout layout(const Ctx &c, bool adjoint) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(bytes);
        return r;
    };
    const size_t ND = (size_t)(c.has_body ? c.D.ND : 1);
    const size_t bN = (size_t)(c.has_body ? c.D.boxN : 1);
    const size_t e = c.elt, d = (size_t)c.dim, K = (size_t)c.K;
    const size_t stateB = (size_t)c.S * e;
    const size_t rec = (K + 1) * B_REC * sizeof(double);
    L.krT = take(ND * e);
    L.krD = take(ND * 8);
    L.st1 = take(stateB);
    L.ustar = take(d * bN * e);
    L.Bf = take(2 * rec);
    L.Binit = take(B_REC * 8);
    L.part = take(std::max((size_t)c.nblk * 8, (size_t)c.ntile * 8) * 8);
    L.counter = take(16);
    L.flag = take(16);
    L.span = take(2 * NSPAN * sizeof(unsigned long long));
    L.cpl = take((CPL_BLOCKS * 4 + 4) * sizeof(double));
    const size_t axN = axial_elems(c);
    L.K1f = take(axN * e);
    if (adjoint) {
        L.K1r = take(K * axN * e);
        L.AU = take(3 * axN * e);
        const size_t Kc = (size_t)(c.Kc > 0 ? c.Kc : 1);
        L.seg_n = up((Kc + 1) * stateB);
        L.ustar_seg_n = up(Kc * d * bN * e);
        L.Bseg_n = up((Kc + 2) * rec);
        L.seg = take(2 * L.seg_n);
        L.ustar_seg = take(2 * L.ustar_seg_n);
        L.Bseg = take(2 * L.Bseg_n);
        L.pre_n = (c.dim == 2 && c.has_body) ? up(Kc * pre_elems(c) * e) : 0;
        L.pre = take(2 * L.pre_n);
        L.ab = take(2 * stateB);
        L.kapk = take(K * bN * e);
        L.usk = take(K * d * bN * e);
        L.uk = take(K * d * bN * e);
        L.ustb = take(d * bN * e);
        L.kb = take(bN * e);
        L.usb = take(d * bN * e);
        L.URb = take(d * ND * e);
        L.krb = take(ND * 8);
        L.part1 = take((size_t)c.nblk * 8 * 8);
        L.part3 = take((size_t)c.nblk * 8 * 8);
        L.rec = take(2 * AR_SIZE * 8);
        if (c.paper && c.has_body) {
            L.f2F = take((size_t)F2F_N * bN * e);
            L.f2hq = take(4 * bN * e);
            L.f2ups = take(2 * d * (size_t)c.g.N * e);
            L.f2pn = take((size_t)blocks((long long)bN, F2_NT) * F2_NNODE * 8);
            L.f2pd = take((size_t)blocks((long long)ND, F2_NT) * F2_NDES * 8);
            L.f2rec = take(F2_REC * 8);
        }
    }
    L.total = o;
    return L;
}

// checkpoint store: header, states, body records
struct CkptHeader {
    char magic[8];
    int dim, prec, K, Kc, NT, ncp;
    long long N, ND;
    int H[3], L[3];
    long long boxN;
    int rot;
    double U[3];  // reference velocity of the stored states (v = u - U)
};

size_t ckpt_count(const Ctx &c) { return c.Kc > 0 ? (size_t)((c.NT + c.Kc - 1) / c.Kc) : 0; }
size_t ckpt_state_off(const Ctx &c, size_t i) { return up(sizeof(CkptHeader)) + i * up((size_t)c.S * c.elt); }
size_t ckpt_body_off(const Ctx &c, size_t i) {
    return ckpt_state_off(c, ckpt_count(c)) + i * B_REC * sizeof(double);
}
size_t ckpt_bytes(const Ctx &c) { return ckpt_body_off(c, ckpt_count(c)); }

template <typename T> T *at(void *base, size_t off) { return (T *)((char *)base + off); }

// ------------------------------------------------------------------ kernels by type
// Lanes per footprint node in the gather-form mapping kernels: 2D footprints are small
// (latency-bound), so the candidate loop of a node is split over 4 lanes.
template <int DIM> constexpr int lpn() { return DIM == 2 ? 4 : 1; }

// Calls f(dim, rot) with compile-time constants matching the problem.
template <typename F> void dispatch(const Ctx &c, F &&f) {
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    if (c.dim == 2) {
        if (c.rot) f(I2{}, std::true_type{});
        else f(I2{}, std::false_type{});
    } else {
        if (c.rot) f(I3{}, std::true_type{});
        else f(I3{}, std::false_type{});
    }
}

// Blocks of `kernel` that the device holds at once (occupancy x compute units); 512 if
// the runtime cannot say.
template <typename K> long long resident_blocks(K kernel, int threads) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
        cus < 1)
        return 512;
    return (long long)per_cu * cus;
}

template <typename T> struct Run {
    const Ctx &c;
    hipStream_t st;
    Prof *pf;
    T *ax = nullptr;  // 3D: axial sums of kappa_ref (k_axial), one pose per iteration run

    // Adjoint record (body_rev): two copies, since an R1 that steps the record reads one
    // and writes the other (rcur: the current one); pend: the iteration whose partials
    // (part3) still wait for their record step, or -1.
    mutable int rcur = 0, pend = -1;
    // The next R1 steps the record itself (every block reads all partials) on small
    // grids (in 2D a dedicated wave per block, overlapped with the interpolation);
    // larger ones use k_r3_finish after each R3.
    bool defer_finish() const { return c.nblk <= (c.dim == 2 ? 1024 : 256); }

    // The cross-block finish of the design-point reductions runs in the last block to
    // arrive while the grid is small; beyond that the arrival counter serialises the
    // blocks and a one-block finish kernel is cheaper.
    bool last_block_ok() const { return c.nblk <= 256; }

    // z planes per block of the 2.5D 3D kernels. A block costs about (planes + 2) plane
    // steps (two planes of lead-in), and `resident` blocks run at once (occupancy x
    // CUs); pick the chunk (4..32 planes) that minimises rounds x (planes + 2).
    // the 3D LKS kernels address a whole field (4 components) with 32-bit byte offsets
    // below BOFF_NONE, else one plane at a time
    bool whole_fields() const { return !c.plane3d; }
    int zchunk(int ox, int oy, long long resident) const {
        const long long bxy = (long long)blocks(c.g.n[0], ox) * blocks(c.g.n[1], oy);
        int best = 32;
        long long best_cost = -1;
        for (int zc = 32; zc >= 4; zc--) {
            const long long nb = bxy * blocks(c.g.n[2], zc);
            const long long cost = (nb + resident - 1) / resident * (zc + 2);
            if (best_cost < 0 || cost < best_cost) best = zc, best_cost = cost;
        }
        return best;
    }

    // Launch shape of the 2D column-march kernels: strips of `width` columns (the first
    // shifted left by `off`), each cut into runs of `rows` rows, one wave per run. The
    // runs are as long as possible while every wave of the grid is resident at once
    // (`resident` waves), and at least 2 rows long.
    void col_march(int width, int off, long long resident, int &rows, int &nstrip, int &nwave) const {
        nstrip = (int)blocks(c.g.n[0] + off, width);
        const long long runs = std::max(1LL, resident / nstrip);
        rows = (int)std::max(2LL, (c.g.n[1] + runs - 1) / runs);
        nwave = nstrip * (int)blocks(c.g.n[1], rows);
    }
    // fold (2D): the boundary values of `in` are formed on load (see k_gather2d)
    void gather(const T *in, T *out, bool fold = false) const {
        if (c.dim == 2 && c.march_fwd) {
            static const long long res = resident_blocks(k_gather2d_march<T, false>, C2_NT);
            int rows, nstrip, nwave;
            col_march(C2_W, 0, res * (C2_NT / 64), rows, nstrip, nwave);
            const dim3 grid(blocks(nwave, C2_NT / 64));
            const int fd = fold ? 1 : 0;
            pf->run_span(LKS_K_GATHER, LKS_K_GATHER_SPAN, [&](hipEvent_t e0, hipEvent_t e1, unsigned long long *ts) {
                if (ts)
                    hipLaunchKernelGGL((k_gather2d_march<T, true>), grid, dim3(C2_NT), 0, st, c.g, T(c.A), c.bc, fd,
                                       rows, nstrip, nwave, in, out, ts);
                else
                    hipExtLaunchKernelGGL((k_gather2d_march<T, false>), grid, dim3(C2_NT), 0, st, e0, e1, 0, c.g,
                                          T(c.A), c.bc, fd, rows, nstrip, nwave, in, out, ts);
            });
        } else if (c.dim == 2) {
            dim3 grid(blocks(c.g.n[0], G2_TX), blocks(c.g.n[1], G2_TY));
            const int fd = fold ? 1 : 0;
            pf->run_span(LKS_K_GATHER, LKS_K_GATHER_SPAN, [&](hipEvent_t e0, hipEvent_t e1, unsigned long long *ts) {
                if (ts)
                    hipLaunchKernelGGL((k_gather2d<T, true>), grid, dim3(G2_TX, G2_TY), 0, st, c.g, T(c.A), c.bc, fd,
                                       in, out, ts);
                else
                    hipExtLaunchKernelGGL((k_gather2d<T, false>), grid, dim3(G2_TX, G2_TY), 0, st, e0, e1, 0, c.g,
                                          T(c.A), c.bc, fd, in, out, ts);
            });
        } else {
            static const long long res = resident_blocks(k_gather3d<T, false, true>, G3<T>::NT);
            const int zc = zchunk(G3<T>::OX, G3<T>::OY, res);
            const dim3 grid(blocks(c.g.n[0], G3<T>::OX), blocks(c.g.n[1], G3<T>::OY), blocks(c.g.n[2], zc));
            // 3D: launch events only (long launches)
            pf->run_span(LKS_K_GATHER, -1, [&](hipEvent_t e0, hipEvent_t e1, unsigned long long *) {
                if (whole_fields())
                    hipExtLaunchKernelGGL((k_gather3d<T, false, true>), grid, dim3(G3<T>::TX, G3<T>::TY), 0, st, e0,
                                          e1, 0, c.g, T(c.A), FeqU<T>::make(c.g.U), zc, in, out, nullptr);
                else
                    hipExtLaunchKernelGGL((k_gather3d<T, false, false>), grid, dim3(G3<T>::TX, G3<T>::TY), 0, st, e0,
                                          e1, 0, c.g, T(c.A), FeqU<T>::make(c.g.U), zc, in, out, nullptr);
            });
        }
    }
    void bcs(T *s) const {
        if (!c.face_total) return;
        pf->run(LKS_K_BC, [&](hipEvent_t e0, hipEvent_t e1) {
            if (c.dim == 2)
                hipExtLaunchKernelGGL((k_bc<2, T>), dim3(blocks(c.face_total, 256)), dim3(256), 0, st, e0, e1, 0, c.g, c.bc, s,
                                   c.face_axes, c.face_total);
            else
                hipExtLaunchKernelGGL((k_bc<3, T>), dim3(blocks(c.face_total, 256)), dim3(256), 0, st, e0, e1, 0, c.g, c.bc, s,
                                   c.face_axes, c.face_total);
        });
    }
    // the n_itr fluid <-> body iterations of one step
    void body_loop(T *state, double *Bk, double *Bnext0, const T *krT, const double *krD, T *ustar,
                   double *part, unsigned *counter, int *flag) const {
        T *u = state + c.g.N;
        if (c.tt2) {
            body_loop_fused(u, Bk, Bnext0, krT, krD, ustar, part, flag);
            return;
        }
        dispatch(c, [&](auto dm, auto rt) {
            constexpr int DIM = decltype(dm)::value;
            constexpr bool ROT = decltype(rt)::value;
            for (int k = 0; k < c.K; k++) {
                pf->run(LKS_K_SPREAD, [&](hipEvent_t e0, hipEvent_t e1) {
                    hipEvent_t es = e0;
                    if (DIM == 3) {  // axial sums of kappa_ref at B^(k)
                        hipExtLaunchKernelGGL((k_axial<1, T>), dim3(blocks((long long)axial_elems(c), 256), 1), dim3(256),
                                              0, st, e0, nullptr, 0, c.D, Bk, k, krT, (long long)c.D.ND, ax);
                        es = nullptr;
                    }
                    if constexpr (DIM == 3 && ROT)  // one wave per box row (k_spread_fwd_rows)
                        hipExtLaunchKernelGGL((k_spread_fwd_rows<T, ROT>), dim3(blocks(box_rows(c), 4)), dim3(256), 0, st,
                                              es, e1, 0, c.g, c.D, Bk, k, (const T *)ax, u, ustar);
                    else
                        hipExtLaunchKernelGGL((k_spread_fwd<DIM, T, ROT, lpn<DIM>()>),
                                              dim3(blocks(c.D.boxN * lpn<DIM>(), 256)), dim3(256), 0, st, es, e1, 0,
                                              c.g, c.D, Bk, k, krT, (const T *)ax, u, ustar);
                });
                pf->run(LKS_K_INTERP, [&](hipEvent_t e0, hipEvent_t e1) {
                    hipExtLaunchKernelGGL((k_interp_force<DIM, T>), dim3(c.nblk), dim3(c.dblk), 0, st, e0,
                                          last_block_ok() ? e1 : nullptr, 0, c.g, c.D, c.bp, u,
                                       krD, Bk, k, c.K, Bnext0, part, counter, flag, last_block_ok() ? 1 : 0);
                    if (!last_block_ok())
                        hipExtLaunchKernelGGL((k_interp_finish<DIM>), dim3(1), dim3(1024), 0, st, nullptr, e1, 0, c.D, c.bp, Bk, k, c.K,
                                           Bnext0, part, c.nblk, flag);
                });
            }
        });
    }
    // 2D: one fused kernel per iteration, then B^(K) and the step's spread
    void body_loop_fused(T *u, double *Bk, double *Bnext0, const T *krT, const double *krD, T *ustar,
                         double *part, int *flag) const {
        const size_t half = (size_t)c.ntile * 4;
        auto run = [&](auto rt, auto tt) {
            constexpr bool ROT = decltype(rt)::value;
            constexpr int TT = decltype(tt)::value;
            for (int k = 0; k < c.K; k++) {
                const double *pin = part + (size_t)((k + 1) & 1) * half;
                double *pout = part + (size_t)(k & 1) * half;
                pf->run(LKS_K_ITER, [&](hipEvent_t e0, hipEvent_t e1) {
                    hipExtLaunchKernelGGL((k_iter2d<T, ROT, TT>), dim3(c.ntile), dim3(It2<TT>::NT), 0, st, e0, e1, 0,
                                          c.g, c.D, c.bp, Bk, k, krT, krD, (const T *)u, pin, c.ntile, pout, flag);
                });
            }
            const double *plast = part + (size_t)((c.K - 1) & 1) * half;
            pf->run(LKS_K_ITER_FINAL, [&](hipEvent_t e0, hipEvent_t e1) {
                hipExtLaunchKernelGGL((k_iter_final2d<T, ROT, 4>), dim3(blocks(c.D.boxN * 4, 256) + 1), dim3(256), 0, st,
                                      e0, e1, 0, c.g, c.D, c.bp, Bk, c.K, krT, u, ustar, plast, c.ntile, Bnext0,
                                      flag);
            });
        };
        const bool r = c.rot;
        if (c.tt2 == 8) {
            if (r) run(std::true_type{}, std::integral_constant<int, 8>{});
            else run(std::false_type{}, std::integral_constant<int, 8>{});
        } else {
            if (r) run(std::true_type{}, std::integral_constant<int, 16>{});
            else run(std::false_type{}, std::integral_constant<int, 16>{});
        }
    }
    // reverse of the body loop of one step (records Bk, footprint u* of the step)
    // footprint fields of every iteration of one step (kappa^(k), u^S^(k), u^(k)) from the
    // stored iterates and u*, for the reverse sweep
    void adj_fields(const double *Bk, const T *ustar, const T *krT, T *kapk, T *usk, T *uk) const {
        const dim3 gb(blocks(c.D.boxN * (c.dim == 2 ? 4 : 1), 256), c.K);
        dispatch(c, [&](auto dm, auto rt) {
            constexpr int DIM = decltype(dm)::value;
            constexpr bool ROT = decltype(rt)::value;
            pf->run(LKS_K_ADJ_RECOMPUTE, [&](hipEvent_t e0, hipEvent_t e1) {
                hipEvent_t es = e0;
                if (DIM == 3) {  // axial sums of kappa_ref at B^(0) .. B^(K-1)
                    hipExtLaunchKernelGGL((k_axial<1, T>), dim3(blocks((long long)axial_elems(c), 256), c.K), dim3(256), 0,
                                          st, e0, nullptr, 0, c.D, Bk, 0, krT, (long long)c.D.ND, ax);
                    es = nullptr;
                }
                if constexpr (DIM == 3 && ROT)  // one wave per box row and pose (k_adj_recompute_rows)
                    hipExtLaunchKernelGGL((k_adj_recompute_rows<T, ROT>), dim3(blocks(box_rows(c), 4), c.K), dim3(256), 0,
                                          st, es, e1, 0, c.g, c.D, Bk, (const T *)ax, ustar, kapk, usk, uk);
                else
                    hipExtLaunchKernelGGL((k_adj_recompute<DIM, T, ROT, lpn<DIM>()>), gb, dim3(256), 0, st, es, e1, 0,
                                          c.g, c.D, Bk, krT, (const T *)ax, ustar, kapk, usk, uk);
            });
        });
    }
    // reverse of the body loop of one step (records Bk, footprint u* of the step); pre
    // (2D): the step's footprint fields, formed beside the segment's forward recompute
    void body_rev(const double *Bk, const T *ustar, const T *ab, const T *krT, const double *krD, const Layout &L,
                  void *w, const T *pre) const {
        T *kapk = at<T>(w, L.kapk), *usk = at<T>(w, L.usk), *uk = at<T>(w, L.uk);
        T *ustb = at<T>(w, L.ustb), *kb = at<T>(w, L.kb), *usb = at<T>(w, L.usb), *URb = at<T>(w, L.URb);
        double *krb = at<double>(w, L.krb), *p1 = at<double>(w, L.part1), *p3 = at<double>(w, L.part3);
        int *flag = at<int>(w, L.flag);
        auto recb = [&](int b) { return at<double>(w, L.rec) + (size_t)b * AR_SIZE; };
        T *AU = at<T>(w, L.AU);
        const size_t bN = (size_t)c.D.boxN;
        if (pre) {
            kapk = const_cast<T *>(pre);
            usk = kapk + (size_t)c.K * bN;
            uk = usk + (size_t)c.K * c.dim * bN;
        } else {
            adj_fields(Bk, ustar, krT, kapk, usk, uk);
        }
        dispatch(c, [&](auto dm, auto rt) {
            constexpr int DIM = decltype(dm)::value;
            constexpr bool ROT = decltype(rt)::value;
            for (int k = c.K - 1; k >= 0; k--) {
                // record step of the pending iteration inside this R1 (reads recb(rcur) and
                // the partials in p3, writes recb(1 - rcur))
                const bool fin = pend >= 0;
                const double *rin = recb(rcur);
                double *rout = recb(1 - rcur);
                const unsigned pnb = fin ? (unsigned)c.nblk : 0u;
                const int kfin = pend;
                pf->run(LKS_K_ADJ_R1, [&](hipEvent_t e0, hipEvent_t e1) {
                    bool done = false;
                    if constexpr (DIM == 3 && std::is_same<T, float>::value) {
                        if (c.tile3) {
                            hipExtLaunchKernelGGL((k_adj_r1<DIM, T, true>), dim3(c.nblk), dim3(c.dblk), 0, st, e0, e1, 0,
                                                  c.g, c.D, c.bp, Bk, k, uk, krD, rin, rout, (const double *)p3,
                                                  pnb, kfin, URb, krb, p1, flag);
                            done = true;
                        }
                    }
                    if (!done)
                        hipExtLaunchKernelGGL((k_adj_r1<DIM, T>), dim3(c.nblk), dim3(R1blk<DIM>::v), 0, st, e0, e1, 0, c.g,
                                              c.D, c.bp, Bk, k, uk, krD, rin, rout, (const double *)p3, pnb, kfin,
                                              URb, krb, p1, flag);
                });
                if (fin) {
                    rcur = 1 - rcur;
                    pend = -1;
                }
                pf->run(LKS_K_ADJ_R2, [&](hipEvent_t e0, hipEvent_t e1) {
                    hipEvent_t es = e0;
                    if (DIM == 3) {  // axial sums of URb at B^(k)
                        hipExtLaunchKernelGGL((k_axial<3, T>), dim3(blocks((long long)axial_elems(c), 256), 1), dim3(256),
                                              0, st, e0, nullptr, 0, c.D, Bk, k, (const T *)URb, (long long)c.D.ND, AU);
                        es = nullptr;
                    }
                    if constexpr (DIM == 3 && ROT)  // one wave per box row (k_adj_r2_rows)
                        hipExtLaunchKernelGGL((k_adj_r2_rows<T, ROT>), dim3(blocks(box_rows(c), 4)), dim3(256), 0, st, es,
                                              e1, 0, c.g, c.bc, c.D, Bk, k, c.K, ab, (const T *)AU, kapk, usk, uk, ustb,
                                              kb, usb);
                    else
                        hipExtLaunchKernelGGL((k_adj_r2<DIM, T, ROT, lpn<DIM>()>),
                                              dim3(blocks(c.D.boxN * lpn<DIM>(), 256)), dim3(256), 0, st, es, e1, 0, c.g,
                                              c.bc, c.D, Bk, k, c.K, ab, URb, (const T *)AU, kapk, usk, uk, ustb, kb, usb);
                });
                pf->run(LKS_K_ADJ_R3, [&](hipEvent_t e0, hipEvent_t e1) {
                    const bool d = defer_finish();
                    hipExtLaunchKernelGGL((k_adj_r3<DIM, T>), dim3(c.nblk), dim3(c.dblk), 0, st, e0, d ? e1 : nullptr, 0,
                                          c.g, c.D, Bk, k, kb, usb, krD, krb, (const double *)p1, p3);
                    if (!d)
                        hipExtLaunchKernelGGL((k_r3_finish<DIM>), dim3(1), dim3(1024), 0, st, nullptr, e1, 0, c.bp, k,
                                              (const double *)p3, (unsigned)c.nblk, recb(rcur));
                });
                if (defer_finish()) pend = k;
            }
        });
    }
    // Record step of a pending iteration (after the last R3); returns the current record.
    double *rev_flush(const Layout &L, void *w) const {
        double *rec = at<double>(w, L.rec) + (size_t)rcur * AR_SIZE;
        if (pend >= 0) {
            const double *p3 = at<double>(w, L.part3);
            if (c.dim == 2)
                hipLaunchKernelGGL(k_r3_finish<2>, dim3(1), dim3(1024), 0, st, c.bp, pend, p3, (unsigned)c.nblk, rec);
            else
                hipLaunchKernelGGL(k_r3_finish<3>, dim3(1), dim3(1024), 0, st, c.bp, pend, p3, (unsigned)c.nblk, rec);
            pend = -1;
        }
        return rec;
    }
    // In 3D the cotangent ab is consumed: k_adj_fold3d and k_adj_clear3d prepare it in place.
    void adj_gather(T *ab, const T *ustb, const double *Bprev, const T *sprev, T *out, T *ups = nullptr) const {
        const int hb = c.has_body ? 1 : 0;
        pf->run_span(LKS_K_ADJ_GATHER, c.dim == 2 ? LKS_K_ADJ_GATHER_SPAN : -1,
                     [&](hipEvent_t e0, hipEvent_t e1, unsigned long long *ts) {
            if (c.dim == 2 && c.march_adj) {
                static const long long res = resident_blocks(k_adjgather2d_march<T, false>, A2_NT);
                // shift the strips by one column where a strip edge would cut the two-lane
                // reach of the one-sided transpose next to the high x face
                const int off = !c.g.per[0] && (c.g.n[0] - 62) % A2_W == 0 ? 1 : 0;
                int rows, nstrip, nwave;
                col_march(A2_W, off, res * (A2_NT / 64), rows, nstrip, nwave);
                const dim3 grid(blocks(nwave, A2_NT / 64));
                if (ts)
                    hipLaunchKernelGGL((k_adjgather2d_march<T, true>), grid, dim3(A2_NT), 0, st, c.g, c.bc, T(c.A),
                                       rows, nstrip, nwave, off, ab, ustb, Bprev, c.D, hb, sprev, out, ts, ups);
                else
                    hipExtLaunchKernelGGL((k_adjgather2d_march<T, false>), grid, dim3(A2_NT), 0, st, e0, e1, 0, c.g,
                                          c.bc, T(c.A), rows, nstrip, nwave, off, ab, ustb, Bprev, c.D, hb, sprev,
                                          out, ts, ups);
            } else if (c.dim == 2) {
                dim3 grid(blocks(c.g.n[0], G2_TX), blocks(c.g.n[1], G2_TY));
                if (ts)
                    hipLaunchKernelGGL((k_adjgather2d<T, true>), grid, dim3(G2_TX, G2_TY), 0, st, c.g, c.bc, T(c.A),
                                       ab, ustb, Bprev, c.D, hb, sprev, out, ts, ups);
                else
                    hipExtLaunchKernelGGL((k_adjgather2d<T, false>), grid, dim3(G2_TX, G2_TY), 0, st, e0, e1, 0,
                                          c.g, c.bc, T(c.A), ab, ustb, Bprev, c.D, hb, sprev, out, ts, ups);
            } else {
                static const long long res = resident_blocks(k_adjgather3d<T, false, false, true>, A3<T>::NT);
                // shift the tiles of a non-periodic axis by one node where a tile
                // boundary would fall on node n-2 (see k_adjgather3d)
                const int offx = !c.g.per[0] && (c.g.n[0] - 2) % A3<T>::OX == 0 ? 1 : 0;
                const int offy = !c.g.per[1] && (c.g.n[1] - 2) % A3<T>::OY == 0 ? 1 : 0;
                const int zc = zchunk(A3<T>::OX, A3<T>::OY, res);
                const dim3 grid(blocks(c.g.n[0] + offx, A3<T>::OX), blocks(c.g.n[1] + offy, A3<T>::OY),
                                blocks(c.g.n[2], zc));
                const long long m = layer_count(c.g.n, c.g.per);
                const long long nclr = m + (c.has_body ? c.D.boxN : 0);
                hipEvent_t es = e0;
                if (m > 0) {
                    hipExtLaunchKernelGGL((k_adj_fold3d<T>), dim3(blocks(m, 256)), dim3(256), 0, st, es, nullptr, 0,
                                          c.g, c.bc, ab, m);
                    es = nullptr;
                }
                if (nclr > 0) {
                    hipExtLaunchKernelGGL((k_adj_clear3d<T>), dim3(blocks(nclr, 256)), dim3(256), 0, st, es, nullptr,
                                          0, c.g, ab, m, c.D, Bprev, ustb, hb);
                    es = nullptr;
                }
                const dim3 blk(A3<T>::TX, A3<T>::TY);
                const T A = T(c.A);
                const T *abc = ab;
                if (whole_fields()) {
                    if (ups)
                        hipExtLaunchKernelGGL((k_adjgather3d<T, false, true, true>), grid, blk, 0, st, es, e1, 0, c.g,
                                              A, zc, offx, offy, abc, sprev, out, ts, ups);
                    else
                        hipExtLaunchKernelGGL((k_adjgather3d<T, false, false, true>), grid, blk, 0, st, es, e1, 0, c.g,
                                              A, zc, offx, offy, abc, sprev, out, ts, ups);
                } else {
                    if (ups)
                        hipExtLaunchKernelGGL((k_adjgather3d<T, false, true, false>), grid, blk, 0, st, es, e1, 0, c.g,
                                              A, zc, offx, offy, abc, sprev, out, ts, ups);
                    else
                        hipExtLaunchKernelGGL((k_adjgather3d<T, false, false, false>), grid, blk, 0, st, es, e1, 0,
                                              c.g, A, zc, offx, offy, abc, sprev, out, ts, ups);
                }
            }
        });
    }
    // The paper's adjoint variant at the time level of step j (f2.h): Bk the step's
    // records (box from B(t-1), pose B(t) = its last), state the forward state at t, ab
    // the adjoint at t (for the boundary fold), ups its moment u~*; writes the box input
    // ustb of the next ALKS step and adds the level's sensitivity to krb.
    void f2_level(const double *Bk, const T *state, const T *ab, const T *ups, T *ustb, const T *krT,
                  const double *krD, double *krb, const Layout &L, void *w, double seed, int obj) const {
        const double *B = Bk + (size_t)c.K * B_REC;
        T *F = at<T>(w, L.f2F), *hq = at<T>(w, L.f2hq);
        double *pn = at<double>(w, L.f2pn), *pd = at<double>(w, L.f2pd), *rec = at<double>(w, L.f2rec);
        const unsigned nbb = blocks(c.D.boxN, F2_NT), nbd = blocks(c.D.ND, F2_NT);
        dispatch(c, [&](auto dm, auto rt) {
            constexpr int DIM = decltype(dm)::value;
            constexpr bool ROT = decltype(rt)::value;
            hipLaunchKernelGGL((k_f2_fields<DIM, T, ROT>), dim3(nbb), dim3(F2_NT), 0, st, c.g, c.D, Bk, B, krT, state,
                               F, rec);
            for (int it = 0; it < c.K; it++) {
                const int last = it == c.K - 1;
                hipLaunchKernelGGL((k_f2_node<DIM, T>), dim3(nbb), dim3(F2_NT), 0, st, c.g, c.bc, c.D, Bk, B,
                                   (const T *)F, ups, (const double *)rec, hq, pn, last, ab, ustb);
                hipLaunchKernelGGL((k_f2_design<DIM, T>), dim3(nbd), dim3(F2_NT), 0, st, c.g, c.D, Bk, B, krD,
                                   (const T *)F, (const T *)hq, (const double *)rec, pd, 0, krb);
                hipLaunchKernelGGL((k_f2_update<DIM>), dim3(1), dim3(1024), 0, st, c.bp, obj, seed,
                                   (const double *)pn, nbb, (const double *)pd, nbd, rec, last);
            }
            hipLaunchKernelGGL((k_f2_design<DIM, T>), dim3(nbd), dim3(F2_NT), 0, st, c.g, c.D, Bk, B, krD,
                               (const T *)F, (const T *)hq, (const double *)rec, pd, 1, krb);
        });
    }
    void kappa_ref(const T *gamma, T *krT, double *krD) const {
        if (!c.has_body) return;
        hipLaunchKernelGGL(k_kappa_ref<T>, dim3(blocks(c.D.ND, 256)), dim3(256), 0, st, c.D.ND, c.bp.kmax, c.bp.q,
                           gamma, krT, krD);
    }
};

// Coupling constants K[4] (device) at pose B (a record with cos/sin) from kappa_ref in
// FP64; part holds CPL_BLOCKS * 4 doubles.
void coupling_launch(const Ctx &c, hipStream_t st, const double *B, const double *krD, double *part, double *K) {
    const unsigned nb = std::min(blocks(c.D.boxN + c.D.ND, 256), CPL_BLOCKS);
    dispatch(c, [&](auto dm, auto rt) {
        constexpr int DIM = decltype(dm)::value;
        constexpr bool ROT = decltype(rt)::value;
        hipLaunchKernelGGL((k_coupling<DIM, ROT>), dim3(nb), dim3(256), 0, st, c.g, c.D, B, krD, part);
        hipLaunchKernelGGL((k_coupling_finish<DIM>), dim3(1), dim3(1024), 0, st, (const double *)part, nb, K);
    });
}

// Stability pre-check of the fluid <-> body iteration (Sec. 3.1): LKS_EUNSTABLE when an
// active degree of freedom has K/M >= 1 (translation) or K_theta/I >= 1 (rotation).
int check_coupling(const Ctx &c, const double *K_d, hipStream_t st) {
    double K[4];
    HIP_TRY(hipMemcpyAsync(K, K_d, sizeof K, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const char *ax = "xyz";
    for (int a = 0; a < c.dim; a++)
        if ((c.bp.dof & (1 << a)) && !(K[a] / c.bp.mass < 1.0))
            return fail(LKS_EUNSTABLE,
                        "fluid <-> body iteration does not contract: K/M = %.4g along %c (K = %.6g, M = %.6g)",
                        K[a] / c.bp.mass, ax[a], K[a], c.bp.mass);
    if ((c.bp.dof & LKS_DOF_ROT) && !(K[3] / c.bp.inertia < 1.0))
        return fail(LKS_EUNSTABLE,
                    "fluid <-> body iteration does not contract: K_theta/I = %.4g (K_theta = %.6g, I = %.6g)",
                    K[3] / c.bp.inertia, K[3], c.bp.inertia);
    return LKS_OK;
}

// Divergence check of a fluid state (flag bit 8).
template <typename T> void check_state(const Ctx &c, hipStream_t st, const T *s, int *flag) {
    const unsigned nb = std::min(blocks(c.g.N, 256), 2048u);
    hipLaunchKernelGGL(k_check_state<T>, dim3(nb), dim3(256), 0, st, c.g, c.dim, s, flag);
}

int check_flag(const Ctx &, const int *flag_d, hipStream_t st) {
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, flag_d, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flag & 1) return fail(LKS_EDIVERGED, "non-finite body state");
    if (flag & 2) return fail(LKS_EDIVERGED, "body moved more than %d nodes within one step", MARGIN);
    if (flag & 8)
        return fail(LKS_EDIVERGED, "fluid state not finite, or faster than the lattice sound speed 1/sqrt(3)");
    if (flag & 4) return fail(LKS_EHIP, "internal: design tile patch exceeds its bound");
    return LKS_OK;
}

template <typename T>
int forward_impl(const Ctx &c0, const lks_problem_t *P, const T *gamma, T *state, double *body, void *ckpt,
                 void *work, double *J, hipStream_t st) {
    Ctx c = c0;
    const Layout L = layout(c, false);
    double b0[12];
    HIP_TRY(hipMemcpyAsync(b0, body, sizeof b0, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int j = 0; j < 8; j++)
        if (!std::isfinite(b0[j])) return fail(LKS_EINVAL, "initial body state not finite");
    const bool rot_any = (c.bp.dof & LKS_DOF_ROT) != 0;
    box_params(c, P, rot_any, b0[6]);
    Prof pf;
    pf.on = (P->flags & LKS_FLAG_PROFILE) != 0;
    pf.st = st;
    pf.arm(at<unsigned long long>(work, L.span), NSPAN, st);
    const int every = c.NT > 32 ? (c.NT + 31) / 32 : 1;
    Run<T> R{c, st, &pf};
    R.ax = at<T>(work, L.K1f);
    T *krT = at<T>(work, L.krT);
    double *krD = at<double>(work, L.krD);
    T *st1 = at<T>(work, L.st1), *ustar = at<T>(work, L.ustar);
    double *Bf = at<double>(work, L.Bf), *Binit = at<double>(work, L.Binit), *part = at<double>(work, L.part);
    unsigned *counter = at<unsigned>(work, L.counter);
    int *flag = at<int>(work, L.flag);
    const size_t rec = (size_t)(c.K + 1) * B_REC;
    const size_t stateB = (size_t)c.S * sizeof(T);
    hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, st, counter, 4);
    hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, st, (unsigned *)flag, 4);
    R.kappa_ref(gamma, krT, krD);
    hipLaunchKernelGGL(k_body_init<2>, dim3(1), dim3(64), 0, st, body, Bf);
    HIP_TRY(hipMemcpyAsync(Binit, Bf, B_REC * sizeof(double), hipMemcpyDeviceToDevice, st));
    if ((P->flags & LKS_FLAG_STABILITY) && c.has_body) {
        double *cp = at<double>(work, L.cpl);
        coupling_launch(c, st, Bf, krD, cp, cp + 4 * CPL_BLOCKS);
        HIP_TRY(hipGetLastError());
        const int rc = check_coupling(c, cp + 4 * CPL_BLOCKS, st);
        if (rc != LKS_OK) return rc;
    }
    if (ckpt) {
        CkptHeader h{};
        memcpy(h.magic, "LKSCKPT", 8);
        h.dim = c.dim;
        h.prec = c.prec;
        h.K = c.K;
        h.Kc = c.Kc;
        h.NT = c.NT;
        h.ncp = (int)ckpt_count(c);
        h.N = c.g.N;
        h.ND = c.has_body ? c.D.ND : 0;
        for (int a = 0; a < 3; a++) {
            h.H[a] = c.D.H[a];
            h.L[a] = c.D.L[a];
        }
        h.boxN = c.D.boxN;
        h.rot = c.rot ? 1 : 0;
        for (int a = 0; a < 3; a++) h.U[a] = c.g.U[a];
        HIP_TRY(hipMemcpyAsync(ckpt, &h, sizeof h, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    const bool shift = c.g.U[0] != 0.0 || c.g.U[1] != 0.0 || c.g.U[2] != 0.0;
    if (shift)
        hipLaunchKernelGGL(k_shift<T>, dim3(blocks(c.g.N, 256)), dim3(256), 0, st, state, c.g.N, c.dim, c.g.U[0],
                           c.g.U[1], c.g.U[2], -1.0);
    T *cur = state, *nxt = st1;
    // the fluid state is checked for divergence at every checkpoint (every 256 steps
    // without checkpoints) and at the end; the flag is read once, after the run
    const int chk = ckpt ? c.Kc : 256;
    // 2D: the boundary values of a step are formed by the next step's LKS kernel as it
    // loads them (k_gather2d with fold), so the state's boundary nodes are brought up to
    // date (k_bc) only where the state is read as a whole: checkpoints, divergence
    // checks and the end. 3D keeps the boundary launch after every step.
    const bool fold = c.dim == 2 && c.face_total > 0;
    for (int t = 1; t <= c.NT; t++) {
        double *Bc = Bf + (size_t)((t - 1) & 1) * rec;
        double *Bn = Bf + (size_t)(t & 1) * rec;
        const bool whole = (t > 1 && (t - 1) % chk == 0) || (ckpt && (t - 1) % c.Kc == 0);
        if (fold && whole && t > 1) R.bcs(cur);
        if (t > 1 && (t - 1) % chk == 0) check_state(c, st, cur, flag);
        if (ckpt && (t - 1) % c.Kc == 0) {
            const size_t ci = (size_t)((t - 1) / c.Kc);
            HIP_TRY(hipMemcpyAsync(at<char>(ckpt, ckpt_state_off(c, ci)), cur, stateB, hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipMemcpyAsync(at<char>(ckpt, ckpt_body_off(c, ci)), Bc, B_REC * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
        }
        pf.sample = (t - 1) % every == 0;
        R.gather(cur, nxt, fold && t > 1);
        if (c.has_body)
            R.body_loop(nxt, Bc, Bn, krT, krD, ustar, part, counter, flag);
        else
            HIP_TRY(hipMemcpyAsync(Bn, Bc, B_REC * sizeof(double), hipMemcpyDeviceToDevice, st));
        if (!fold) R.bcs(nxt);
        T *tmp = cur;
        cur = nxt;
        nxt = tmp;
        if ((t & 255) == 0) HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipGetLastError());
    if (fold && c.NT > 0) R.bcs(cur);
    check_state(c, st, cur, flag);
    if (cur != state) HIP_TRY(hipMemcpyAsync(state, cur, stateB, hipMemcpyDeviceToDevice, st));
    if (shift)
        hipLaunchKernelGGL(k_shift<T>, dim3(blocks(c.g.N, 256)), dim3(256), 0, st, state, c.g.N, c.dim, c.g.U[0],
                           c.g.U[1], c.g.U[2], 1.0);
    const double *Bfinal = Bf + (size_t)(c.NT & 1) * rec;
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(64), 0, st, Binit, Bfinal, P->objective, J, body);
    HIP_TRY(hipGetLastError());
    if (pf.on) {
        HIP_TRY(hipStreamSynchronize(st));
        pf.finish();
    }
    if (P->flags & LKS_FLAG_ASYNC) return LKS_OK;
    return check_flag(c, flag, st);
}

// Second stream of lks_adjoint (segment recompute beside the reverse sweep) and its
// events, created on first use by each host thread on each device and kept for the
// thread's lifetime: calls from one thread are serial, so they can share them, and calls
// from other threads get their own. Default stream priority.
struct SideRes {
    hipStream_t s = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // entry, fwd[2], rev[2]
};
thread_local std::vector<SideRes *> t_side;

int side_resources(SideRes **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if ((int)t_side.size() <= dev) t_side.resize(dev + 1, nullptr);
    if (!t_side[dev]) {
        SideRes r;
        HIP_TRY(hipStreamCreateWithFlags(&r.s, hipStreamNonBlocking));
        for (hipEvent_t &e : r.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        t_side[dev] = new SideRes(r);
    }
    *out = t_side[dev];
    return LKS_OK;
}

template <typename T>
int adjoint_impl(const Ctx &c0, const lks_problem_t *P, const T *gamma, const void *ckpt, void *work, double seed,
                 const T *dstate_T, const double *dbody_T, double *grad, T *dstate0, double *dbody0, hipStream_t st) {
    Ctx c = c0;
    CkptHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, ckpt, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (memcmp(h.magic, "LKSCKPT", 8) != 0 || h.dim != c.dim || h.prec != c.prec || h.K != c.K || h.Kc != c.Kc ||
        h.NT != c.NT || h.N != c.g.N || h.ND != (c.has_body ? c.D.ND : 0) || h.U[0] != c.g.U[0] ||
        h.U[1] != c.g.U[1] || h.U[2] != c.g.U[2])
        return fail(LKS_EINVAL, "checkpoint store does not match the problem (run lks_forward with it first)");
    if (c.has_body && (h.boxN < 1 || h.boxN > c0.D.boxN))  // the workspace holds boxes of c0.D.boxN nodes
        return fail(LKS_EINVAL, "checkpoint store: footprint box larger than the problem's");
    for (int a = 0; a < 3; a++) {
        c.D.H[a] = h.H[a];
        c.D.L[a] = h.L[a];
    }
    c.D.boxN = h.boxN;
    c.rot = h.rot != 0;
    const Layout L = layout(c0, true);  // sized with the worst-case box
    Prof pf;
    pf.on = (P->flags & LKS_FLAG_PROFILE) != 0;
    pf.st = st;
    pf.arm(at<unsigned long long>(work, L.span), NSPAN, st);
    const int every = c.NT > 32 ? (c.NT + 31) / 32 : 1;
    // The forward recompute of a segment runs on a second stream while the reverse
    // sweep of the following segment runs on `st`; two segment buffers alternate, and
    // events order each recompute after the sweep that last used its buffer and each
    // sweep after its recompute.
    // The stream and events are created once per host thread and device and kept (see
    // side_resources); at exit the call waits for the second stream's work, as its own
    // buffers are no longer needed then.
    SideRes *sr = nullptr;
    {
        const int rc = side_resources(&sr);
        if (rc != LKS_OK) return rc;
    }
    struct SideWait {
        hipStream_t s;
        ~SideWait() { (void)hipStreamSynchronize(s); }
    } side{sr->s};
    hipEvent_t evEntry = sr->ev[0], *evFwd = sr->ev + 1, *evRev = sr->ev + 3;
    Run<T> R{c, st, &pf};
    Run<T> F{c, sr->s, &pf};
    F.ax = at<T>(work, L.K1f);
    R.ax = at<T>(work, L.K1r);
    T *krT = at<T>(work, L.krT);
    double *krD = at<double>(work, L.krD);
    double *part = at<double>(work, L.part);
    unsigned *counter = at<unsigned>(work, L.counter);
    int *flag = at<int>(work, L.flag);
    T *ab = at<T>(work, L.ab);
    double *rec = at<double>(work, L.rec), *krb = at<double>(work, L.krb);
    T *ustb = at<T>(work, L.ustb);
    auto segb = [&](int b) { return at<T>(work, L.seg + (size_t)b * L.seg_n); };
    auto ustar_segb = [&](int b) { return at<T>(work, L.ustar_seg + (size_t)b * L.ustar_seg_n); };
    auto Bsegb = [&](int b) { return at<double>(work, L.Bseg + (size_t)b * L.Bseg_n); };
    auto preb = [&](int b) { return at<T>(work, L.pre + (size_t)b * L.pre_n); };
    const size_t recN = (size_t)(c.K + 1) * B_REC;
    const size_t S = (size_t)c.S;
    const size_t fp = (size_t)c.dim * (size_t)c.D.boxN;
    HIP_TRY(hipMemsetAsync(counter, 0, 16, st));
    HIP_TRY(hipMemsetAsync(flag, 0, 16, st));
    R.kappa_ref(gamma, krT, krD);
    if (c.has_body) HIP_TRY(hipMemsetAsync(krb, 0, (size_t)c.D.ND * 8, st));
    // terminal adjoint values: the given cotangent of the final state (else zero), the
    // seed on the objective's coordinate plus the given cotangent of the final body
    if (dstate_T) HIP_TRY(hipMemcpyAsync(ab, dstate_T, S * sizeof(T), hipMemcpyDeviceToDevice, st));
    else HIP_TRY(hipMemsetAsync(ab, 0, S * sizeof(T), st));
    if (c.dim == 2)
        hipLaunchKernelGGL(k_adj_init<2>, dim3(1), dim3(64), 0, st, c.bp, P->objective, seed, dbody_T, rec);
    else
        hipLaunchKernelGGL(k_adj_init<3>, dim3(1), dim3(64), 0, st, c.bp, P->objective, seed, dbody_T, rec);
    HIP_TRY(hipEventRecord(evEntry, st));
    HIP_TRY(hipStreamWaitEvent(sr->s, evEntry, 0));
    T *ab_cur = ab, *ab_nxt = ab + S;
    // the paper's variant: its moment u~* of the current and next level (zero at N_t),
    // and its body-adjoint record (zero at level N_t + 1)
    T *ups_cur = nullptr, *ups_nxt = nullptr;
    if (c.paper && c.has_body) {
        ups_cur = at<T>(work, L.f2ups);
        ups_nxt = ups_cur + (size_t)c.dim * c.g.N;
        HIP_TRY(hipMemsetAsync(ups_cur, 0, (size_t)c.dim * c.g.N * sizeof(T), st));
        hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, st, at<unsigned>(work, L.f2rec), 2 * F2_REC);
    }
    const int ncp = (int)ckpt_count(c);
    // recompute segment ci into buffer ci & 1, keeping every state, footprint u* and iterate
    auto recompute = [&](int ci) -> int {
        const int b = ci & 1;
        const int t0 = ci * c.Kc, t1 = std::min(t0 + c.Kc, c.NT), len = t1 - t0;
        T *seg = segb(b), *ustar_seg = ustar_segb(b);
        double *Bseg = Bsegb(b);
        if (ci + 2 < ncp) HIP_TRY(hipStreamWaitEvent(sr->s, evRev[b], 0));
        HIP_TRY(hipMemcpyAsync(seg, at<const char>(const_cast<void *>(ckpt), ckpt_state_off(c, ci)), S * sizeof(T),
                               hipMemcpyDeviceToDevice, side.s));
        HIP_TRY(hipMemcpyAsync(Bseg + recN, at<const char>(const_cast<void *>(ckpt), ckpt_body_off(c, ci)),
                               B_REC * sizeof(double), hipMemcpyDeviceToDevice, side.s));
        for (int j = 1; j <= len; j++) {
            pf.sample = (t0 + j - 1) % every == 0;
            T *prev = seg + (size_t)(j - 1) * S, *cur = seg + (size_t)j * S;
            double *Bk = Bseg + (size_t)j * recN;
            F.gather(prev, cur);
            if (c.has_body)
                F.body_loop(cur, Bk, Bseg + (size_t)(j + 1) * recN, krT, krD, ustar_seg + (size_t)(j - 1) * fp, part,
                            counter, flag);
            F.bcs(cur);
            if (L.pre_n) {  // 2D: the step's footprint fields for the reverse sweep
                T *pk = preb(b) + (size_t)(j - 1) * pre_elems(c);
                T *pu = pk + (size_t)c.K * c.D.boxN;
                F.adj_fields(Bk, ustar_seg + (size_t)(j - 1) * fp, krT, pk, pu, pu + (size_t)c.K * c.dim * c.D.boxN);
            }
        }
        HIP_TRY(hipEventRecord(evFwd[b], side.s));
        return LKS_OK;
    };
    if (ncp > 0) {
        const int r0 = recompute(ncp - 1);
        if (r0 != LKS_OK) return r0;
    }
    for (int ci = ncp - 1; ci >= 0; ci--) {
        if (ci - 1 >= 0) {
            const int r1 = recompute(ci - 1);
            if (r1 != LKS_OK) return r1;
        }
        const int b = ci & 1;
        const int t0 = ci * c.Kc, t1 = std::min(t0 + c.Kc, c.NT), len = t1 - t0;
        T *seg = segb(b), *ustar_seg = ustar_segb(b);
        double *Bseg = Bsegb(b);
        HIP_TRY(hipStreamWaitEvent(st, evFwd[b], 0));
        // sweep the segment backwards
        for (int j = len; j >= 1; j--) {
            pf.sample = (t0 + j - 1) % every == 0;
            const double *Bk = Bseg + (size_t)j * recN;
            if (c.has_body && c.paper)
                R.f2_level(Bk, seg + (size_t)j * S, ab_cur, ups_cur, ustb, krT, krD, krb, L, work, seed,
                           P->objective);
            else if (c.has_body)
                R.body_rev(Bk, ustar_seg + (size_t)(j - 1) * fp, ab_cur, krT, krD, L, work,
                           L.pre_n ? preb(b) + (size_t)(j - 1) * pre_elems(c) : nullptr);
            R.adj_gather(ab_cur, ustb, Bk, seg + (size_t)(j - 1) * S, ab_nxt, ups_nxt);
            T *tmp = ab_cur;
            ab_cur = ab_nxt;
            ab_nxt = tmp;
            tmp = ups_cur;
            ups_cur = ups_nxt;
            ups_nxt = tmp;
        }
        HIP_TRY(hipEventRecord(evRev[b], st));
        HIP_TRY(hipGetLastError());
    }
    if (c.has_body) {
        if (!c.paper) rec = R.rev_flush(L, work);
        hipLaunchKernelGGL(k_grad_final<T>, dim3(blocks(c.D.ND, 256)), dim3(256), 0, st, c.D.ND, c.bp.kmax, c.bp.q,
                           gamma, krb, grad, rec, P->objective, seed, dbody0);
    }
    else if (dbody0)
        HIP_TRY(hipMemsetAsync(dbody0, 0, 12 * sizeof(double), st));
    if (dstate0) HIP_TRY(hipMemcpyAsync(dstate0, ab_cur, S * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipGetLastError());
    if (pf.on) {
        HIP_TRY(hipStreamSynchronize(st));
        pf.finish();
    }
    if (P->flags & LKS_FLAG_ASYNC) return LKS_OK;
    return check_flag(c, flag, st);
}

}  // namespace

// =================================================================== design filter
namespace {

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

// Problem and filter parameters of lks_design_filter(_adjoint).
int filter_ctx(const lks_problem_t *P, const lks_filter_t *F, Ctx &c, FltArgs &a) {
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!c.has_body) return fail(LKS_EINVAL, "the design filter needs a design grid");
    if (!F) return fail(LKS_EINVAL, "null filter parameters");
    const int rmax = c.dim == 2 ? FltShape<2, float>::RMAX : FltShape<3, float>::RMAX;
    if (!(F->radius > 0.0) || !(F->radius < rmax + 1.0))
        return fail(LKS_EINVAL, "filter radius %g outside (0, %d)", F->radius, rmax + 1);
    if (!(F->beta > 0.0) || !std::isfinite(F->beta)) return fail(LKS_EINVAL, "projection beta must be > 0");
    if (!(F->eta >= 0.0 && F->eta <= 1.0)) return fail(LKS_EINVAL, "projection eta must lie in [0, 1]");
    for (int k = 0; k < 3; k++) a.n[k] = c.D.nd[k];
    a.r = (int)std::floor(F->radius);
    a.R = F->radius;
    a.beta = F->beta;
    a.eta = F->eta;
    return LKS_OK;
}

// Launch configuration of the tile kernel for FltShape<DIM, A>.
template <int DIM, typename A> dim3 filter_grid(const Ctx &c) {
    using F = FltShape<DIM, A>;
    return dim3(blocks(c.D.nd[0], F::TX), blocks(c.D.nd[1], F::TY), blocks(c.D.nd[2], F::TZ));
}

// Runs `launch(e0, e1)` (the unit's first launch takes e0, its last e1), timed under `id`
// with LKS_FLAG_PROFILE.
template <typename L> int filter_timed(bool prof, int id, hipStream_t st, L &&launch) {
    Prof pf;
    pf.on = pf.sample = prof;
    pf.st = st;
    pf.run(id, launch);
    HIP_TRY(hipGetLastError());
    if (pf.on) {
        HIP_TRY(hipStreamSynchronize(st));
        pf.finish();
    }
    return LKS_OK;
}

// Calls f(std::integral_constant<int, r>) for the run-time radius r in [0, RM].
template <int RM, typename Fn> int with_radius(int r, Fn &&f) {
    if constexpr (RM >= 0) {
        if (r == RM) return f(std::integral_constant<int, RM>{});
        return with_radius<RM - 1>(r, f);
    } else {
        return fail(LKS_EINVAL, "filter radius out of range");
    }
}

// Calls f(std::integral_constant<int, K2>) for the smallest compiled tap set of radius RR
// that holds every offset with |d|^2 <= floor(R^2).
template <int DIM, int RR, typename Fn> int with_tapset(double R, Fn &&f) {
    const int k2 = (int)std::floor(R * R);
    if constexpr (DIM == 3 && RR > 0) {
        if (k2 <= FLT_K2<RR, 0>) return f(std::integral_constant<int, FLT_K2<RR, 0>>{});
        if (k2 <= FLT_K2<RR, 1>) return f(std::integral_constant<int, FLT_K2<RR, 1>>{});
    }
    (void)k2;
    return f(std::integral_constant<int, FLT_K2<RR, 2>>{});
}

template <int DIM, typename T>
int filter_fwd(const Ctx &c, const FltArgs &a, bool prof, hipStream_t st, const T *g, T *gt, T *gh) {
    return with_radius<FltShape<DIM, T>::RMAX>(a.r, [&](auto rc) {
        constexpr int RR = decltype(rc)::value;
        return with_tapset<DIM, RR>(a.R, [&](auto kc) {
            constexpr int K2 = decltype(kc)::value;
            return filter_timed(prof, LKS_K_FILTER, st, [&](hipEvent_t e0, hipEvent_t e1) {
                hipExtLaunchKernelGGL((k_filter_tile<DIM, T, RR, K2, true>), filter_grid<DIM, T>(c),
                                      dim3(FltShape<DIM, T>::NT), 0, st, e0, e1, 0, a, g, gt, gh);
            });
        });
    });
}

template <int DIM, typename T>
int filter_adj(const Ctx &c, const FltArgs &a, bool prof, hipStream_t st, const T *gt, const double *gbh,
               double *t, double *gb) {
    return with_radius<FltShape<DIM, double>::RMAX>(a.r, [&](auto rc) {
        constexpr int RR = decltype(rc)::value;
        return with_tapset<DIM, RR>(a.R, [&](auto kc) {
            constexpr int K2 = decltype(kc)::value;
            return filter_timed(prof, LKS_K_FILTER_ADJ, st, [&](hipEvent_t e0, hipEvent_t e1) {
                const long long nd = c.D.ND;
                hipExtLaunchKernelGGL((k_filter_scale<DIM, T, RR>), dim3(blocks(nd, FLT_SCALE_NT * FLT_SCALE_PT)),
                                      dim3(FLT_SCALE_NT), 0, st, e0, nullptr, 0, a, nd, gt, gbh, t);
                hipExtLaunchKernelGGL((k_filter_tile<DIM, double, RR, K2, false>), filter_grid<DIM, double>(c),
                                      dim3(FltShape<DIM, double>::NT), 0, st, nullptr, e1, 0, a,
                                      (const double *)t, gb, (double *)nullptr);
            });
        });
    });
}

}  // namespace

// =================================================================== cyclic design
namespace {

int cyc_ctx(const lks_problem_t *P, int n_sec, Ctx &c, CycArgs &a) {
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!c.has_body) return fail(LKS_EINVAL, "the cyclic design needs a design grid");
    for (int k = 0; k < 3; k++) a.nd[k] = c.D.nd[k];
    a.pi = c.D.pi;
    a.pj = c.D.pj;
    a.ax = c.D.axis;
    a.n_sec = n_sec;
    a.sector_plane = cyc_sector_plane(a.nd[a.pi], a.nd[a.pj], n_sec);
    if (a.sector_plane < 0)
        return fail(LKS_EINVAL, "%d sectors: supported are 1, 2 and (square rotation plane) 4", n_sec);
    return LKS_OK;
}

}  // namespace

// =================================================================== C ABI
namespace {

// MMA workspace: coefficients (MC_COUNT n doubles), block partials, the state.
// ------------------------------------------------------------------ no-allocation scratch
// Workspace of lks_forward_noalloc: a file-scope device array that every GPU the library
// runs on holds until the process ends. Host code never passes its name to a kernel (in
// host code the name is a host-side stand-in): the address is taken once per device,
// with that device current, and kept.
static __device__ __align__(256) unsigned char scratch[LKS_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device id, null until taken

int noalloc_scratch(void **ptr) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LKS_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return LKS_OK;
}

unsigned mma_blocks(long long n) { return std::min(blocks(n, MMA_NT), 1024u); }
size_t mma_work_bytes(long long n) {
    const size_t nb = mma_blocks(n);
    return (size_t)MC_COUNT * (size_t)n * 8 + nb * MMA_M * 8 + 256;
}

}  // namespace

extern "C" {

const char *lks_last_error(void) { return g_err.c_str(); }

int lks_profile_read(int kernel, double *total_ms, long long *samples) {
    if (kernel < 0 || kernel >= LKS_K_COUNT) return fail(LKS_EINVAL, "unknown kernel id %d", kernel);
    if (total_ms) *total_ms = g_prof_ms[kernel];
    if (samples) *samples = g_prof_n[kernel];
    return LKS_OK;
}

void lks_profile_reset(void) {
    for (int k = 0; k < LKS_K_COUNT; k++) {
        g_prof_ms[k] = 0.0;
        g_prof_n[k] = 0;
    }
}

size_t lks_state_elems(const lks_problem_t *P) {
    Ctx c;
    if (make_ctx(P, c) != LKS_OK) return 0;
    return (size_t)c.S;
}

size_t lks_checkpoint_bytes(const lks_problem_t *P) {
    Ctx c;
    if (make_ctx(P, c) != LKS_OK) return 0;
    if (c.Kc < 1) {
        fail(LKS_EINVAL, "ckpt_every must be >= 1 to store checkpoints");
        return 0;
    }
    return ckpt_bytes(c);
}

size_t lks_workspace_bytes(const lks_problem_t *P, int adjoint) {
    Ctx c;
    if (make_ctx(P, c) != LKS_OK) return 0;
    if (adjoint && c.Kc < 1) {
        fail(LKS_EINVAL, "ckpt_every must be >= 1 for the adjoint");
        return 0;
    }
    return layout(c, adjoint != 0).total;
}

int lks_forward(const lks_problem_t *P, const void *gamma, void *state, double *body, void *ckpt,
                size_t ckpt_bytes_, void *work, size_t work_bytes, double *J, void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!state || !body || !work || !J || (c.has_body && !gamma)) return fail(LKS_EINVAL, "null pointer argument");
    if (work_bytes < layout(c, false).total) return fail(LKS_ENOSPACE, "work buffer too small");
    if (ckpt) {
        if (c.Kc < 1) return fail(LKS_EINVAL, "ckpt_every must be >= 1 to store checkpoints");
        if (ckpt_bytes_ < ckpt_bytes(c)) return fail(LKS_ENOSPACE, "checkpoint buffer too small");
    }
    hipStream_t st = (hipStream_t)stream;
    if (c.prec == LKS_FP32)
        return forward_impl<float>(c, P, (const float *)gamma, (float *)state, body, ckpt, work, J, st);
    return forward_impl<double>(c, P, (const double *)gamma, (double *)state, body, ckpt, work, J, st);
}

int lks_forward_noalloc(const lks_problem_t *P, const void *gamma, void *state, double *body, double *J,
                        void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!state || !body || !J || (c.has_body && !gamma)) return fail(LKS_EINVAL, "null pointer argument");
    if (P->flags & LKS_FLAG_PROFILE)
        return fail(LKS_EINVAL, "lks_forward_noalloc: LKS_FLAG_PROFILE is not available (it creates events)");
    const size_t need = layout(c, false).total;
    if (need > LKS_NOALLOC_SCRATCH_BYTES)
        return fail(LKS_ENOSPACE, "lks_forward_noalloc: the problem needs %zu bytes of scratch, the static array holds %zu",
                    need, (size_t)LKS_NOALLOC_SCRATCH_BYTES);
    void *work = nullptr;
    rc = noalloc_scratch(&work);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (c.prec == LKS_FP32)
        return forward_impl<float>(c, P, (const float *)gamma, (float *)state, body, nullptr, work, J, st);
    return forward_impl<double>(c, P, (const double *)gamma, (double *)state, body, nullptr, work, J, st);
}

int lks_adjoint(const lks_problem_t *P, const void *gamma, const void *ckpt, size_t ckpt_bytes_, void *work,
                size_t work_bytes, double seed, const void *dstate_T, const double *dbody_T, double *grad,
                void *dstate0, double *dbody0, void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (c.Kc < 1) return fail(LKS_EINVAL, "ckpt_every must be >= 1");
    if (!ckpt || !work || (c.has_body && (!gamma || !grad))) return fail(LKS_EINVAL, "null pointer argument");
    if (ckpt_bytes_ < ckpt_bytes(c)) return fail(LKS_ENOSPACE, "checkpoint buffer too small");
    if (work_bytes < layout(c, true).total) return fail(LKS_ENOSPACE, "work buffer too small");
    if (!std::isfinite(seed)) return fail(LKS_EINVAL, "seed not finite");
    if (c.paper && !c.has_body) return fail(LKS_EINVAL, "LKS_FLAG_PAPER_ADJOINT needs a design grid");
    if (c.paper && (dstate_T || dbody_T || dstate0 || dbody0))
        return fail(LKS_EINVAL, "LKS_FLAG_PAPER_ADJOINT takes no terminal cotangents and returns no initial ones");
    if (dstate_T && overlap(dstate_T, (size_t)c.S * c.elt, work, work_bytes))
        return fail(LKS_EINVAL, "dstate_T must not overlap work");
    hipStream_t st = (hipStream_t)stream;
    if (c.prec == LKS_FP32)
        return adjoint_impl<float>(c, P, (const float *)gamma, ckpt, work, seed, (const float *)dstate_T, dbody_T,
                                   grad, (float *)dstate0, dbody0, st);
    return adjoint_impl<double>(c, P, (const double *)gamma, ckpt, work, seed, (const double *)dstate_T, dbody_T,
                                grad, (double *)dstate0, dbody0, st);
}

int map_design(const lks_problem_t *P, const void *kappa_ref, const double *body, void *kappa, void *uS,
               void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!c.has_body) return fail(LKS_EINVAL, "map_design needs a design grid");
    if (!kappa_ref || !body || !kappa || !uS) return fail(LKS_EINVAL, "null pointer argument");
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(blocks(c.g.N, 256));
#define MAP_LAUNCH(D_, T_)                                                                                   \
    hipLaunchKernelGGL((k_spread_map<D_, T_>), grid, dim3(256), 0, st, c.g, c.D, body, (const T_ *)kappa_ref, \
                       (T_ *)kappa, (T_ *)uS)
    if (c.dim == 2 && c.prec == LKS_FP32) MAP_LAUNCH(2, float);
    else if (c.dim == 2) MAP_LAUNCH(2, double);
    else if (c.prec == LKS_FP32) MAP_LAUNCH(3, float);
    else MAP_LAUNCH(3, double);
#undef MAP_LAUNCH
    HIP_TRY(hipGetLastError());
    return LKS_OK;
}

int body_step(const lks_problem_t *P, const double *ft, const double *body_prev, double *body, void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!ft || !body_prev || !body) return fail(LKS_EINVAL, "null pointer argument");
    if (body == body_prev) return fail(LKS_EINVAL, "body must not alias body_prev");
    hipStream_t st = (hipStream_t)stream;
    if (c.dim == 2)
        hipLaunchKernelGGL(k_body_step<2>, dim3(1), dim3(64), 0, st, c.bp, ft, body_prev, body);
    else
        hipLaunchKernelGGL(k_body_step<3>, dim3(1), dim3(64), 0, st, c.bp, ft, body_prev, body);
    HIP_TRY(hipGetLastError());
    return LKS_OK;
}

int lks_coupling(const lks_problem_t *P, const void *gamma, const double *body, double *K, void *work,
                 size_t work_bytes, void *stream) {
    g_err.clear();
    Ctx c;
    int rc = make_ctx(P, c);
    if (rc) return rc;
    if (!c.has_body) return fail(LKS_EINVAL, "the problem has no design grid");
    if (!gamma || !body || !K || !work) return fail(LKS_EINVAL, "null pointer argument");
    const Layout L = layout(c, false);
    if (work_bytes < L.total) return fail(LKS_ENOSPACE, "work buffer too small");
    hipStream_t st = (hipStream_t)stream;
    double b0[12];
    HIP_TRY(hipMemcpyAsync(b0, body, sizeof b0, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int j = 0; j < 8; j++)
        if (!std::isfinite(b0[j])) return fail(LKS_EINVAL, "body state not finite");
    box_params(c, P, (c.bp.dof & LKS_DOF_ROT) != 0, b0[6]);
    double *krD = at<double>(work, L.krD), *Bf = at<double>(work, L.Bf), *cp = at<double>(work, L.cpl);
    Prof pf;
    if (c.prec == LKS_FP32) {
        Run<float> R{c, st, &pf};
        R.kappa_ref((const float *)gamma, at<float>(work, L.krT), krD);
    } else {
        Run<double> R{c, st, &pf};
        R.kappa_ref((const double *)gamma, at<double>(work, L.krT), krD);
    }
    hipLaunchKernelGGL(k_body_init<2>, dim3(1), dim3(64), 0, st, body, Bf);
    coupling_launch(c, st, Bf, krD, cp, K);
    HIP_TRY(hipGetLastError());
    return LKS_OK;
}

int lks_design_filter(const lks_problem_t *P, const lks_filter_t *F, const void *gamma, void *gamma_tilde,
                      void *gamma_hat, void *stream) {
    g_err.clear();
    Ctx c;
    FltArgs a;
    int rc = filter_ctx(P, F, c, a);
    if (rc) return rc;
    if (!gamma || !gamma_tilde || !gamma_hat) return fail(LKS_EINVAL, "null pointer argument");
    const size_t nb = (size_t)c.D.ND * c.elt;
    if (overlap(gamma, nb, gamma_tilde, nb) || overlap(gamma, nb, gamma_hat, nb) ||
        overlap(gamma_tilde, nb, gamma_hat, nb))
        return fail(LKS_EINVAL, "gamma, gamma_tilde and gamma_hat must not overlap");
    hipStream_t st = (hipStream_t)stream;
    const bool prof = (P->flags & LKS_FLAG_PROFILE) != 0;
    if (c.dim == 2 && c.prec == LKS_FP32)
        return filter_fwd<2>(c, a, prof, st, (const float *)gamma, (float *)gamma_tilde, (float *)gamma_hat);
    if (c.dim == 2)
        return filter_fwd<2>(c, a, prof, st, (const double *)gamma, (double *)gamma_tilde, (double *)gamma_hat);
    if (c.prec == LKS_FP32)
        return filter_fwd<3>(c, a, prof, st, (const float *)gamma, (float *)gamma_tilde, (float *)gamma_hat);
    return filter_fwd<3>(c, a, prof, st, (const double *)gamma, (double *)gamma_tilde, (double *)gamma_hat);
}

size_t lks_filter_workspace_bytes(const lks_problem_t *P) {
    Ctx c;
    if (make_ctx(P, c) != LKS_OK) return 0;
    if (!c.has_body) {
        fail(LKS_EINVAL, "the design filter needs a design grid");
        return 0;
    }
    return up((size_t)c.D.ND * sizeof(double));
}

int lks_design_filter_adjoint(const lks_problem_t *P, const lks_filter_t *F, const void *gamma_tilde,
                              const double *dJ_dgamma_hat, void *work, size_t work_bytes, double *dJ_dgamma,
                              void *stream) {
    g_err.clear();
    Ctx c;
    FltArgs a;
    int rc = filter_ctx(P, F, c, a);
    if (rc) return rc;
    if (!gamma_tilde || !dJ_dgamma_hat || !work || !dJ_dgamma) return fail(LKS_EINVAL, "null pointer argument");
    const size_t nt = (size_t)c.D.ND * c.elt, nd = (size_t)c.D.ND * sizeof(double);
    if (work_bytes < nd) return fail(LKS_ENOSPACE, "work buffer too small");
    if (overlap(dJ_dgamma, nd, gamma_tilde, nt) || overlap(dJ_dgamma, nd, dJ_dgamma_hat, nd) ||
        overlap(work, nd, gamma_tilde, nt) || overlap(work, nd, dJ_dgamma_hat, nd) || overlap(work, nd, dJ_dgamma, nd))
        return fail(LKS_EINVAL, "dJ_dgamma, work, gamma_tilde and dJ_dgamma_hat must not overlap");
    hipStream_t st = (hipStream_t)stream;
    const bool prof = (P->flags & LKS_FLAG_PROFILE) != 0;
    double *t = (double *)work;
    if (c.dim == 2 && c.prec == LKS_FP32)
        return filter_adj<2>(c, a, prof, st, (const float *)gamma_tilde, dJ_dgamma_hat, t, dJ_dgamma);
    if (c.dim == 2) return filter_adj<2>(c, a, prof, st, (const double *)gamma_tilde, dJ_dgamma_hat, t, dJ_dgamma);
    if (c.prec == LKS_FP32)
        return filter_adj<3>(c, a, prof, st, (const float *)gamma_tilde, dJ_dgamma_hat, t, dJ_dgamma);
    return filter_adj<3>(c, a, prof, st, (const double *)gamma_tilde, dJ_dgamma_hat, t, dJ_dgamma);
}

size_t lks_cyclic_sector_points(const lks_problem_t *P, int n_sectors) {
    Ctx c;
    CycArgs a;
    if (cyc_ctx(P, n_sectors, c, a) != LKS_OK) return 0;
    return (size_t)(a.sector_plane * a.nd[a.ax]);
}

int lks_design_cyclic_expand(const lks_problem_t *P, int n_sectors, const void *gamma_sector, void *gamma,
                             void *stream) {
    g_err.clear();
    Ctx c;
    CycArgs a;
    int rc = cyc_ctx(P, n_sectors, c, a);
    if (rc) return rc;
    if (!gamma_sector || !gamma) return fail(LKS_EINVAL, "null pointer argument");
    const size_t ns = (size_t)(a.sector_plane * a.nd[a.ax]);
    if (overlap(gamma_sector, ns * c.elt, gamma, (size_t)c.D.ND * c.elt))
        return fail(LKS_EINVAL, "gamma_sector and gamma must not overlap");
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(blocks(c.D.ND, 256));
    return filter_timed((P->flags & LKS_FLAG_PROFILE) != 0, LKS_K_CYC_EXPAND, st, [&](hipEvent_t e0, hipEvent_t e1) {
        if (c.prec == LKS_FP32)
            hipExtLaunchKernelGGL(k_cyc_expand<float>, grid, dim3(256), 0, st, e0, e1, 0, a,
                                  (const float *)gamma_sector, (float *)gamma);
        else
            hipExtLaunchKernelGGL(k_cyc_expand<double>, grid, dim3(256), 0, st, e0, e1, 0, a,
                                  (const double *)gamma_sector, (double *)gamma);
    });
}

int lks_design_cyclic_collect(const lks_problem_t *P, int n_sectors, const double *grad, double *grad_sector,
                              void *stream) {
    g_err.clear();
    Ctx c;
    CycArgs a;
    int rc = cyc_ctx(P, n_sectors, c, a);
    if (rc) return rc;
    if (!grad || !grad_sector) return fail(LKS_EINVAL, "null pointer argument");
    const long long ns = a.sector_plane * a.nd[a.ax];
    if (overlap(grad, (size_t)c.D.ND * 8, grad_sector, (size_t)ns * 8))
        return fail(LKS_EINVAL, "grad and grad_sector must not overlap");
    hipStream_t st = (hipStream_t)stream;
    return filter_timed((P->flags & LKS_FLAG_PROFILE) != 0, LKS_K_CYC_COLLECT, st, [&](hipEvent_t e0, hipEvent_t e1) {
        hipExtLaunchKernelGGL(k_cyc_collect, dim3(blocks(ns, 256)), dim3(256), 0, st, e0, e1, 0, a, grad, grad_sector);
    });
}

size_t lks_mma_workspace_bytes(long long n) {
    if (n < 1) {
        fail(LKS_EINVAL, "n < 1");
        return 0;
    }
    return mma_work_bytes(n);
}

int lks_mma_update(const lks_mma_t *opt, long long n, int iter, double *x, const double *xold1, const double *xold2,
                   double *low, double *upp, const double *df0, const double *g1, const double *dg1, double *lambda,
                   void *work, size_t work_bytes, void *stream) {
    if (!opt) return fail(LKS_EINVAL, "null MMA parameters");
    if (n < 1) return fail(LKS_EINVAL, "n < 1");
    if (iter < 1) return fail(LKS_EINVAL, "iter < 1");
    if (!(opt->xmin < opt->xmax) || !std::isfinite(opt->xmin) || !std::isfinite(opt->xmax))
        return fail(LKS_EINVAL, "need xmin < xmax");
    if (!(opt->move > 0.0)) return fail(LKS_EINVAL, "move limit must be > 0");
    if (!std::isfinite(opt->f0_scale)) return fail(LKS_EINVAL, "f0_scale must be finite");
    if (!x || !low || !upp || !df0 || !g1 || !dg1 || !work) return fail(LKS_EINVAL, "null pointer");
    if (iter > 2 && (!xold1 || !xold2)) return fail(LKS_EINVAL, "iter > 2 needs x^(k-1) and x^(k-2)");
    if (work_bytes < mma_work_bytes(n)) return fail(LKS_EINVAL, "workspace too small");
    const size_t nb8 = (size_t)n * 8;
    const void *ins[] = {xold1, xold2, df0, dg1, g1, lambda};
    const size_t insz[] = {nb8, nb8, nb8, nb8, 8, 8};
    void *outs[] = {x, low, upp};
    for (void *o : outs) {
        for (int i = 0; i < 6; i++)
            if (ins[i] && overlap(o, nb8, ins[i], insz[i])) return fail(LKS_EINVAL, "an output overlaps an input");
        if (overlap(o, nb8, work, work_bytes)) return fail(LKS_EINVAL, "an output overlaps the workspace");
    }
    for (int i = 0; i < 6; i++)
        if (ins[i] && overlap(work, work_bytes, ins[i], insz[i])) return fail(LKS_EINVAL, "an input overlaps the workspace");
    if (overlap(x, nb8, low, nb8) || overlap(x, nb8, upp, nb8) || overlap(low, nb8, upp, nb8))
        return fail(LKS_EINVAL, "x, low and upp overlap");
    hipStream_t st = (hipStream_t)stream;
    MmaArgs a;
    a.xmin = opt->xmin;
    a.xmax = opt->xmax;
    a.move = opt->move;
    a.f0_scale = opt->f0_scale;
    a.iter = iter;
    const unsigned nb = mma_blocks(n);
    double *coef = (double *)work;
    double *part = coef + (size_t)MC_COUNT * n;
    MmaState *ms = (MmaState *)(part + (size_t)nb * MMA_M);
    hipLaunchKernelGGL(k_mma_prep, dim3(nb), dim3(MMA_NT), 0, st, a, n, (const double *)x, xold1, xold2, low, upp,
                       df0, dg1, coef, part);
    hipLaunchKernelGGL(k_mma_r1, dim3(1), dim3(MMA_NT), 0, st, (const double *)part, (int)nb, g1, ms);
    for (int pass = 0; pass < MMA_PASSES; pass++) {
        hipLaunchKernelGGL(k_mma_dual, dim3(nb), dim3(MMA_NT), 0, st, n, pass, (const double *)coef,
                           (const MmaState *)ms, part);
        hipLaunchKernelGGL(k_mma_pick, dim3(1), dim3(MMA_PICK_NT), 0, st, pass, (const double *)part, (int)nb, ms);
    }
    hipLaunchKernelGGL(k_mma_x, dim3(nb), dim3(MMA_NT), 0, st, n, (const double *)coef, (const MmaState *)ms, x,
                       lambda);
    HIP_TRY(hipGetLastError());
    return LKS_OK;
}

int lks_volume_constraint(long long n, const double *gh, double vmin, double *G, double *dG, void *work,
                          size_t work_bytes, void *stream) {
    if (n < 1) return fail(LKS_EINVAL, "n < 1");
    if (!(vmin > 0.0) || !std::isfinite(vmin)) return fail(LKS_EINVAL, "vmin must be > 0");
    if (!gh || !G || !work) return fail(LKS_EINVAL, "null pointer");
    if (work_bytes < mma_work_bytes(n)) return fail(LKS_EINVAL, "workspace too small");
    const size_t nb8 = (size_t)n * 8;
    if (overlap(G, 8, gh, nb8) || (dG && (overlap(dG, nb8, gh, nb8) || overlap(dG, nb8, G, 8))))
        return fail(LKS_EINVAL, "outputs overlap the input");
    if (overlap(work, work_bytes, gh, nb8) || overlap(work, work_bytes, G, 8) ||
        (dG && overlap(work, work_bytes, dG, nb8)))
        return fail(LKS_EINVAL, "the workspace overlaps an argument");
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = mma_blocks(n);
    double *part = (double *)work;
    hipLaunchKernelGGL(k_vol_part, dim3(nb), dim3(MMA_NT), 0, st, n, gh, part);
    hipLaunchKernelGGL(k_vol_finish, dim3(nb), dim3(MMA_NT), 0, st, n, vmin, (const double *)part, (int)nb, G, dG);
    HIP_TRY(hipGetLastError());
    return LKS_OK;
}

}  // extern "C"
