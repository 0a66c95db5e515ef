// MMA design update on the GPU (FP64): the method of moving asymptotes for one
// inequality constraint, which the paper uses to update the design (Sec. 3.5,
// Algorithm 1: gamma^k, dJ/dgamma, G, dG/dgamma -> gamma^(k+1)).
//
// Per variable j (one thread each, grid-stride): the moving asymptotes L_j < x_j < U_j,
// the move limits [alpha_j, beta_j] and the coefficients p_0j, q_0j, p_1j, q_1j of the
// convex separable approximations f~_i = r_i + sum_j p_ij / (U_j - x_j) + q_ij / (x_j - L_j)
// (k_mma_prep). The subproblem min f~_0 s.t. f~_1 <= 0 is solved through its dual: for a
// multiplier lam >= 0 the minimiser x_j(lam) is in closed form, and the dual derivative
// h(lam) = f~_1(x(lam)) is non-increasing. lam is found by multi-section: each pass
// evaluates h at MMA_M multipliers at once (every thread adds its variables' terms for
// all of them, fixed-order block sums stored multiplier-major, then one block with a
// wave per multiplier sums them in a fixed order and keeps the bracket [lo, hi] with
// h(lo) > 0 >= h(hi)); the first pass uses a
// geometric ladder from 0 to 10^(MMA_LOG_HI), the next ones split the bracket evenly.
// The update is x_j(hi) (k_mma_x). No atomics; two runs give the same bits.
#pragma once

namespace lks {

constexpr int MMA_NT = 256;       // threads per block
constexpr int MMA_M = 16;         // multipliers per pass
constexpr int MMA_PASSES = 16;    // passes (the bracket shrinks 15-fold per pass)
constexpr double MMA_ASYINIT = 0.5, MMA_ASYDECR = 0.7, MMA_ASYINCR = 1.2, MMA_ALBEFA = 0.1, MMA_RAA0 = 1e-5;
constexpr double MMA_LOG_LO = -16.0, MMA_LOG_HI = 20.0;  // ladder of the first pass: 0, 10^LO .. 10^HI

struct MmaArgs {
    double xmin, xmax, move, f0_scale;
    int iter;  // 1, 2, ...
};

// Device state of one update: r_1, the bracket, and whether lam is final.
struct MmaState {
    double r1, lo, hi;
    int done;
};

// Coefficients per variable (SoA, n each): p0, q0, p1, q1, L, U, alpha, beta.
enum { MC_P0 = 0, MC_Q0, MC_P1, MC_Q1, MC_L, MC_U, MC_A, MC_B, MC_COUNT };

__device__ __forceinline__ double mma_x_of(double lam, const double c[MC_COUNT]) {
    const double sp = sqrt(c[MC_P0] + lam * c[MC_P1]), sq = sqrt(c[MC_Q0] + lam * c[MC_Q1]);
    const double xs = (sp * c[MC_L] + sq * c[MC_U]) / (sp + sq);
    return fmin(fmax(xs, c[MC_A]), c[MC_B]);
}

// p_1 / (U - x) + q_1 / (x - L) over one division (x lies strictly inside (L, U)).
__device__ __forceinline__ double mma_h_term(double lam, const double c[MC_COUNT]) {
    const double x = mma_x_of(lam, c);
    const double a = c[MC_U] - x, b = x - c[MC_L];
    return (c[MC_P1] * b + c[MC_Q1] * a) / (a * b);
}

// Block sum of NV values per thread (fixed order: per wave an xor tree, then the
// waves in order); thread j < NV stores sum j into out[j * gridDim.x + blockIdx.x].
template <int NV>
__device__ __forceinline__ void mma_block_store(double v[NV], double *__restrict__ out) {
    __shared__ double red[NV][MMA_NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        double s = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[j][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < MMA_NT / 64; w++) s += red[threadIdx.x][w];
        out[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

// Steps 1-3 per variable, and each block's part of sum_j p_1j/(U_j - x_j) + q_1j/(x_j - L_j).
__global__ __launch_bounds__(MMA_NT) void k_mma_prep(MmaArgs a, long long n, const double *__restrict__ x,
                                                     const double *__restrict__ xold1,
                                                     const double *__restrict__ xold2, double *__restrict__ low,
                                                     double *__restrict__ upp, const double *__restrict__ df0,
                                                     const double *__restrict__ dg1, double *__restrict__ coef,
                                                     double *__restrict__ part) {
    const double w = a.xmax - a.xmin;
    double acc = 0.0;
    for (long long j = (long long)blockIdx.x * MMA_NT + threadIdx.x; j < n; j += (long long)gridDim.x * MMA_NT) {
        const double xj = x[j];
        double L, U;
        if (a.iter <= 2) {
            L = xj - MMA_ASYINIT * w;
            U = xj + MMA_ASYINIT * w;
        } else {
            const double x1 = xold1[j], x2 = xold2[j];
            const double s = (xj - x1) * (x1 - x2);
            const double gam = s < 0.0 ? MMA_ASYDECR : (s > 0.0 ? MMA_ASYINCR : 1.0);
            L = xj - gam * (x1 - low[j]);
            U = xj + gam * (upp[j] - x1);
            L = fmin(fmax(L, xj - 10.0 * w), xj - 0.01 * w);
            U = fmax(fmin(U, xj + 10.0 * w), xj + 0.01 * w);
        }
        low[j] = L;
        upp[j] = U;
        const double al = fmax(fmax(L + MMA_ALBEFA * (xj - L), xj - a.move * w), a.xmin);
        const double be = fmin(fmin(U - MMA_ALBEFA * (U - xj), xj + a.move * w), a.xmax);
        const double ux2 = (U - xj) * (U - xj), xl2 = (xj - L) * (xj - L);
        double pq[4];
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const double d = i == 0 ? a.f0_scale * df0[j] : dg1[j];
            const double dp = fmax(d, 0.0), dm = fmax(-d, 0.0);
            pq[2 * i] = ux2 * (1.001 * dp + 0.001 * dm + MMA_RAA0 / w);
            pq[2 * i + 1] = xl2 * (0.001 * dp + 1.001 * dm + MMA_RAA0 / w);
        }
        coef[MC_P0 * n + j] = pq[0];
        coef[MC_Q0 * n + j] = pq[1];
        coef[MC_P1 * n + j] = pq[2];
        coef[MC_Q1 * n + j] = pq[3];
        coef[MC_L * n + j] = L;
        coef[MC_U * n + j] = U;
        coef[MC_A * n + j] = al;
        coef[MC_B * n + j] = be;
        acc += pq[2] / (U - xj) + pq[3] / (xj - L);
    }
    double v[1] = {acc};
    mma_block_store<1>(v, part);
}

// One block: r_1 = g_1 - sum of the prep partials (block order); the state starts with
// the ladder pass.
__global__ __launch_bounds__(MMA_NT) void k_mma_r1(const double *__restrict__ part, int nb,
                                                   const double *__restrict__ g1, MmaState *__restrict__ st) {
    __shared__ double red[MMA_NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += MMA_NT) s += part[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < MMA_NT / 64; w++) t += red[w];
        st->r1 = g1[0] - t;
        st->lo = 0.0;
        st->hi = 0.0;
        st->done = 0;
    }
}

// The multipliers of a pass: the ladder (pass 0) or the bracket split evenly.
__device__ __forceinline__ double mma_lambda(int pass, const MmaState &s, int i) {
    if (pass == 0)
        return i == 0 ? 0.0 : exp10(MMA_LOG_LO + (MMA_LOG_HI - MMA_LOG_LO) * (double)(i - 1) / (double)(MMA_M - 2));
    return s.lo + (s.hi - s.lo) * (double)i / (double)(MMA_M - 1);
}

// Each block's part of sum_j h-terms at the pass's MMA_M multipliers.
__global__ __launch_bounds__(MMA_NT) void k_mma_dual(long long n, int pass, const double *__restrict__ coef,
                                                     const MmaState *__restrict__ st, double *__restrict__ part) {
    const MmaState s = *st;
    double acc[MMA_M];
#pragma unroll
    for (int i = 0; i < MMA_M; i++) acc[i] = 0.0;
    if (!s.done) {
        double lam[MMA_M];
#pragma unroll
        for (int i = 0; i < MMA_M; i++) lam[i] = mma_lambda(pass, s, i);
        for (long long j = (long long)blockIdx.x * MMA_NT + threadIdx.x; j < n; j += (long long)gridDim.x * MMA_NT) {
            double c[MC_COUNT];
#pragma unroll
            for (int k = 0; k < MC_COUNT; k++) c[k] = coef[k * n + j];
#pragma unroll
            for (int i = 0; i < MMA_M; i++) acc[i] += mma_h_term(lam[i], c);
        }
    }
    mma_block_store<MMA_M>(acc, part);
}

// One block, a wave per multiplier: h at the pass's multipliers from the partials (lane l
// adds blocks l, l + 64, ..., then a fixed xor tree), then the new bracket: the first
// multiplier with h <= 0 closes it; at the ladder's 0 the update is lam = 0; if none, lam
// is the last multiplier (the approximated constraint cannot be met within the move
// limits).
constexpr int MMA_PICK_NT = MMA_M * 64;
__global__ __launch_bounds__(MMA_PICK_NT) void k_mma_pick(int pass, const double *__restrict__ part, int nb,
                                                          MmaState *__restrict__ st) {
    __shared__ double h[MMA_M];
    const MmaState s = *st;
    if (s.done) return;
    const int i = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double *pi = part + (size_t)i * nb;
    double a = 0.0;
    for (int b = lane; b < nb; b += 64) a += pi[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) h[i] = s.r1 + a;
    __syncthreads();
    if (threadIdx.x != 0) return;
    int first = -1;
    for (int k = 0; k < MMA_M; k++)
        if (h[k] <= 0.0) {
            first = k;
            break;
        }
    MmaState o = s;
    if (first < 0) {  // infeasible up to the last multiplier
        o.lo = o.hi = mma_lambda(pass, s, MMA_M - 1);
        o.done = 1;
    } else if (first == 0) {  // pass 0: h(0) <= 0; later passes keep h(lo) > 0, so first > 0
        o.lo = o.hi = mma_lambda(pass, s, 0);
        o.done = pass == 0 ? 1 : 0;
    } else {
        o.lo = mma_lambda(pass, s, first - 1);
        o.hi = mma_lambda(pass, s, first);
        o.done = o.lo == o.hi;
    }
    *st = o;
}

// Step 4's result: x_j = x_j(hi).
__global__ __launch_bounds__(MMA_NT) void k_mma_x(long long n, const double *__restrict__ coef,
                                                  const MmaState *__restrict__ st, double *__restrict__ x,
                                                  double *__restrict__ lam_out) {
    const double lam = st->hi;
    for (long long j = (long long)blockIdx.x * MMA_NT + threadIdx.x; j < n; j += (long long)gridDim.x * MMA_NT) {
        double c[MC_COUNT];
#pragma unroll
        for (int k = 0; k < MC_COUNT; k++) c[k] = coef[k * n + j];
        x[j] = mma_x_of(lam, c);
    }
    if (lam_out && blockIdx.x == 0 && threadIdx.x == 0) *lam_out = lam;
}

// Volume constraint (Eq. constraint, read as a minimum-volume constraint):
// G = 1 - sum(gh) / (vmin n), dG/dgh_j = -1 / (vmin n). Block partials of sum(gh).
__global__ __launch_bounds__(MMA_NT) void k_vol_part(long long n, const double *__restrict__ gh,
                                                     double *__restrict__ part) {
    double acc = 0.0;
    for (long long j = (long long)blockIdx.x * MMA_NT + threadIdx.x; j < n; j += (long long)gridDim.x * MMA_NT)
        acc += gh[j];
    double v[1] = {acc};
    mma_block_store<1>(v, part);
}

__global__ __launch_bounds__(MMA_NT) void k_vol_finish(long long n, double vmin, const double *__restrict__ part,
                                                       int nb, double *__restrict__ G, double *__restrict__ dG) {
    if (blockIdx.x == 0) {
        __shared__ double red[MMA_NT / 64];
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += MMA_NT) s += part[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < MMA_NT / 64; w++) t += red[w];
            G[0] = 1.0 - t / (vmin * (double)n);
        }
    }
    if (dG) {
        const double d = -1.0 / (vmin * (double)n);
        for (long long j = (long long)blockIdx.x * MMA_NT + threadIdx.x; j < n; j += (long long)gridDim.x * MMA_NT)
            dG[j] = d;
    }
}

}  // namespace lks
