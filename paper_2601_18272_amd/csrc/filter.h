// filter.h -- density filter and Heaviside projection of the design field (Sec. 3.2,
// Eqs. filter and projection) and their reverse, on the design grid (spacing one).
//
//   gt_i = sum_j w_ij g_j / W_i,  w_ij = (R - |x_i - x_j|) / R on |x_i - x_j| <= R,
//          W_i = sum_j w_ij, j over the design grid (the cone is cut at the grid's edge);
//   gh_i = (tanh(beta eta) + tanh(beta (gt_i - eta))) / (tanh(beta eta) + tanh(beta (1 - eta))).
// Reverse: gb_j = sum_i w_ij t_i with t_i = gbh_i (d gh / d gt)_i / W_i (w is symmetric).
//
// A block owns a tile of design points and stages the tile plus a floor(R) halo in LDS
// (zero off the grid), together with the weights by offset. The taps of a row (dy, dz)
// of the cube run over |dx| <= the ball's half-width, which is the same for the whole
// block; weights of taps outside the ball are zero in the table. W_i is the sum of the
// whole table unless i's cube leaves the grid. Sums run in a fixed order.
#pragma once
#include "lks_device.h"

namespace lks {

struct FltArgs {
    int n[3];
    int r;  // floor(R)
    double R, beta, eta;
};

template <int DIM> struct Flt {
    static constexpr int TX = DIM == 2 ? 32 : 16, TY = DIM == 2 ? 16 : 8, TZ = DIM == 2 ? 1 : 4;
    static constexpr int NT = TX * TY * TZ;
    static constexpr int RMAX = DIM == 2 ? 8 : 4;  // largest floor(R)
    static constexpr int HN = (TX + 2 * RMAX) * (TY + 2 * RMAX) * (DIM == 2 ? 1 : TZ + 2 * RMAX);
    static constexpr int WE = 2 * RMAX + 1;
    static constexpr int WN = DIM == 2 ? WE * WE : WE * WE * WE;
};

// Weight of the offset (dx, dy, dz); the same FP64 expression for every tap.
__device__ __forceinline__ double flt_w(double R, int dx, int dy, int dz) {
    const double d = sqrt((double)(dx * dx + dy * dy + dz * dz));
    return d <= R ? (R - d) / R : 0.0;
}

// Half-width in x of the ball's row (dy, dz), rounded up (extra taps have weight 0);
// -1 if the row misses the ball.
__device__ __forceinline__ int flt_row(const FltArgs &a, int dy, int dz) {
    const double s = a.R * a.R - (double)(dy * dy + dz * dz);
    return s < 0.0 ? -1 : min(a.r, (int)sqrt(s) + 1);
}

// Fill the weight table (FP64 and working precision) and return, through wsum, the sum
// of all its weights (wave 0 reduces, fixed order).
template <int DIM, typename T>
__device__ __forceinline__ void flt_table(const FltArgs &a, double *wd, T *wt, double *wsum) {
    const int r = a.r, e = 2 * r + 1, n = DIM == 2 ? e * e : e * e * e;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        const int dx = l % e - r, dy = (l / e) % e - r, dz = DIM == 2 ? 0 : l / (e * e) - r;
        const double w = flt_w(a.R, dx, dy, dz);
        wd[l] = w;
        wt[l] = T(w);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int l = threadIdx.x; l < n; l += 64) s += wd[l];
        s = wave_sum(s);
        if (threadIdx.x == 0) *wsum = s;
    }
}

// W_i for a point whose cube reaches the grid's edge.
template <int DIM>
__device__ __forceinline__ double flt_wsum_edge(const FltArgs &a, const double *wd, int x, int y, int z) {
    const int r = a.r, e = 2 * r + 1, rz = DIM == 2 ? 0 : r;
    double s = 0.0;
    for (int dz = -rz; dz <= rz; dz++) {
        if (z + dz < 0 || z + dz >= a.n[2]) continue;
        for (int dy = -r; dy <= r; dy++) {
            if (y + dy < 0 || y + dy >= a.n[1]) continue;
            const double *row = wd + r + e * ((dy + r) + e * (dz + rz));
            for (int dx = max(-r, -x); dx <= min(r, a.n[0] - 1 - x); dx++) s += row[dx];
        }
    }
    return s;
}

template <int DIM> __device__ __forceinline__ bool flt_full(const FltArgs &a, int x, int y, int z) {
    const int r = a.r;
    return x >= r && x < a.n[0] - r && y >= r && y < a.n[1] - r && (DIM == 2 || (z >= r && z < a.n[2] - r));
}

// Weighted sum over the ball around the tile point (tx, ty, tz) of the staged tile.
template <int DIM, typename T, typename A>
__device__ __forceinline__ A flt_gather(const FltArgs &a, const T *wt, const A *tile, int hx, int hy, int tx, int ty,
                                        int tz) {
    const int r = a.r, e = 2 * r + 1, rz = DIM == 2 ? 0 : r;
    A s = 0;
    for (int dz = -rz; dz <= rz; dz++)
        for (int dy = -r; dy <= r; dy++) {
            const int xr = flt_row(a, dy, dz);
            const A *trow = tile + (tx + r) + hx * ((ty + r + dy) + hy * (DIM == 2 ? 0 : tz + r + dz));
            const T *wrow = wt + r + e * ((dy + r) + e * (dz + rz));
            for (int dx = -xr; dx <= xr; dx++) s += A(wrow[dx]) * trow[dx];
        }
    return s;
}

template <int DIM> __device__ __forceinline__ void flt_tile_origin(int o[3]) {
    o[0] = blockIdx.x * Flt<DIM>::TX;
    o[1] = blockIdx.y * Flt<DIM>::TY;
    o[2] = blockIdx.z * Flt<DIM>::TZ;
}

template <int DIM>
__device__ __forceinline__ bool flt_halo_point(const FltArgs &a, const int o[3], int l, int hx, int hy, int &x, int &y,
                                               int &z) {
    x = o[0] - a.r + l % hx;
    y = o[1] - a.r + (l / hx) % hy;
    z = DIM == 2 ? 0 : o[2] - a.r + l / (hx * hy);
    return x >= 0 && x < a.n[0] && y >= 0 && y < a.n[1] && z >= 0 && z < a.n[2];
}

// Forward: filter and project, in working precision T (weights and W_i from FP64).
template <int DIM, typename T>
__global__ __launch_bounds__(Flt<DIM>::NT) void k_filter_fwd(FltArgs a, const T *__restrict__ g,
                                                            T *__restrict__ gt, T *__restrict__ gh) {
    using F = Flt<DIM>;
    __shared__ double wd[F::WN];
    __shared__ T wt[F::WN];
    __shared__ T tile[F::HN];
    __shared__ double wfull;
    int o[3];
    flt_tile_origin<DIM>(o);
    const int hx = F::TX + 2 * a.r, hy = F::TY + 2 * a.r, hz = DIM == 2 ? 1 : F::TZ + 2 * a.r;
    for (int l = threadIdx.x; l < hx * hy * hz; l += F::NT) {
        int x, y, z;
        const bool in = flt_halo_point<DIM>(a, o, l, hx, hy, x, y, z);
        tile[l] = in ? g[x + (long long)a.n[0] * (y + (long long)a.n[1] * z)] : T(0);
    }
    flt_table<DIM>(a, wd, wt, &wfull);
    __syncthreads();
    const int tx = threadIdx.x % F::TX, ty = (threadIdx.x / F::TX) % F::TY, tz = threadIdx.x / (F::TX * F::TY);
    const int x = o[0] + tx, y = o[1] + ty, z = o[2] + tz;
    if (x < a.n[0] && y < a.n[1] && z < a.n[2]) {
        const T num = flt_gather<DIM, T, T>(a, wt, tile, hx, hy, tx, ty, tz);
        const double W = flt_full<DIM>(a, x, y, z) ? wfull : flt_wsum_edge<DIM>(a, wd, x, y, z);
        const T v = num / T(W);
        const long long id = x + (long long)a.n[0] * (y + (long long)a.n[1] * z);
        gt[id] = v;
        const T be = T(a.beta), et = T(a.eta);
        gh[id] = (tanh(be * et) + tanh(be * (v - et))) / (tanh(be * et) + tanh(be * (T(1) - et)));
    }
}

// Reverse, FP64: t_i on the tile and its halo (zero off the grid), then the gather.
template <int DIM, typename T>
__global__ __launch_bounds__(Flt<DIM>::NT) void k_filter_adj(FltArgs a, const T *__restrict__ gt,
                                                            const double *__restrict__ gbh,
                                                            double *__restrict__ gb) {
    using F = Flt<DIM>;
    __shared__ double wd[F::WN];
    __shared__ double tile[F::HN];
    __shared__ double wfull;
    int o[3];
    flt_tile_origin<DIM>(o);
    flt_table<DIM>(a, wd, wd, &wfull);
    __syncthreads();
    const double den = tanh(a.beta * a.eta) + tanh(a.beta * (1.0 - a.eta));
    const int hx = F::TX + 2 * a.r, hy = F::TY + 2 * a.r, hz = DIM == 2 ? 1 : F::TZ + 2 * a.r;
    for (int l = threadIdx.x; l < hx * hy * hz; l += F::NT) {
        int x, y, z;
        double t = 0.0;
        if (flt_halo_point<DIM>(a, o, l, hx, hy, x, y, z)) {
            const long long id = x + (long long)a.n[0] * (y + (long long)a.n[1] * z);
            const double W = flt_full<DIM>(a, x, y, z) ? wfull : flt_wsum_edge<DIM>(a, wd, x, y, z);
            const double th = tanh(a.beta * ((double)gt[id] - a.eta));
            t = gbh[id] * (a.beta * (1.0 - th * th) / den) / W;
        }
        tile[l] = t;
    }
    __syncthreads();
    const int tx = threadIdx.x % F::TX, ty = (threadIdx.x / F::TX) % F::TY, tz = threadIdx.x / (F::TX * F::TY);
    const int x = o[0] + tx, y = o[1] + ty, z = o[2] + tz;
    if (x < a.n[0] && y < a.n[1] && z < a.n[2])
        gb[x + (long long)a.n[0] * (y + (long long)a.n[1] * z)] = flt_gather<DIM, double, double>(a, wd, tile, hx, hy, tx, ty, tz);
}

}  // namespace lks
