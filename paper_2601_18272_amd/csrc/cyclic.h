// cyclic.h -- cyclic periodic design (Sec. 4.2): the design variables live on one sector
// and are repeated by the rotations about the rotation axis through the design grid's
// centre; the sensitivities on the design grid are collected back onto the sector.
//
// Plane coordinates (u, v) run along the rotation plane's axes (pi, pj), w along the
// axis. Groups that map a Cartesian grid onto itself: n = 1; n = 2 (half turn,
// (u, v) -> (nu-1-u, nv-1-v), plane index q -> nu nv - 1 - q); n = 4 on a square plane
// of side s (quarter turn R(u, v) = (s-1-v, u)). The sector:
//   n = 1: the plane;  n = 2: plane indices q <= nu nv - 1 - q, index q;
//   n = 4: the pinwheel F = {u < ceil(s/2), v < floor(s/2)}, index u + ceil(s/2) v, and
//          for odd s the centre as the last index. R, R^2, R^3 map F onto
//          A1 = {u >= ceil, v < ceil}, A2 = {u >= floor, v >= ceil}, A3 = {u < floor, v >= floor}.
// Sector index = plane sector index + (plane sector size) w.
#pragma once
#include "lks_device.h"

namespace lks {

struct CycArgs {
    int nd[3];
    int pi, pj, ax;  // rotation plane axes and rotation axis
    int n_sec;
    long long sector_plane;  // sector points per plane
};

__host__ __device__ inline long long cyc_sector_plane(int nu, int nv, int n_sec) {
    if (n_sec == 1) return (long long)nu * nv;
    if (n_sec == 2) return ((long long)nu * nv + 1) / 2;
    if (n_sec == 4 && nu == nv) return (long long)((nu + 1) / 2) * (nu / 2) + (nu % 2);
    return -1;
}

// Plane sector index of the orbit of (u, v).
__device__ __forceinline__ long long cyc_rep(const CycArgs &a, int u, int v) {
    const int nu = a.nd[a.pi], nv = a.nd[a.pj];
    if (a.n_sec == 1) return u + (long long)nu * v;
    if (a.n_sec == 2) {
        const long long q = u + (long long)nu * v, r = (long long)nu * nv - 1 - q;
        return q < r ? q : r;
    }
    const int s = nu, cu = (s + 1) / 2, cv = s / 2;
    int u0 = u, v0 = v;                              // F
    if (u >= cu && v < cu) u0 = v, v0 = s - 1 - u;   // A1 = R F
    else if (u >= cv && v >= cu) u0 = s - 1 - u, v0 = s - 1 - v;  // A2 = R^2 F
    else if (u < cv && v >= cv) u0 = s - 1 - v, v0 = u;           // A3 = R^3 F
    else if (u >= cu || v >= cv) return (long long)cu * cv;       // the centre (odd s)
    return u0 + (long long)cu * v0;
}

// Expansion: gamma[m] = gamma_sector[sector index of m], one thread per design point.
template <typename T>
__global__ __launch_bounds__(256) void k_cyc_expand(CycArgs a, const T *__restrict__ gs, T *__restrict__ g) {
    const long long nd = (long long)a.nd[0] * a.nd[1] * a.nd[2];
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nd) return;
    const int c[3] = {(int)(m % a.nd[0]), (int)((m / a.nd[0]) % a.nd[1]), (int)(m / ((long long)a.nd[0] * a.nd[1]))};
    g[m] = gs[cyc_rep(a, c[a.pi], c[a.pj]) + a.sector_plane * c[a.ax]];
}

// Collection (FP64): each sector point sums the sensitivities of its orbit in the order
// of the group's powers (R^0, R^1, ...), fixed points once. One thread per sector point.
__global__ __launch_bounds__(256) void k_cyc_collect(CycArgs a, const double *__restrict__ grad,
                                                    double *__restrict__ gs) {
    const long long ns = a.sector_plane * a.nd[a.ax];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int nu = a.nd[a.pi], nv = a.nd[a.pj];
    const long long sp = s % a.sector_plane;
    const int w = (int)(s / a.sector_plane);
    // the sector point's plane coordinates
    int u0, v0;
    if (a.n_sec == 4) {
        const int cu = (nu + 1) / 2, cv = nu / 2;
        if (sp == (long long)cu * cv) u0 = v0 = nu / 2;  // centre
        else u0 = (int)(sp % cu), v0 = (int)(sp / cu);
    } else {
        u0 = (int)(sp % nu), v0 = (int)(sp / nu);
    }
    int mu[4] = {u0, 0, 0, 0}, mv[4] = {v0, 0, 0, 0}, nm = 1;
    if (a.n_sec == 2) {
        mu[1] = nu - 1 - u0, mv[1] = nv - 1 - v0;
        nm = (mu[1] == u0 && mv[1] == v0) ? 1 : 2;
    } else if (a.n_sec == 4) {
        const int s1 = nu - 1;
        mu[1] = s1 - v0, mv[1] = u0;
        mu[2] = s1 - u0, mv[2] = s1 - v0;
        mu[3] = v0, mv[3] = s1 - u0;
        nm = (mu[1] == u0 && mv[1] == v0) ? 1 : 4;
    }
    double sum = 0.0;
    for (int k = 0; k < nm; k++) {
        int c[3];
        c[a.pi] = mu[k];
        c[a.pj] = mv[k];
        c[a.ax] = w;
        sum += grad[c[0] + (long long)a.nd[0] * (c[1] + (long long)a.nd[1] * c[2])];
    }
    gs[s] = sum;
}

}  // namespace lks
