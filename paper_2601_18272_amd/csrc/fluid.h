// fluid.h -- lattice kinetic scheme on the analysis grid (gfx950).
//
// Forward (Sec. 2.2): with tau = 1 the post-streaming moments of node x are
//   p*(x) = 1/3 sum_i f_i(x - c_i),   u*(x) = sum_i c_i f_i(x - c_i),
//   f_i = w_i (3p + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) + w_i A sum_ab (d_a u_b + d_b u_a) c_a c_b
// (Eqs. local_equilibrium_function, p_tmp, u_tmp; the -3/2 sign is the reading of the
// printed +3/2). Gradients: central differences, second-order one-sided along the
// normal on boundary nodes of non-periodic faces.
//
// Adjoint: the exact transpose. With g_i(x) = p*bar(x)/3 + c_i . u*bar(x) on interior
// nodes, the moments pi = sum_i w_i g_i(y + c_i), ups_a = sum_i w_i c_ia g_i(y + c_i),
// sig_ab = sum_i w_i c_ia c_ib g_i(y + c_i) (the ALKS moments p~, u~, s~ of Eqs.
// ap_tmp..as_tmp) give
//   pbar(y) = 3 pi,  ubar_b(y) = 3 ups_b + 9 sig_ba u_a - 3 pi u_b + 2A sum_a D_a^T sig_ab,
// with D_a^T the transpose of the boundary-aware difference operator.
#pragma once
#include "lks_device.h"

namespace lks {

// ===================================================================== forward, 2D
// 64 x 8 tile, one node per thread. Push form: every source node of the tile plus a
// one-node ring evaluates its nine f_i once into LDS; each node then gathers the nine
// values that stream into it. p, u are staged with a two-node ring (gradients of the
// ring nodes).
constexpr int G2_TX = 64, G2_TY = 8;

template <typename T>
__global__ __launch_bounds__(512) void k_gather2d(Grid g, T A, const T *__restrict__ sin_,
                                                  T *__restrict__ sout) {
    constexpr int RX = G2_TX + 4, RY = G2_TY + 4;  // p, u with a 2-ring
    constexpr int FX = G2_TX + 2, FY = G2_TY + 2;  // f with a 1-ring
    __shared__ T sp[RY][RX], sux[RY][RX], suy[RY][RX];
    __shared__ T sf[9][FY][FX];
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1];
    const int x0 = blockIdx.x * G2_TX, y0 = blockIdx.y * G2_TY;
    const int tid = threadIdx.x + G2_TX * threadIdx.y;

    for (int l = tid; l < RX * RY; l += 512) {
        const int lx = l % RX, ly = l / RX;
        int x = x0 + lx - 2, y = y0 + ly - 2;
        T vp = 0, vx = 0, vy = 0;
        if (wrap_coord(x, nx, g.per[0]) && wrap_coord(y, ny, g.per[1])) {
            const long long id = (long long)x + (long long)nx * y;
            vp = sin_[id];
            vx = sin_[N + id];
            vy = sin_[2 * N + id];
        }
        sp[ly][lx] = vp;
        sux[ly][lx] = vx;
        suy[ly][lx] = vy;
    }
    __syncthreads();

    const T w0 = T(4.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
    for (int l = tid; l < FX * FY; l += 512) {
        const int fx = l % FX, fy = l / FX;
        const int lx = fx + 1, ly = fy + 1;  // position in the 2-ring arrays
        int x = x0 + fx - 1, y = y0 + fy - 1;
        const bool ok = wrap_coord(x, nx, g.per[0]) && wrap_coord(y, ny, g.per[1]);
        T f[9];
        if (ok) {
            // S_ab = d_a u_b
            T dxux, dxuy, dyux, dyuy;
            if (g.per[0] || (x > 0 && x < nx - 1)) {
                dxux = T(0.5) * (sux[ly][lx + 1] - sux[ly][lx - 1]);
                dxuy = T(0.5) * (suy[ly][lx + 1] - suy[ly][lx - 1]);
            } else if (x == 0) {
                dxux = T(0.5) * (T(-3) * sux[ly][lx] + T(4) * sux[ly][lx + 1] - sux[ly][lx + 2]);
                dxuy = T(0.5) * (T(-3) * suy[ly][lx] + T(4) * suy[ly][lx + 1] - suy[ly][lx + 2]);
            } else {
                dxux = T(0.5) * (T(3) * sux[ly][lx] - T(4) * sux[ly][lx - 1] + sux[ly][lx - 2]);
                dxuy = T(0.5) * (T(3) * suy[ly][lx] - T(4) * suy[ly][lx - 1] + suy[ly][lx - 2]);
            }
            if (g.per[1] || (y > 0 && y < ny - 1)) {
                dyux = T(0.5) * (sux[ly + 1][lx] - sux[ly - 1][lx]);
                dyuy = T(0.5) * (suy[ly + 1][lx] - suy[ly - 1][lx]);
            } else if (y == 0) {
                dyux = T(0.5) * (T(-3) * sux[ly][lx] + T(4) * sux[ly + 1][lx] - sux[ly + 2][lx]);
                dyuy = T(0.5) * (T(-3) * suy[ly][lx] + T(4) * suy[ly + 1][lx] - suy[ly + 2][lx]);
            } else {
                dyux = T(0.5) * (T(3) * sux[ly][lx] - T(4) * sux[ly - 1][lx] + sux[ly - 2][lx]);
                dyuy = T(0.5) * (T(3) * suy[ly][lx] - T(4) * suy[ly - 1][lx] + suy[ly - 2][lx]);
            }
            const T p = sp[ly][lx], ux = sux[ly][lx], uy = suy[ly][lx];
            // f_i = w_i (3p - 3/2 u.u + 3 c.u + 9/2 (c.u)^2 + A c.(S + S^T).c)
            const T base = T(3) * p - T(1.5) * (ux * ux + uy * uy);
            const T axx = T(2) * A * dxux, ayy = T(2) * A * dyuy, axy = T(2) * A * (dxuy + dyux);
            f[0] = w0 * base;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                const int cx = Lat<2>::c(i, 0), cy = Lat<2>::c(i, 1);
                const T cu = T(cx) * ux + T(cy) * uy;
                const T an = T(cx * cx) * axx + T(cy * cy) * ayy + T(cx * cy) * axy;
                f[i] = (i < 5 ? w1 : w2) * (base + T(3) * cu + T(4.5) * cu * cu + an);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; i++) f[i] = 0;
        }
#pragma unroll
        for (int i = 0; i < 9; i++) sf[i][fy][fx] = f[i];
    }
    __syncthreads();

    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    if ((!g.per[0] && (x == 0 || x == nx - 1)) || (!g.per[1] && (y == 0 || y == ny - 1))) return;
    T ps = 0, usx = 0, usy = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const int cx = Lat<2>::c(i, 0), cy = Lat<2>::c(i, 1);
        const T f = sf[i][threadIdx.y + 1 - cy][threadIdx.x + 1 - cx];
        ps += f;
        usx += T(cx) * f;
        usy += T(cy) * f;
    }
    const long long id = (long long)x + (long long)nx * y;
    sout[id] = ps * T(1.0 / 3.0);
    sout[N + id] = usx;
    sout[2 * N + id] = usy;
}

// ===================================================================== forward, 3D
// First version: one node per thread, f_i(x - c_i) evaluated from global loads
// (the neighbourhood is L1/L2 resident).
template <typename T>
__device__ __forceinline__ T ld(const T *__restrict__ a, long long i) {
    return a[i];
}

template <typename T>
__device__ __forceinline__ void grad3(const Grid &g, const T *__restrict__ u, const int y[3], T S[3][3]) {
    const long long N = g.N;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        T cf[3];
        int cnt;
        const int n = g.n[a];
        int ya = y[a];
        int o[3];
        if (g.per[a] || (ya > 0 && ya < n - 1)) {
            o[0] = ya + 1;
            o[1] = ya - 1;
            cf[0] = T(0.5);
            cf[1] = T(-0.5);
            cnt = 2;
            if (g.per[a]) {
                if (o[0] >= n) o[0] -= n;
                if (o[1] < 0) o[1] += n;
            }
        } else if (ya == 0) {
            o[0] = 0;
            o[1] = 1;
            o[2] = 2;
            cf[0] = T(-1.5);
            cf[1] = T(2);
            cf[2] = T(-0.5);
            cnt = 3;
        } else {
            o[0] = n - 1;
            o[1] = n - 2;
            o[2] = n - 3;
            cf[0] = T(1.5);
            cf[1] = T(-2);
            cf[2] = T(0.5);
            cnt = 3;
        }
        T acc[3] = {0, 0, 0};
        for (int j = 0; j < cnt; j++) {
            int z[3] = {y[0], y[1], y[2]};
            z[a] = o[j];
            const long long id = node_id(g, z[0], z[1], z[2]);
#pragma unroll
            for (int b = 0; b < 3; b++) acc[b] += cf[j] * ld(u, b * N + id);
        }
#pragma unroll
        for (int b = 0; b < 3; b++) S[a][b] = acc[b];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather3d(Grid g, T A, const T *__restrict__ sin_,
                                                  T *__restrict__ sout) {
    const long long N = g.N;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    int x[3];
    x[0] = (int)(id % g.n[0]);
    x[1] = (int)((id / g.n[0]) % g.n[1]);
    x[2] = (int)(id / ((long long)g.n[0] * g.n[1]));
    if (!is_interior<3>(g, x)) return;
    const T *u = sin_ + N;
    T ps = 0, us[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < 15; i++) {
        int y[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            y[a] = x[a] - Lat<3>::c(i, a);
            wrap_coord(y[a], g.n[a], g.per[a]);
        }
        const long long yi = node_id(g, y[0], y[1], y[2]);
        const T p = sin_[yi];
        T uy[3];
#pragma unroll
        for (int a = 0; a < 3; a++) uy[a] = u[a * N + yi];
        T S[3][3];
        grad3<T>(g, u, y, S);
        T cu = 0, uu = 0, an = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cu += T(Lat<3>::c(i, a)) * uy[a];
            uu += uy[a] * uy[a];
        }
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                an += T(Lat<3>::c(i, a) * Lat<3>::c(i, b)) * (S[a][b] + S[b][a]);
        const T f = T(Lat<3>::w(i)) * (T(3) * p + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu + A * an);
        ps += f;
#pragma unroll
        for (int a = 0; a < 3; a++) us[a] += T(Lat<3>::c(i, a)) * f;
    }
    sout[id] = ps * T(1.0 / 3.0);
#pragma unroll
    for (int a = 0; a < 3; a++) sout[(1 + a) * N + id] = us[a];
}

// ===================================================================== boundary values
// One thread per node of every non-periodic face; edge nodes are visited by several
// faces and write the same value. Copies read interior nodes only.
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_bc(Grid g, Bc bc, T *__restrict__ s, int face_axes,
                                            long long face_total) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= face_total) return;
    // locate the face: faces are enumerated axis by axis (low then high side)
    long long rem = t;
    int x[3] = {0, 0, 0};
    bool found = false;
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        if (found || !(face_axes & (1 << a))) continue;
        const long long fsz = g.N / g.n[a];
        if (rem < 2 * fsz) {
            const int side = rem >= fsz;
            long long k = rem - side * fsz;
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const int nb = g.n[b];
            x[a] = side ? g.n[a] - 1 : 0;
            x[b] = (int)(k % nb);
            x[c] = (int)(k / nb);
            found = true;
        } else {
            rem -= 2 * fsz;
        }
    }
    if (!found) return;
    BcNode r;
    bc_resolve<DIM>(g, bc, x, r);
    const long long N = g.N;
    const long long id = node_id(g, x[0], x[1], x[2]);
    const long long in = node_id(g, r.in[0], r.in[1], r.in[2]);
    s[id] = r.p_fixed ? T(r.p) : s[in];
#pragma unroll
    for (int a = 0; a < DIM; a++) s[(1 + a) * N + id] = r.u_fixed ? T(r.u[a]) : s[(1 + a) * N + in];
}

// ===================================================================== adjoint helpers
// Cotangent that reaches interior node x from the state at t: its own entry plus the
// entries of the boundary nodes that copy x (transpose of the boundary treatment).
template <int DIM, typename T>
__device__ __forceinline__ void fold_bc(const Grid &g, const Bc &bc, const T *__restrict__ ab,
                                        const int x[3], long long id, T &pb, T ub[3], bool want_u) {
    const long long N = g.N;
    pb = ab[id];
#pragma unroll
    for (int a = 0; a < 3; a++) ub[a] = (a < DIM && want_u) ? ab[(1 + a) * N + id] : T(0);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool any = false;
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        if (g.per[a]) continue;
        if (x[a] == 1) {
            lo[a] = -1;
            any = true;
        }
        if (x[a] == g.n[a] - 2) {
            hi[a] = 1;
            any = true;
        }
    }
    if (!any) return;
    for (int dz = lo[2]; dz <= hi[2]; dz++)
        for (int dy = lo[1]; dy <= hi[1]; dy++)
            for (int dx = lo[0]; dx <= hi[0]; dx++) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                // only offsets that land on the boundary along each shifted axis
                const int d[3] = {dx, dy, dz};
                int b[3];
                bool ok = true;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    b[a] = x[a] + d[a];
                    if (d[a] != 0 && !(b[a] == 0 || b[a] == g.n[a] - 1)) ok = false;
                }
                if (!ok) continue;
                BcNode r;
                bc_resolve<DIM>(g, bc, b, r);
                if (r.in[0] != x[0] || r.in[1] != x[1] || r.in[2] != x[2]) continue;
                const long long bi = node_id(g, b[0], b[1], b[2]);
                if (!r.p_fixed) pb += ab[bi];
                if (want_u && !r.u_fixed)
#pragma unroll
                    for (int a = 0; a < DIM; a++) ub[a] += ab[(1 + a) * N + bi];
            }
}

// Coefficients with which sig(y), y = z + off * e_a, enters D_a^T sig at node z.
// Returns the number of (off, coef) pairs (at most 5).
template <typename T>
__device__ __forceinline__ int dT_stencil(int za, int n, int per, int off[5], T coef[5]) {
    int k = 0;
    if (per) {
        off[k] = -1;
        coef[k++] = T(0.5);
        off[k] = 1;
        coef[k++] = T(-0.5);
        return k;
    }
    // y = z - e (central unless on the low boundary)
    if (za - 1 >= 0) {
        off[k] = -1;
        coef[k++] = (za - 1 == 0) ? T(2) : T(0.5);
    }
    // y = z + e (central unless on the high boundary)
    if (za + 1 <= n - 1) {
        off[k] = 1;
        coef[k++] = (za + 1 == n - 1) ? T(-2) : T(-0.5);
    }
    if (za == 0) {
        off[k] = 0;
        coef[k++] = T(-1.5);
    }
    if (za == n - 1) {
        off[k] = 0;
        coef[k++] = T(1.5);
    }
    if (za - 2 == 0) {
        off[k] = -2;
        coef[k++] = T(-0.5);
    }
    if (za + 2 == n - 1) {
        off[k] = 2;
        coef[k++] = T(0.5);
    }
    return k;
}

struct Box {
    int o[3];
    int L[3];
};

template <int DIM>
__device__ __forceinline__ long long box_index(const Box &bx, const int x[3]) {
    long long l = 0;
#pragma unroll
    for (int a = DIM - 1; a >= 0; a--) {
        const int v = x[a] - bx.o[a];
        if (v < 0 || v >= bx.L[a]) return -1;
        l = l * bx.L[a] + v;
    }
    return l;
}

// p*bar, u*bar at interior node x (the cotangents of the post-streaming moments).
template <int DIM, typename T>
__device__ __forceinline__ void star_bar(const Grid &g, const Bc &bc, const T *__restrict__ ab,
                                         const T *__restrict__ ustb, const Box &bx, bool has_box,
                                         long long boxN, const int x[3], long long id, T &pb, T ub[3]) {
    const long long bi = has_box ? box_index<DIM>(bx, x) : -1;
    fold_bc<DIM, T>(g, bc, ab, x, id, pb, ub, bi < 0);
    if (bi >= 0)
#pragma unroll
        for (int a = 0; a < DIM; a++) ub[a] = ustb[a * boxN + bi];
}

// ===================================================================== adjoint, 2D
// 64 x 8 tile. Stage p*bar, u*bar with a 3-node ring (zero off the interior), form
// the moments (pi, ups, sig) on the tile plus a 2-ring, then the outputs.
template <typename T>
__global__ __launch_bounds__(512) void k_adjgather2d(Grid g, Bc bc, T A, const T *__restrict__ ab,
                                                     const T *__restrict__ ustb, const double *__restrict__ Bprev,
                                                     Design D, int has_box, const T *__restrict__ sprev,
                                                     T *__restrict__ out) {
    constexpr int RX = G2_TX + 6, RY = G2_TY + 6;
    constexpr int MX = G2_TX + 4, MY = G2_TY + 4;
    __shared__ T sP[RY][RX], sU[RY][RX], sV[RY][RX];
    __shared__ T mpi[MY][MX], mux[MY][MX], muy[MY][MX], mxx[MY][MX], myy[MY][MX], mxy[MY][MX];
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1];
    const int x0 = blockIdx.x * G2_TX, y0 = blockIdx.y * G2_TY;
    const int tid = threadIdx.x + G2_TX * threadIdx.y;
    Box bx;
    if (has_box) {
        box_origin<2>(D, Bprev, bx.o);
        bx.L[0] = D.L[0];
        bx.L[1] = D.L[1];
        bx.L[2] = 1;
    }
    for (int l = tid; l < RX * RY; l += 512) {
        const int lx = l % RX, ly = l / RX;
        int xx[3] = {x0 + lx - 3, y0 + ly - 3, 0};
        T vp = 0, vu = 0, vv = 0;
        if (wrap_coord(xx[0], nx, g.per[0]) && wrap_coord(xx[1], ny, g.per[1]) && is_interior<2>(g, xx)) {
            const long long id = (long long)xx[0] + (long long)nx * xx[1];
            T ub[3];
            star_bar<2, T>(g, bc, ab, ustb, bx, has_box, D.boxN, xx, id, vp, ub);
            vu = ub[0];
            vv = ub[1];
        }
        sP[ly][lx] = vp * T(1.0 / 3.0);
        sU[ly][lx] = vu;
        sV[ly][lx] = vv;
    }
    __syncthreads();
    for (int l = tid; l < MX * MY; l += 512) {
        const int mx = l % MX, my = l / MX;
        const int lx = mx + 1, ly = my + 1;  // in the 3-ring arrays
        T pi = 0, ux = 0, uy = 0, sxx = 0, syy = 0, sxy = 0;
#pragma unroll
        for (int i = 0; i < 9; i++) {
            const int cx = Lat<2>::c(i, 0), cy = Lat<2>::c(i, 1);
            const T gi = sP[ly + cy][lx + cx] + T(cx) * sU[ly + cy][lx + cx] + T(cy) * sV[ly + cy][lx + cx];
            const T wg = T(Lat<2>::w(i)) * gi;
            pi += wg;
            ux += T(cx) * wg;
            uy += T(cy) * wg;
            sxx += T(cx * cx) * wg;
            syy += T(cy * cy) * wg;
            sxy += T(cx * cy) * wg;
        }
        mpi[my][mx] = pi;
        mux[my][mx] = ux;
        muy[my][mx] = uy;
        mxx[my][mx] = sxx;
        myy[my][mx] = syy;
        mxy[my][mx] = sxy;
    }
    __syncthreads();
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int mx = threadIdx.x + 2, my = threadIdx.y + 2;
    const long long id = (long long)x + (long long)nx * y;
    const T u0 = sprev[N + id], u1 = sprev[2 * N + id];
    const T pi = mpi[my][mx];
    T ox = T(3) * mux[my][mx] + T(9) * (mxx[my][mx] * u0 + mxy[my][mx] * u1) - T(3) * pi * u0;
    T oy = T(3) * muy[my][mx] + T(9) * (mxy[my][mx] * u0 + myy[my][mx] * u1) - T(3) * pi * u1;
    int off[5];
    T cf[5];
    const T A2 = T(2) * A;
    int k = dT_stencil<T>(x, nx, g.per[0], off, cf);
    for (int j = 0; j < k; j++) {  // a = x: sig_xx -> u_x, sig_xy -> u_y
        ox += A2 * cf[j] * mxx[my][mx + off[j]];
        oy += A2 * cf[j] * mxy[my][mx + off[j]];
    }
    k = dT_stencil<T>(y, ny, g.per[1], off, cf);
    for (int j = 0; j < k; j++) {  // a = y: sig_yx -> u_x, sig_yy -> u_y
        ox += A2 * cf[j] * mxy[my + off[j]][mx];
        oy += A2 * cf[j] * myy[my + off[j]][mx];
    }
    out[id] = T(3) * pi;
    out[N + id] = ox;
    out[2 * N + id] = oy;
}

// ===================================================================== adjoint, 3D
// First version, two passes through global memory: moments (pi, ups[3], sig[6]) of
// every node into `mom` (10 x N), then the outputs.
template <typename T>
__global__ __launch_bounds__(256) void k_adjmom3d(Grid g, Bc bc, const T *__restrict__ ab,
                                                  const T *__restrict__ ustb, const double *__restrict__ Bprev,
                                                  Design D, int has_box, T *__restrict__ mom) {
    const long long N = g.N;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    int y[3];
    y[0] = (int)(id % g.n[0]);
    y[1] = (int)((id / g.n[0]) % g.n[1]);
    y[2] = (int)(id / ((long long)g.n[0] * g.n[1]));
    Box bx;
    if (has_box) {
        box_origin<3>(D, Bprev, bx.o);
        bx.L[0] = D.L[0];
        bx.L[1] = D.L[1];
        bx.L[2] = D.L[2];
    }
    T m[10];
#pragma unroll
    for (int j = 0; j < 10; j++) m[j] = 0;
    for (int i = 0; i < 15; i++) {
        int z[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            z[a] = y[a] + Lat<3>::c(i, a);
            ok = ok && wrap_coord(z[a], g.n[a], g.per[a]);
        }
        if (!ok || !is_interior<3>(g, z)) continue;
        const long long zi = node_id(g, z[0], z[1], z[2]);
        T pb, ub[3];
        star_bar<3, T>(g, bc, ab, ustb, bx, has_box, D.boxN, z, zi, pb, ub);
        T gi = pb * T(1.0 / 3.0);
#pragma unroll
        for (int a = 0; a < 3; a++) gi += T(Lat<3>::c(i, a)) * ub[a];
        const T wg = T(Lat<3>::w(i)) * gi;
        const int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
        m[0] += wg;
        m[1] += T(cx) * wg;
        m[2] += T(cy) * wg;
        m[3] += T(cz) * wg;
        m[4] += T(cx * cx) * wg;  // xx
        m[5] += T(cy * cy) * wg;  // yy
        m[6] += T(cz * cz) * wg;  // zz
        m[7] += T(cx * cy) * wg;  // xy
        m[8] += T(cx * cz) * wg;  // xz
        m[9] += T(cy * cz) * wg;  // yz
    }
#pragma unroll
    for (int j = 0; j < 10; j++) mom[j * N + id] = m[j];
}

__device__ __forceinline__ int sig_index(int a, int b) {
    // symmetric index into mom[4..9]
    if (a == b) return 4 + a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 7 : 8) : 9;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adjout3d(Grid g, T A, const T *__restrict__ mom,
                                                  const T *__restrict__ sprev, T *__restrict__ out) {
    const long long N = g.N;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    int z[3];
    z[0] = (int)(id % g.n[0]);
    z[1] = (int)((id / g.n[0]) % g.n[1]);
    z[2] = (int)(id / ((long long)g.n[0] * g.n[1]));
    T u[3];
#pragma unroll
    for (int a = 0; a < 3; a++) u[a] = sprev[(1 + a) * N + id];
    const T pi = mom[id];
    T o[3];
#pragma unroll
    for (int b = 0; b < 3; b++) {
        T v = T(3) * mom[(1 + b) * N + id] - T(3) * pi * u[b];
#pragma unroll
        for (int a = 0; a < 3; a++) v += T(9) * mom[sig_index(b, a) * N + id] * u[a];
        o[b] = v;
    }
    const T A2 = T(2) * A;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        int off[5];
        T cf[5];
        const int k = dT_stencil<T>(z[a], g.n[a], g.per[a], off, cf);
        for (int j = 0; j < k; j++) {
            int y[3] = {z[0], z[1], z[2]};
            y[a] += off[j];
            wrap_coord(y[a], g.n[a], g.per[a]);
            const long long yi = node_id(g, y[0], y[1], y[2]);
#pragma unroll
            for (int b = 0; b < 3; b++) o[b] += A2 * cf[j] * mom[sig_index(a, b) * N + yi];
        }
    }
    out[id] = T(3) * pi;
#pragma unroll
    for (int b = 0; b < 3; b++) out[(1 + b) * N + id] = o[b];
}

}  // namespace lks
