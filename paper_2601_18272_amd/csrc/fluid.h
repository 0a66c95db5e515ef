// fluid.h -- lattice kinetic scheme on the analysis grid (gfx950).
//
// Forward (Sec. 2.2): with tau = 1 the post-streaming moments of node x are
//   p*(x) = 1/3 sum_i f_i(x - c_i),   u*(x) = sum_i c_i f_i(x - c_i),
//   f_i = w_i (3p + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) + w_i A sum_ab (d_a u_b + d_b u_a) c_a c_b
// (Eqs. local_equilibrium_function, p_tmp, u_tmp; the -3/2 sign is the reading of the
// printed +3/2). Gradients: central differences, second-order one-sided along the
// normal on boundary nodes of non-periodic faces.
//
// The state holds v = u - U (Grid::U). The equilibrium of the uniform flow,
// f_i^U = w_i (3 c.U + 9/2 (c.U)^2 - 3/2 U.U), satisfies sum_i f_i^U = 0 and
// sum_i c_i f_i^U = U, so with df_i = f_i - f_i^U,
//   df_i = w_i (3p + 3 c.v + 9 (c.U)(c.v) + 9/2 (c.v)^2 - 3 U.v - 3/2 v.v) + w_i A (...),
//   p* = 1/3 sum_i df_i(x - c_i),   v* = sum_i c_i df_i(x - c_i),
// the same update with every term small (the gradients of u and v are equal).
//
// Adjoint: the exact transpose. With g_i(x) = p*bar(x)/3 + c_i . u*bar(x) on interior
// nodes, the moments pi = sum_i w_i g_i(y + c_i), ups_a = sum_i w_i c_ia g_i(y + c_i),
// sig_ab = sum_i w_i c_ia c_ib g_i(y + c_i) (the ALKS moments p~, u~, s~ of Eqs.
// ap_tmp..as_tmp) give
//   pbar(y) = 3 pi,  ubar_b(y) = 3 ups_b + 9 sig_ba u_a - 3 pi u_b + 2A sum_a D_a^T sig_ab,
// with D_a^T the transpose of the boundary-aware difference operator and u = U + v the
// forward velocity. The cotangents of u and of v = u - U are the same.
#pragma once
#include <type_traits>

#include "lks_device.h"

namespace lks {

// ===================================================================== forward, 2D
// 64 x 8 tile, one node per thread. Push form: every source node of the tile plus a
// one-node ring evaluates its nine f_i once into LDS; each node then gathers the nine
// values that stream into it. p, u are staged with a two-node ring (gradients of the
// ring nodes).
constexpr int G2_TX = 64, G2_TY = 8;

// With fold, the boundary nodes of sin_ are not read: their values are formed on load
// from the interior node they copy (bc_resolve), as k_bc would have stored them, so the
// forward step needs no separate boundary launch.
template <typename T, bool SP>
__global__ __launch_bounds__(512) void k_gather2d(Grid g, T A, Bc bc, int fold, const T *__restrict__ sin_,
                                                  T *__restrict__ sout, unsigned long long *ts) {
    constexpr int RX = G2_TX + 4, RY = G2_TY + 4;  // p, u with a 2-ring
    constexpr int FX = G2_TX + 2, FY = G2_TY + 2;  // f with a 1-ring
    __shared__ T sp[RY][RX], sux[RY][RX], suy[RY][RX];
    __shared__ T sf[9][FY][FX];
    if (SP) span_begin(ts);
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1];
    const uint3 tb = xcd_tile();
    const int x0 = tb.x * G2_TX, y0 = tb.y * G2_TY;
    const int tid = threadIdx.x + G2_TX * threadIdx.y;

    for (int l = tid; l < RX * RY; l += 512) {
        const int lx = l % RX, ly = l / RX;
        int x = x0 + lx - 2, y = y0 + ly - 2;
        T vp = 0, vx = 0, vy = 0;
        if (wrap_coord(x, nx, g.per[0]) && wrap_coord(y, ny, g.per[1])) {
            // the node itself, or with fold for a boundary node the interior node it
            // copies; the three loads are issued the same way for every node, the
            // prescribed values replace them afterwards
            int sx = x, sy = y;
            bool pfix = false, ufix = false;
            T pv = 0, uxv = 0, uyv = 0;
            if (fold && ((!g.per[0] && (x == 0 || x == nx - 1)) || (!g.per[1] && (y == 0 || y == ny - 1)))) {
                const int xx[3] = {x, y, 0};
                BcNode r;
                bc_resolve<2>(g, bc, xx, r);
                sx = r.in[0];
                sy = r.in[1];
                pfix = r.p_fixed;
                ufix = r.u_fixed;
                pv = T(r.p);
                uxv = T(r.u[0] - g.U[0]);
                uyv = T(r.u[1] - g.U[1]);
            }
            const long long id = (long long)sx + (long long)nx * sy;
            vp = sin_[id];
            vx = sin_[N + id];
            vy = sin_[2 * N + id];
            if (pfix) vp = pv;
            if (ufix) {
                vx = uxv;
                vy = uyv;
            }
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
            // df_i = w_i (3p - 3 U.v - 3/2 v.v + 3 c.v + 9 (c.U)(c.v) + 9/2 (c.v)^2
            // + A c.(S + S^T).c) (ux, uy hold v), formed for the pairs +-c at once: the even
            // part w (base + (9 c.U + 9/2 c.v)(c.v) + A c.(S + S^T).c) is shared, the odd
            // part 3 w c.v changes sign; no term with a zero component of c
            const T Ux = gU<T>(g, 0), Uy = gU<T>(g, 1);
            const T base = T(3) * p - T(1.5) * (ux * ux + uy * uy) - T(3) * (Ux * ux + Uy * uy);
            const T A2 = T(2) * A;
            const T axx = A2 * dxux, ayy = A2 * dyuy, axy = A2 * (dxuy + dyux);
            f[0] = w0 * base;
            {
                const T ev = w1 * (base + (T(9) * Ux + T(4.5) * ux) * ux + axx), od = T(3) * w1 * ux;
                f[1] = ev + od;
                f[2] = ev - od;
            }
            {
                const T ev = w1 * (base + (T(9) * Uy + T(4.5) * uy) * uy + ayy), od = T(3) * w1 * uy;
                f[3] = ev + od;
                f[4] = ev - od;
            }
            const T bd = base + axx + ayy;
            {
                const T cu = ux + uy, cU = Ux + Uy;
                const T ev = w2 * (bd + (T(9) * cU + T(4.5) * cu) * cu + axy), od = T(3) * w2 * cu;
                f[5] = ev + od;
                f[6] = ev - od;
            }
            {
                const T cu = ux - uy, cU = Ux - Uy;
                const T ev = w2 * (bd + (T(9) * cU + T(4.5) * cu) * cu - axy), od = T(3) * w2 * cu;
                f[7] = ev + od;
                f[8] = ev - od;
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
    const bool act = x < nx && y < ny && !((!g.per[0] && (x == 0 || x == nx - 1)) ||
                                           (!g.per[1] && (y == 0 || y == ny - 1)));
    if (act) {
        // the f_i streaming into the node, then the moments with the signs of c written out
        T fi[9];
#pragma unroll
        for (int i = 0; i < 9; i++)
            fi[i] = sf[i][threadIdx.y + 1 - Lat<2>::c(i, 1)][threadIdx.x + 1 - Lat<2>::c(i, 0)];
        const T d56 = fi[5] - fi[6], d78 = fi[7] - fi[8];
        const T ps = fi[0] + (fi[1] + fi[2]) + (fi[3] + fi[4]) + (fi[5] + fi[6]) + (fi[7] + fi[8]);
        const T usx = (fi[1] - fi[2]) + d56 + d78;
        const T usy = (fi[3] - fi[4]) + d56 - d78;
        const long long id = (long long)x + (long long)nx * y;
        sout[id] = ps * T(1.0 / 3.0);
        sout[N + id] = usx;
        sout[2 * N + id] = usy;
    }
    if (SP) span_end(ts);
}

// ===================================================================== forward, 3D
// 2.5D blocking. A block of TX x TY threads is the tile of source columns (x, y) whose
// f_i it evaluates, one column per thread; it writes the inner (TX-2) x (TY-2) columns
// and marches along z over ZC output planes. Per source plane s each thread evaluates
// the 15 f_i of its node into LDS and pushes them (by the gather of its output column)
// to the destination planes s-1, s, s+1, whose moments it keeps in registers. The
// thread's own column of p, u for planes s-2..s+2 (the z-derivative, one-sided at a
// wall, reaches two planes) lives in registers, filled one plane ahead; only u of
// plane s with a one-node ring is staged in LDS for the x and y derivatives.
template <typename T> struct G3 {
    static constexpr int TX = 64, TY = 8, NT = TX * TY;
    static constexpr int OX = TX - 2, OY = TY - 2;  // output tile
    static constexpr int WX = TX + 2, WY = TY + 2;  // staged u plane
    static constexpr int RING = 2 * WX + 2 * TY;    // staged nodes outside the tile
};

// Twice the derivative along one axis from the values at offsets -2..2: central in the
// interior and on periodic axes, second-order one-sided on the end nodes of a
// non-periodic axis.
template <typename T>
__device__ __forceinline__ T d2(T m2, T m1, T c, T p1, T p2, int v, int n, int per) {
    T d = p1 - m1;
    if (!per && (v == 0 || v == n - 1)) d = v == 0 ? T(-3) * c + T(4) * p1 - p2 : T(3) * c - T(4) * m1 + m2;
    return d;
}

// Weighted equilibria F_i = w_i f_i of one D3Q15 node (Lat<3> order), from p, u and
// D[a][b] = 2 d_a u_b. Opposite directions share the quadratic part and differ in the
// sign of 3 c.u, so each +-c pair costs one evaluation; the weights are folded into
// the per-class constants.
// With the deviation form (u holds v, U the reference velocity) the base gains -3 U.v
// and the quadratic part of pair c gains 9 (c.U)(c.v). Those coefficients are uniform
// over the grid: formed once on the host (FeqU) and passed as a kernel argument, so
// they stay in scalar registers.
template <typename T> struct FeqU {
    T m3U[3];  // -3 U_a
    T k1[3];   // 9 w1 U_a          (axis pairs)
    T k2[4];   // 9 w2 (c_k . U)    (corner pairs, c_k = (1, +-1, +-1))
    static FeqU make(const double U[3]) {
        FeqU f;
        for (int a = 0; a < 3; a++) {
            f.m3U[a] = T(-3.0 * U[a]);
            f.k1[a] = T(U[a]);  // 9 w1 = 1
        }
        const double cU[4] = {U[0] + U[1] + U[2], U[0] + U[1] - U[2], U[0] - U[1] + U[2], U[0] - U[1] - U[2]};
        for (int k = 0; k < 4; k++) f.k2[k] = T(9.0 / 72.0 * cU[k]);
        return f;
    }
};

template <typename T>
__device__ __forceinline__ void feq3(T p, const T u[3], const FeqU<T> &fu, const T D[3][3], T A, T F[15]) {
    constexpr T w0 = T(2.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 72.0);
    const T B = T(3) * p - T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) +
                (fu.m3U[0] * u[0] + fu.m3U[1] * u[1] + fu.m3U[2] * u[2]);
    F[0] = w0 * B;
    const T B1 = w1 * B, a1 = w1 * A;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const T sq = B1 + a1 * D[a][a] + (T(4.5) * w1 * u[a] + fu.k1[a]) * u[a];
        const T li = (T(3) * w1) * u[a];
        F[1 + 2 * a] = sq + li;
        F[2 + 2 * a] = sq - li;
    }
    const T a2 = w2 * A;
    const T C = w2 * B + a2 * (D[0][0] + D[1][1] + D[2][2]);
    const T exy = a2 * (D[0][1] + D[1][0]), exz = a2 * (D[0][2] + D[2][0]), eyz = a2 * (D[1][2] + D[2][1]);
    // corner pairs (i, opposite): (+,+,+) 7/14, (+,+,-) 8/13, (+,-,+) 9/12, (+,-,-) 10/11
    const T cu[4] = {u[0] + u[1] + u[2], u[0] + u[1] - u[2], u[0] - u[1] + u[2], u[0] - u[1] - u[2]};
    const T q[4] = {exy + exz + eyz, exy - exz - eyz, exz - exy - eyz, eyz - exy - exz};
    constexpr int ip[4] = {7, 8, 9, 10}, im[4] = {14, 13, 12, 11};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const T sq = C + q[k] + (T(4.5) * w2 * cu[k] + fu.k2[k]) * cu[k];
        const T li = (T(3) * w2) * cu[k];
        F[ip[k]] = sq + li;
        F[im[k]] = sq - li;
    }
}

template <typename T, bool SP>
__global__ __launch_bounds__(G3<T>::NT, sizeof(T) == 4 ? 6 : 2) void k_gather3d(Grid g, T A, FeqU<T> fu, int ZC,
                                                        const T *__restrict__ sin_, T *__restrict__ sout,
                                                        unsigned long long *ts) {
    using G = G3<T>;
    constexpr int TX = G::TX, TY = G::TY, WX = G::WX, WY = G::WY;
    __shared__ T wu[2][3][WY][WX];
    __shared__ T fb[15][TY][TX];
    if (SP) span_begin(ts);
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const uint3 tb = xcd_tile();
    const int x0 = tb.x * G::OX, y0 = tb.y * G::OY;
    const int z0 = tb.z * ZC, z1 = min(z0 + ZC, nz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;

    // this thread's source column
    int cx = x0 - 1 + tx, cy = y0 - 1 + ty;
    const bool colok = wrap_coord(cx, nx, g.per[0]) && wrap_coord(cy, ny, g.per[1]);
    const long long col = colok ? (long long)cx + (long long)nx * cy : 0;
    // ring node of the staged plane handled by this thread (tid < RING)
    int rx = 0, ry = 0;
    if (tid < 2 * WX) {
        rx = tid % WX;
        ry = tid < WX ? 0 : WY - 1;
    } else if (tid < G::RING) {
        const int k = tid - 2 * WX;
        ry = 1 + (k >> 1);
        rx = (k & 1) ? WX - 1 : 0;
    }
    int gx = x0 - 2 + rx, gy = y0 - 2 + ry;
    const bool ringok = tid < G::RING && wrap_coord(gx, nx, g.per[0]) && wrap_coord(gy, ny, g.per[1]);
    const long long rcol = ringok ? (long long)gx + (long long)nx * gy : 0;

    const long long plane = (long long)nx * ny;
    auto load_col = [&](int zp, T v[4]) {
        int zw = zp;
        const bool ok = colok && wrap_coord(zw, nz, g.per[2]);
        const long long id = col + plane * zw;
#pragma unroll
        for (int c = 0; c < 4; c++) v[c] = ok ? sin_[c * N + id] : T(0);
    };
    auto load_ring = [&](int zp, T v[3]) {
        int zw = zp;
        const bool ok = ringok && wrap_coord(zw, nz, g.per[2]);
        const long long id = rcol + plane * zw;
#pragma unroll
        for (int c = 0; c < 3; c++) v[c] = ok ? sin_[(c + 1) * N + id] : T(0);
    };

    T q[5][4];  // own column, planes s-2 .. s+2
#pragma unroll
    for (int j = 0; j < 5; j++) load_col(z0 - 3 + j, q[j]);
    T rv[3];
    load_ring(z0 - 1, rv);

    T accP[3] = {0, 0, 0}, accU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int s = z0 - 1; s <= z1; s++) {
        const int b = s & 1;
        // stage u of plane s: own node and ring node
#pragma unroll
        for (int c = 0; c < 3; c++) wu[b][c][ty + 1][tx + 1] = q[2][1 + c];
        if (tid < G::RING) {
#pragma unroll
            for (int c = 0; c < 3; c++) wu[b][c][ry][rx] = rv[c];
        }
        // next planes in flight while this one is evaluated
        const bool more = s + 3 <= z1 + 2;
        T nq[4], nr[3];
        if (more) load_col(s + 3, nq);
        if (s + 1 <= z1) load_ring(s + 1, nr);
        __syncthreads();

        // Sources off the grid (non-periodic axes) only feed boundary nodes, which this
        // kernel does not write; their f_i are evaluated from zeros and never used.
        int zs = s;
        (void)wrap_coord(zs, nz, g.per[2]);
        T f[15];
        {
            const int lx = tx + 1, ly = ty + 1;
            T D[3][3];  // D[a][b] = 2 d_a u_b
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const T(*U)[WX] = wu[b][c];
                D[0][c] = d2(U[ly][lx - 2 < 0 ? 0 : lx - 2], U[ly][lx - 1], U[ly][lx], U[ly][lx + 1],
                             U[ly][lx + 2 >= WX ? WX - 1 : lx + 2], cx, nx, g.per[0]);
                D[1][c] = d2(U[ly - 2 < 0 ? 0 : ly - 2][lx], U[ly - 1][lx], U[ly][lx], U[ly + 1][lx],
                             U[ly + 2 >= WY ? WY - 1 : ly + 2][lx], cy, ny, g.per[1]);
                D[2][c] = d2(q[0][1 + c], q[1][1 + c], q[2][1 + c], q[3][1 + c], q[4][1 + c], zs, nz, g.per[2]);
            }
            const T u[3] = {q[2][1], q[2][2], q[2][3]};
            feq3(q[2][0], u, fu, D, A, f);
        }
#pragma unroll
        for (int i = 0; i < 15; i++) fb[i][ty][tx] = f[i];
        __syncthreads();

        const bool out = tx < G::OX && ty < G::OY;
        if (out) {
#pragma unroll
            for (int i = 0; i < 15; i++) {
                const int ex = Lat<3>::c(i, 0), ey = Lat<3>::c(i, 1), ez = Lat<3>::c(i, 2);
                const T v = fb[i][ty + 1 - ey][tx + 1 - ex];
                accP[ez + 1] += v;
                accU[ez + 1][0] += T(ex) * v;
                accU[ez + 1][1] += T(ey) * v;
                accU[ez + 1][2] += T(ez) * v;
            }
            // destination plane s - 1 has received all its sources
            const int zd = s - 1, x = x0 + tx, y = y0 + ty;
            if (zd >= z0 && zd < z1 && x < nx && y < ny) {
                const int xx[3] = {x, y, zd};
                if (is_interior<3>(g, xx)) {
                    const long long id = (long long)x + (long long)nx * ((long long)y + (long long)ny * zd);
                    sout[id] = accP[0] * T(1.0 / 3.0);
#pragma unroll
                    for (int a = 0; a < 3; a++) sout[(1 + a) * N + id] = accU[0][a];
                }
            }
        }
        accP[0] = accP[1];
        accP[1] = accP[2];
        accP[2] = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            accU[0][a] = accU[1][a];
            accU[1][a] = accU[2][a];
            accU[2][a] = 0;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
#pragma unroll
            for (int c = 0; c < 4; c++) q[j][c] = q[j + 1][c];
        }
        if (more) {
#pragma unroll
            for (int c = 0; c < 4; c++) q[4][c] = nq[c];
        }
        if (s + 1 <= z1) {
#pragma unroll
            for (int c = 0; c < 3; c++) rv[c] = nr[c];
        }
    }
    if (SP) span_end(ts);
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
    // a prescribed velocity is stored as its deviation from U
#pragma unroll
    for (int a = 0; a < DIM; a++) s[(1 + a) * N + id] = r.u_fixed ? T(r.u[a] - g.U[a]) : s[(1 + a) * N + in];
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

// o += scale * (D_a^T sig)(z) for three sig components, with get(off, v) returning the
// components at z + off * e_a; the same coefficients as dT_stencil in straight-line
// form (no local arrays), central away from the ends of a non-periodic axis.
template <typename T, typename F>
__device__ __forceinline__ void dT_apply3(int za, int n, int per, T scale, F &&get, T o[3]) {
    auto add = [&](T cf, auto offc) {
        T v[3];
        get(decltype(offc)::value, v);
        const T k = scale * cf;
        o[0] += k * v[0];
        o[1] += k * v[1];
        o[2] += k * v[2];
    };
    using m2 = std::integral_constant<int, -2>;
    using m1 = std::integral_constant<int, -1>;
    using z0 = std::integral_constant<int, 0>;
    using p1 = std::integral_constant<int, 1>;
    using p2 = std::integral_constant<int, 2>;
    if (per || (za >= 3 && za <= n - 4)) {
        add(T(0.5), m1{});
        add(T(-0.5), p1{});
        return;
    }
    if (za - 1 >= 0) add((za - 1 == 0) ? T(2) : T(0.5), m1{});
    if (za + 1 <= n - 1) add((za + 1 == n - 1) ? T(-2) : T(-0.5), p1{});
    if (za == 0) add(T(-1.5), z0{});
    if (za == n - 1) add(T(1.5), z0{});
    if (za - 2 == 0) add(T(-0.5), m2{});
    if (za + 2 == n - 1) add(T(0.5), p2{});
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
template <typename T, bool SP>
__global__ __launch_bounds__(512) void k_adjgather2d(Grid g, Bc bc, T A, const T *__restrict__ ab,
                                                     const T *__restrict__ ustb, const double *__restrict__ Bprev,
                                                     Design D, int has_box, const T *__restrict__ sprev,
                                                     T *__restrict__ out, unsigned long long *ts,
                                                     T *__restrict__ ups) {
    constexpr int RX = G2_TX + 6, RY = G2_TY + 6;
    constexpr int MX = G2_TX + 4, MY = G2_TY + 4;
    __shared__ T sP[RY][RX], sU[RY][RX], sV[RY][RX];
    __shared__ T mpi[MY][MX], mux[MY][MX], muy[MY][MX], mxx[MY][MX], myy[MY][MX], mxy[MY][MX];
    if (SP) span_begin(ts);
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1];
    const uint3 tb = xcd_tile();
    const int x0 = tb.x * G2_TX, y0 = tb.y * G2_TY;
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
        // g_i = (p*bar/3 + c_i.u*bar)(x + c_i) and the moments sum_i w_i g_i (1, c_i, c_i c_i),
        // with the signs of c written out (no term with a zero component of c)
        const T g0 = sP[ly][lx];
        const T g1 = sP[ly][lx + 1] + sU[ly][lx + 1], g2 = sP[ly][lx - 1] - sU[ly][lx - 1];
        const T g3 = sP[ly + 1][lx] + sV[ly + 1][lx], g4 = sP[ly - 1][lx] - sV[ly - 1][lx];
        const T g5 = sP[ly + 1][lx + 1] + sU[ly + 1][lx + 1] + sV[ly + 1][lx + 1];
        const T g6 = sP[ly - 1][lx - 1] - sU[ly - 1][lx - 1] - sV[ly - 1][lx - 1];
        const T g7 = sP[ly - 1][lx + 1] + sU[ly - 1][lx + 1] - sV[ly - 1][lx + 1];
        const T g8 = sP[ly + 1][lx - 1] - sU[ly + 1][lx - 1] + sV[ly + 1][lx - 1];
        const T w0 = T(4.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
        const T e1 = g1 + g2, e2 = g3 + g4, s56 = g5 + g6, s78 = g7 + g8, d56 = g5 - g6, d78 = g7 - g8;
        const T dd = w2 * (s56 + s78);
        const T pi = w0 * g0 + w1 * (e1 + e2) + dd;
        const T ux = w1 * (g1 - g2) + w2 * (d56 + d78);
        const T uy = w1 * (g3 - g4) + w2 * (d56 - d78);
        const T sxx = w1 * e1 + dd, syy = w1 * e2 + dd, sxy = w2 * (s56 - s78);
        mpi[my][mx] = pi;
        mux[my][mx] = ux;
        muy[my][mx] = uy;
        mxx[my][mx] = sxx;
        myy[my][mx] = syy;
        mxy[my][mx] = sxy;
    }
    __syncthreads();
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x < nx && y < ny) {
        const int mx = threadIdx.x + 2, my = threadIdx.y + 2;
        const long long id = (long long)x + (long long)nx * y;
        const T u0 = gU<T>(g, 0) + sprev[N + id], u1 = gU<T>(g, 1) + sprev[2 * N + id];
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
        if (ups) {  // the moment ups itself (the paper's u~*), for its adjoint variant
            ups[id] = mux[my][mx];
            ups[N + id] = muy[my][mx];
        }
    }
    if (SP) span_end(ts);
}

// ===================================================================== adjoint, 3D
// The cotangent g of the post-streaming moments (p*bar / 3, u*bar) that the 3D kernel
// reads is prepared in place in `ab` by two small launches over the walls and the body
// box, so the bulk kernel reads plain arrays:
//   k_adj_fold3d: each interior node one layer in from a non-periodic wall adds the
//     entries of the wall nodes that copy it (fold_bc; the wall nodes are only read);
//   k_adj_clear3d: the wall nodes are zeroed (the moments see no cotangent there), and
//     u*bar of the interior nodes of the body box is replaced by ustb.
// The sums are those of star_bar, in the same order.

// Node t of the layers `lay` and n_a - 1 - lay of the non-periodic axes a = 0, 1, 2 in
// turn: t = (a, side, i, j) with side 0 for layer lay, and i, j over the other two axes
// (the lower one fastest). Returns the axis, or -1 past the end. layer_count < 2^31
// (checked on the host): 32-bit arithmetic.
__device__ __forceinline__ int layer_node(const Grid &g, long long t64, int lay, int x[3]) {
    unsigned t = (unsigned)t64;
    for (int a = 0; a < 3; a++) {
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        const unsigned nb = (unsigned)g.n[b], face = nb * (unsigned)g.n[c];
        if (g.per[a]) continue;
        if (t >= 2 * face) {
            t -= 2 * face;
            continue;
        }
        const unsigned side = t >= face ? 1u : 0u;
        const unsigned r = t - side * face, q = r / nb;
        x[a] = side ? g.n[a] - 1 - lay : lay;
        x[b] = (int)(r - q * nb);
        x[c] = (int)q;
        return a;
    }
    return -1;
}

// Interior nodes one layer in from a non-periodic wall, each once: a node that also lies
// on such a layer of an earlier axis belongs to that axis.
__device__ __forceinline__ bool shell_node(const Grid &g, long long t, int x[3]) {
    const int a = layer_node(g, t, 1, x);
    if (a < 0 || !is_interior<3>(g, x)) return false;
    for (int e = 0; e < a; e++)
        if (!g.per[e] && (x[e] == 1 || x[e] == g.n[e] - 2)) return false;
    return true;
}

// Nodes of one layer pair per non-periodic axis (the launch size of layer_node).
__host__ __device__ inline long long layer_count(const int n[3], const int per[3]) {
    long long m = 0;
    for (int a = 0; a < 3; a++)
        if (!per[a]) m += 2LL * n[a == 0 ? 1 : 0] * n[a == 2 ? 1 : 2];
    return m;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_fold3d(Grid g, Bc bc, T *__restrict__ ab, long long m) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x[3];
    if (t >= m || !shell_node(g, t, x)) return;
    const long long id = node_id(g, x[0], x[1], x[2]);
    T pb, ub[3];
    fold_bc<3, T>(g, bc, ab, x, id, pb, ub, true);
    ab[id] = pb;
#pragma unroll
    for (int a = 0; a < 3; a++) ab[(1 + a) * g.N + id] = ub[a];
}

// Threads [0, m) zero the wall nodes (the faces of the non-periodic axes, in the same
// enumeration with layers 0 and n_a - 1; nodes on several faces are written more than
// once, with the same zeros), threads [m, m + boxN) set u*bar of the box nodes.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_clear3d(Grid g, T *__restrict__ ab, long long m, Design D,
                                                     const double *__restrict__ Bprev, const T *__restrict__ ustb,
                                                     int has_box) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long N = g.N;
    int x[3];
    if (t < m) {
        if (layer_node(g, t, 0, x) < 0) return;
        const long long id = node_id(g, x[0], x[1], x[2]);
#pragma unroll
        for (int k = 0; k < 4; k++) ab[k * N + id] = T(0);
        return;
    }
    t -= m;
    if (!has_box || t >= D.boxN) return;
    // box node t: x = o + (t in the box's x-fastest order), on the grid and interior
    // (boxN < 2^31: 32-bit division)
    int o[3];
    box_origin<3>(D, Bprev, o);
    unsigned r = (unsigned)t;
    for (int a = 0; a < 3; a++) {
        const unsigned L = (unsigned)D.L[a], q = r / L;
        x[a] = o[a] + (int)(r - q * L);
        r = q;
        if (x[a] < 0 || x[a] >= g.n[a]) return;
    }
    if (!is_interior<3>(g, x)) return;
    const long long id = node_id(g, x[0], x[1], x[2]);
#pragma unroll
    for (int a = 0; a < 3; a++) ab[(1 + a) * N + id] = ustb[a * D.boxN + t];
}

// 2.5D blocking like the forward kernel. A block of TX x TY threads is the tile of
// columns whose moments pi, ups, sig it evaluates (one column per thread); it writes the
// inner (TX-2) x (TY-2) columns. Per plane s: g of plane s+1 (own column and a one-node
// ring) goes into a three-plane LDS ring, the moments of plane s are formed from the
// ring, the in-plane transposed-difference terms need sig of the x and y neighbours
// (LDS), the z term the own column's sig history (registers), so a column's output is
// complete two planes later. The global loads run one plane ahead in registers (g of
// plane s+2, the previous state of plane s+1), so their latency overlaps the work and
// the barriers of plane s.
//
// The second-order one-sided difference on a wall node reaches two nodes inward, so the
// transpose at the node two away from a wall needs sig on the wall node. Tile origins
// are shifted by `off` (0 or 1 per axis, chosen on the host) so that no tile boundary
// falls on node 2 or node n-2 of a non-periodic axis; the one-node moment ring then
// always contains the wall node where it is needed.
template <typename T> struct A3 {
    static constexpr int TX = 64, TY = 8, NT = TX * TY;
    static constexpr int OX = TX - 2, OY = TY - 2;
    static constexpr int WX = TX + 2, WY = TY + 2;
    static constexpr int RING = 2 * WX + 2 * TY;
};

// ab as prepared by k_adj_fold3d and k_adj_clear3d.
template <typename T, bool SP>
__global__ __launch_bounds__(A3<T>::NT, sizeof(T) == 4 ? 4 : 2) void k_adjgather3d(
    Grid g, T A, int ZC, int offx, int offy, const T *__restrict__ ab, const T *__restrict__ sprev,
    T *__restrict__ out, unsigned long long *ts, T *__restrict__ ups) {
    using G = A3<T>;
    constexpr int TX = G::TX, TY = G::TY, WX = G::WX, WY = G::WY;
    __shared__ T gr[3][4][WY][WX];  // g = (p*bar / 3, u*bar) of planes s-1, s, s+1
    __shared__ T sg[5][TY][TX];     // sig_xx, sig_xy, sig_xz, sig_yy, sig_yz of plane s
    if (SP) span_begin(ts);
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const uint3 tb = xcd_tile();
    const int x0 = (int)tb.x * G::OX - offx, y0 = (int)tb.y * G::OY - offy;
    const int z0 = tb.z * ZC, z1 = min(z0 + ZC, nz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
    // own column (x, y as the output node when inside the output tile)
    const int ox = x0 - 1 + tx, oy = y0 - 1 + ty;
    int cx = ox, cy = oy;
    const bool colok = wrap_coord(cx, nx, g.per[0]) && wrap_coord(cy, ny, g.per[1]);
    // ring node of the g planes handled by this thread (tid < RING)
    int rx = 0, ry = 0;
    if (tid < 2 * WX) {
        rx = tid % WX;
        ry = tid < WX ? 0 : WY - 1;
    } else if (tid < G::RING) {
        const int k = tid - 2 * WX;
        ry = 1 + (k >> 1);
        rx = (k & 1) ? WX - 1 : 0;
    }
    int gx = x0 - 2 + rx, gy = y0 - 2 + ry;
    const bool ringok = tid < G::RING && wrap_coord(gx, nx, g.per[0]) && wrap_coord(gy, ny, g.per[1]);
    const long long cid = (long long)cx + (long long)nx * cy, rid = (long long)gx + (long long)nx * gy;
    const long long plane = (long long)nx * ny;

    // g at plane zp of the own column and the ring node (zero off the grid)
    T gc[4], gq[4];
    auto load = [&](int zp) {
        int zw = zp;
        const bool zok = wrap_coord(zw, nz, g.per[2]);
        const long long zo = (long long)zw * plane;
#pragma unroll
        for (int c = 0; c < 4; c++) gc[c] = (zok && colok) ? ab[c * N + zo + cid] : T(0);
#pragma unroll
        for (int c = 0; c < 4; c++) gq[c] = (zok && ringok) ? ab[c * N + zo + rid] : T(0);
    };
    auto store = [&](int zp) {
        const int sl = ((zp % 3) + 3) % 3;
        gr[sl][0][ty + 1][tx + 1] = gc[0] * T(1.0 / 3.0);
#pragma unroll
        for (int c = 1; c < 4; c++) gr[sl][c][ty + 1][tx + 1] = gc[c];
        if (tid < G::RING) {
            gr[sl][0][ry][rx] = gq[0] * T(1.0 / 3.0);
#pragma unroll
            for (int c = 1; c < 4; c++) gr[sl][c][ry][rx] = gq[c];
        }
    };

    const bool outcol = tx >= 1 && tx <= G::OX && ty >= 1 && ty <= G::OY && ox >= 0 && ox < nx && oy >= 0 &&
                        oy < ny;
    const long long oid = (long long)ox + (long long)nx * oy;
    // previous state u at the output column of plane s (loaded a plane ahead)
    T uc[3] = {0, 0, 0};
    auto load_u = [&](int zp) {
        const bool ok = outcol && zp >= z0 && zp < z1;
#pragma unroll
        for (int a = 0; a < 3; a++) uc[a] = ok ? gU<T>(g, a) + sprev[(1 + a) * N + (long long)zp * plane + oid] : T(0);
    };
    T part[3][4];  // local + in-plane terms of planes s-2, s-1, s
    T hz[5][3];    // sig_xz, sig_yz, sig_zz of planes s-4 .. s
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) part[j][c] = 0;
#pragma unroll
    for (int j = 0; j < 5; j++) hz[j][0] = hz[j][1] = hz[j][2] = 0;
    const T A2 = T(2) * A;
    constexpr T w0 = T(2.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 72.0);

    load(z0 - 3);
    store(z0 - 3);
    load(z0 - 2);
    store(z0 - 2);
    load(z0 - 1);
    load_u(z0 - 2);
    for (int s = z0 - 2; s <= z1 + 1; s++) {
        store(s + 1);
        const T u0 = uc[0], u1 = uc[1], u2 = uc[2];
        if (s + 2 <= z1 + 2) load(s + 2);
        load_u(s + 1);
        __syncthreads();
        // moments of plane s at the own node: g_i taken at the node + c_i
        const int sm = ((s - 1) % 3 + 3) % 3, s0 = ((s % 3) + 3) % 3, sp = ((s + 1) % 3 + 3) % 3;
        const int lx = tx + 1, ly = ty + 1;
        T pi, up[3], sxx, syy, szz, sxy, sxz, syz;
        {
            // rest and axis pairs: s = g(+e) + g(-e), d = g(+e) - g(-e)
            const T g0 = gr[s0][0][ly][lx];
            T sa[3], da[3];
            {
                const T gp = gr[s0][0][ly][lx + 1] + gr[s0][1][ly][lx + 1];
                const T gm = gr[s0][0][ly][lx - 1] - gr[s0][1][ly][lx - 1];
                sa[0] = gp + gm;
                da[0] = gp - gm;
            }
            {
                const T gp = gr[s0][0][ly + 1][lx] + gr[s0][2][ly + 1][lx];
                const T gm = gr[s0][0][ly - 1][lx] - gr[s0][2][ly - 1][lx];
                sa[1] = gp + gm;
                da[1] = gp - gm;
            }
            {
                const T gp = gr[sp][0][ly][lx] + gr[sp][3][ly][lx];
                const T gm = gr[sm][0][ly][lx] - gr[sm][3][ly][lx];
                sa[2] = gp + gm;
                da[2] = gp - gm;
            }
            // corner pairs (+,+,+), (+,+,-), (+,-,+), (+,-,-) and their opposites
            T sc[4], dc[4];
            constexpr int cyk[4] = {1, 1, -1, -1}, czk[4] = {1, -1, 1, -1};
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int ey = cyk[k], ez = czk[k];
                const int zl = ez > 0 ? sp : sm, zo = ez > 0 ? sm : sp;
                const T gp = gr[zl][0][ly + ey][lx + 1] + gr[zl][1][ly + ey][lx + 1] +
                             T(ey) * gr[zl][2][ly + ey][lx + 1] + T(ez) * gr[zl][3][ly + ey][lx + 1];
                const T gm = gr[zo][0][ly - ey][lx - 1] - gr[zo][1][ly - ey][lx - 1] -
                             T(ey) * gr[zo][2][ly - ey][lx - 1] - T(ez) * gr[zo][3][ly - ey][lx - 1];
                sc[k] = gp + gm;
                dc[k] = gp - gm;
            }
            const T scs = (sc[0] + sc[1]) + (sc[2] + sc[3]);
            pi = w0 * g0 + w1 * (sa[0] + sa[1] + sa[2]) + w2 * scs;
            up[0] = w1 * da[0] + w2 * ((dc[0] + dc[1]) + (dc[2] + dc[3]));
            up[1] = w1 * da[1] + w2 * ((dc[0] + dc[1]) - (dc[2] + dc[3]));
            up[2] = w1 * da[2] + w2 * ((dc[0] - dc[1]) + (dc[2] - dc[3]));
            sxx = w1 * sa[0] + w2 * scs;
            syy = w1 * sa[1] + w2 * scs;
            szz = w1 * sa[2] + w2 * scs;
            sxy = w2 * ((sc[0] + sc[1]) - (sc[2] + sc[3]));
            sxz = w2 * ((sc[0] - sc[1]) + (sc[2] - sc[3]));
            syz = w2 * ((sc[0] - sc[1]) - (sc[2] - sc[3]));
        }
        sg[0][ty][tx] = sxx;
        sg[1][ty][tx] = sxy;
        sg[2][ty][tx] = sxz;
        sg[3][ty][tx] = syy;
        sg[4][ty][tx] = syz;
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int c = 0; c < 3; c++) hz[j][c] = hz[j + 1][c];
        hz[4][0] = sxz;
        hz[4][1] = syz;
        hz[4][2] = szz;
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int c = 0; c < 4; c++) part[j][c] = part[j + 1][c];
        part[2][0] = part[2][1] = part[2][2] = part[2][3] = 0;
        __syncthreads();
        if (outcol && s >= z0 && s < z1) {
            T o0 = T(3) * up[0] + T(9) * (sxx * u0 + sxy * u1 + sxz * u2) - T(3) * pi * u0;
            T o1 = T(3) * up[1] + T(9) * (sxy * u0 + syy * u1 + syz * u2) - T(3) * pi * u1;
            T o2 = T(3) * up[2] + T(9) * (sxz * u0 + syz * u1 + szz * u2) - T(3) * pi * u2;
            T o[3] = {o0, o1, o2};
            dT_apply3<T>(ox, nx, g.per[0], A2, [&](int d, T v[3]) {  // a = x: sig_xb -> u_b
                const int xi = min(max(tx + d, 0), TX - 1);
                v[0] = sg[0][ty][xi];
                v[1] = sg[1][ty][xi];
                v[2] = sg[2][ty][xi];
            }, o);
            dT_apply3<T>(oy, ny, g.per[1], A2, [&](int d, T v[3]) {  // a = y: sig_yb -> u_b
                const int yi = min(max(ty + d, 0), TY - 1);
                v[0] = sg[1][yi][tx];
                v[1] = sg[3][yi][tx];
                v[2] = sg[4][yi][tx];
            }, o);
            o0 = o[0];
            o1 = o[1];
            o2 = o[2];
            part[2][0] = T(3) * pi;
            part[2][1] = o0;
            part[2][2] = o1;
            part[2][3] = o2;
            if (ups) {  // the moment ups itself (the paper's u~*), for its adjoint variant
                const long long id = oid + (long long)s * plane;
                ups[id] = up[0];
                ups[N + id] = up[1];
                ups[2 * N + id] = up[2];
            }
        }
        const int zo = s - 2;
        if (outcol && zo >= z0 && zo < z1) {
            T o[3] = {part[0][1], part[0][2], part[0][3]};
            // a = z: sig_zb -> u_b from the history (plane zo + d is entry d + 2)
            dT_apply3<T>(zo, nz, g.per[2], A2, [&](int d, T v[3]) {
                v[0] = hz[d + 2][0];
                v[1] = hz[d + 2][1];
                v[2] = hz[d + 2][2];
            }, o);
            const long long id = oid + (long long)zo * plane;
            out[id] = part[0][0];
            out[N + id] = o[0];
            out[2 * N + id] = o[1];
            out[3 * N + id] = o[2];
        }
    }
    if (SP) span_end(ts);
}

// ===================================================================== divergence check
// Flag bit 8 when some node of the state holds a non-finite pressure or velocity, or a
// speed |u| = |U + v| beyond the lattice sound speed 1/sqrt(3), where the scheme no
// longer represents a flow. Grid-stride; an atomic only from a wave that found one.
template <typename T>
__global__ __launch_bounds__(256) void k_check_state(Grid g, int dim, const T *__restrict__ s,
                                                     int *__restrict__ flag) {
    const long long N = g.N;
    bool bad = false;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const T p = s[i];
        double uu = 0.0;
        bool fin = isfinite((double)p);
        for (int a = 0; a < dim; a++) {
            const double u = g.U[a] + (double)s[(1 + a) * N + i];
            fin = fin && isfinite(u);
            uu += u * u;
        }
        bad = bad || !fin || !(uu <= 1.0 / 3.0);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 8);
}

}  // namespace lks
