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
// 2.5D blocking: a TX x TY tile of (x, y) columns marches along z over ZC output
// planes. For every source plane s, the f_i of the tile plus a one-node (x, y) ring are
// evaluated once into LDS and pushed to the destination planes s-1, s, s+1, whose
// moments each thread keeps in registers for its column. p, u of planes s-2..s+2 sit
// in a 5-slot LDS ring with a two-node (x, y) ring (the one-sided z-derivative at a
// wall reaches two planes).
template <typename T> struct G3 {
    static constexpr int TX = 64, TY = sizeof(T) == 4 ? 8 : 4, NT = TX * TY;
};

template <typename T>
__device__ __forceinline__ T d1(T m2, T m1, T c, T p1, T p2, int v, int n, int per) {
    // derivative along one axis from the values at offsets -2..2 (boundary-aware)
    if (per || (v > 0 && v < n - 1)) return T(0.5) * (p1 - m1);
    if (v == 0) return T(0.5) * (T(-3) * c + T(4) * p1 - p2);
    return T(0.5) * (T(3) * c - T(4) * m1 + m2);
}

template <typename T>
__global__ __launch_bounds__(G3<T>::NT) void k_gather3d(Grid g, T A, int ZC, const T *__restrict__ sin_,
                                                        T *__restrict__ sout) {
    constexpr int TX = G3<T>::TX, TY = G3<T>::TY, NT = G3<T>::NT;
    constexpr int RX = TX + 4, RY = TY + 4, FX = TX + 2, FY = TY + 2;
    __shared__ T win[5][4][RY][RX];
    __shared__ T fb[15][FY][FX];
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * ZC, z1 = min(z0 + ZC, nz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;

    // plane loads: each thread owns the ring-window entries l = tid + j*NT; a plane is
    // fetched into registers one iteration ahead and stored into its LDS slot after the
    // slot's previous plane is no longer read (software pipelining of the HBM latency)
    constexpr int PER = (RX * RY + NT - 1) / NT;
    T pre[PER][4];
    auto fetch = [&](int zp) {
        int zw = zp;
        const bool zok = wrap_coord(zw, nz, g.per[2]);
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int l = tid + j * NT;
            const int lx = l % RX, ly = l / RX;
            int x = x0 + lx - 2, y = y0 + ly - 2;
#pragma unroll
            for (int c = 0; c < 4; c++) pre[j][c] = 0;
            if (l < RX * RY && zok && wrap_coord(x, nx, g.per[0]) && wrap_coord(y, ny, g.per[1])) {
                const long long id = (long long)x + (long long)nx * ((long long)y + (long long)ny * zw);
#pragma unroll
                for (int c = 0; c < 4; c++) pre[j][c] = sin_[c * N + id];
            }
        }
    };
    auto store = [&](int zp) {
        const int slot = ((zp % 5) + 5) % 5;
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int l = tid + j * NT;
            if (l < RX * RY) {
                const int lx = l % RX, ly = l / RX;
#pragma unroll
                for (int c = 0; c < 4; c++) win[slot][c][ly][lx] = pre[j][c];
            }
        }
    };

    T accP[3] = {0, 0, 0}, accU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int zp = z0 - 3; zp <= z0 + 1; zp++) {
        fetch(zp);
        store(zp);
    }
    for (int s = z0 - 1; s <= z1; s++) {
        const bool more = s + 3 <= z1 + 2;  // planes up to z1 + 2 are read (last s = z1)
        if (more) fetch(s + 3);
        __syncthreads();
        int zs = s;
        const bool sok = wrap_coord(zs, nz, g.per[2]);
        const int sm2 = ((s - 2) % 5 + 5) % 5, sm1 = ((s - 1) % 5 + 5) % 5, s0 = ((s % 5) + 5) % 5;
        const int sp1 = ((s + 1) % 5 + 5) % 5, sp2 = ((s + 2) % 5 + 5) % 5;
        for (int l = tid; l < FX * FY; l += NT) {
            const int fx = l % FX, fy = l / FX;
            const int lx = fx + 1, ly = fy + 1;
            int x = x0 + fx - 1, y = y0 + fy - 1;
            const bool ok = sok && wrap_coord(x, nx, g.per[0]) && wrap_coord(y, ny, g.per[1]);
            T f[15];
            if (ok) {
                T S[3][3];  // S[a][b] = d_a u_b
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    const T(*U)[RX] = win[s0][1 + b];
                    S[0][b] = d1(U[ly][lx - 2 < 0 ? 0 : lx - 2], U[ly][lx - 1], U[ly][lx], U[ly][lx + 1],
                                 U[ly][lx + 2 >= RX ? RX - 1 : lx + 2], x, nx, g.per[0]);
                    S[1][b] = d1(U[ly - 2 < 0 ? 0 : ly - 2][lx], U[ly - 1][lx], U[ly][lx], U[ly + 1][lx],
                                 U[ly + 2 >= RY ? RY - 1 : ly + 2][lx], y, ny, g.per[1]);
                    S[2][b] = d1(win[sm2][1 + b][ly][lx], win[sm1][1 + b][ly][lx], U[ly][lx],
                                 win[sp1][1 + b][ly][lx], win[sp2][1 + b][ly][lx], zs, nz, g.per[2]);
                }
                const T p = win[s0][0][ly][lx];
                const T u[3] = {win[s0][1][ly][lx], win[s0][2][ly][lx], win[s0][3][ly][lx]};
                const T base = T(3) * p - T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                // A c.(S + S^T).c = 2A (sum_a c_a^2 S_aa + sum_{a<b} c_a c_b (S_ab + S_ba))
                const T dxx = T(2) * A * S[0][0], dyy = T(2) * A * S[1][1], dzz = T(2) * A * S[2][2];
                const T exy = T(2) * A * (S[0][1] + S[1][0]), exz = T(2) * A * (S[0][2] + S[2][0]);
                const T eyz = T(2) * A * (S[1][2] + S[2][1]);
#pragma unroll
                for (int i = 0; i < 15; i++) {
                    const int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
                    const T cu = T(cx) * u[0] + T(cy) * u[1] + T(cz) * u[2];
                    const T an = T(cx * cx) * dxx + T(cy * cy) * dyy + T(cz * cz) * dzz + T(cx * cy) * exy +
                                 T(cx * cz) * exz + T(cy * cz) * eyz;
                    f[i] = T(Lat<3>::w(i)) * (base + T(3) * cu + T(4.5) * cu * cu + an);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 15; i++) f[i] = 0;
            }
#pragma unroll
            for (int i = 0; i < 15; i++) fb[i][fy][fx] = f[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 15; i++) {
            const int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
            const T f = fb[i][ty + 1 - cy][tx + 1 - cx];
            accP[cz + 1] += f;
            accU[cz + 1][0] += T(cx) * f;
            accU[cz + 1][1] += T(cy) * f;
            accU[cz + 1][2] += T(cz) * f;
        }
        __syncthreads();
        // destination plane s - 1 has received all its sources
        const int zd = s - 1;
        const int x = x0 + tx, y = y0 + ty;
        if (zd >= z0 && zd < z1 && x < nx && y < ny) {
            const int xx[3] = {x, y, zd};
            if (is_interior<3>(g, xx)) {
                const long long id = (long long)x + (long long)nx * ((long long)y + (long long)ny * zd);
                sout[id] = accP[0] * T(1.0 / 3.0);
#pragma unroll
                for (int a = 0; a < 3; a++) sout[(1 + a) * N + id] = accU[0][a];
            }
        }
        if (more) store(s + 3);
        accP[0] = accP[1];
        accP[1] = accP[2];
        accP[2] = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            accU[0][a] = accU[1][a];
            accU[1][a] = accU[2][a];
            accU[2][a] = 0;
        }
    }
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
// 2.5D blocking as in the forward. For every plane s: the inputs g (p*bar/3, u*bar) of
// the planes s-1..s+1 with a 3-node (x, y) ring sit in a 3-slot LDS ring; the ten
// moments (pi, ups, sig) of plane s are formed on a 2-node ring; each thread then forms
// its node's local and in-plane transpose terms for plane s (kept in registers) and
// records its column's sig_z* history; plane s-2 is completed with the z-transpose
// terms and written.
template <typename T> struct A3 {
    static constexpr int TX = 64, TY = sizeof(T) == 4 ? 8 : 4, NT = TX * TY;
};

template <typename T>
__global__ __launch_bounds__(A3<T>::NT) void k_adjgather3d(Grid g, Bc bc, T A, int ZC, const T *__restrict__ ab,
                                                           const T *__restrict__ ustb,
                                                           const double *__restrict__ Bprev, Design D, int has_box,
                                                           const T *__restrict__ sprev, T *__restrict__ out) {
    constexpr int TX = A3<T>::TX, TY = A3<T>::TY, NT = A3<T>::NT;
    constexpr int GX = TX + 6, GY = TY + 6, MX = TX + 4, MY = TY + 4;
    __shared__ T gw[3][4][GY][GX];
    __shared__ T mo[10][MY][MX];  // pi, ux, uy, uz, sxx, syy, szz, sxy, sxz, syz
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * ZC, z1 = min(z0 + ZC, nz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
    Box bx;
    if (has_box) {
        box_origin<3>(D, Bprev, bx.o);
        bx.L[0] = D.L[0];
        bx.L[1] = D.L[1];
        bx.L[2] = D.L[2];
    }
    auto load_plane = [&](int zp) {
        int zw = zp;
        const bool zok = wrap_coord(zw, nz, g.per[2]);
        const int slot = ((zp % 3) + 3) % 3;
        for (int l = tid; l < GX * GY; l += NT) {
            const int lx = l % GX, ly = l / GX;
            int xx[3] = {x0 + lx - 3, y0 + ly - 3, zw};
            T v[4] = {0, 0, 0, 0};
            if (zok && wrap_coord(xx[0], nx, g.per[0]) && wrap_coord(xx[1], ny, g.per[1]) &&
                is_interior<3>(g, xx)) {
                const long long id = node_id(g, xx[0], xx[1], xx[2]);
                T pb, ub[3];
                star_bar<3, T>(g, bc, ab, ustb, bx, has_box, D.boxN, xx, id, pb, ub);
                v[0] = pb * T(1.0 / 3.0);
                v[1] = ub[0];
                v[2] = ub[1];
                v[3] = ub[2];
            }
#pragma unroll
            for (int c = 0; c < 4; c++) gw[slot][c][ly][lx] = v[c];
        }
    };
    const int x = x0 + tx, y = y0 + ty;
    const bool col_ok = x < nx && y < ny;
    T part[3][4];   // local + in-plane terms of planes s-2, s-1, s
    T hz[5][3];     // sig_xz, sig_yz, sig_zz of planes s-4..s
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) part[j][c] = 0;
#pragma unroll
    for (int j = 0; j < 5; j++) hz[j][0] = hz[j][1] = hz[j][2] = 0;
    const T A2 = T(2) * A;
    load_plane(z0 - 3);
    load_plane(z0 - 2);
    for (int s = z0 - 2; s <= z1 + 1; s++) {
        load_plane(s + 1);
        __syncthreads();
        const int gm = ((s - 1) % 3 + 3) % 3, g0 = ((s % 3) + 3) % 3, gp = ((s + 1) % 3 + 3) % 3;
        for (int l = tid; l < MX * MY; l += NT) {
            const int mx = l % MX, my = l / MX;
            const int lx = mx + 1, ly = my + 1;  // in the 3-ring arrays
            T m[10];
#pragma unroll
            for (int j = 0; j < 10; j++) m[j] = 0;
#pragma unroll
            for (int i = 0; i < 15; i++) {
                const int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
                const int sl = cz < 0 ? gm : (cz > 0 ? gp : g0);
                const T gi = gw[sl][0][ly + cy][lx + cx] + T(cx) * gw[sl][1][ly + cy][lx + cx] +
                             T(cy) * gw[sl][2][ly + cy][lx + cx] + T(cz) * gw[sl][3][ly + cy][lx + cx];
                const T wg = T(Lat<3>::w(i)) * gi;
                m[0] += wg;
                m[1] += T(cx) * wg;
                m[2] += T(cy) * wg;
                m[3] += T(cz) * wg;
                m[4] += T(cx * cx) * wg;
                m[5] += T(cy * cy) * wg;
                m[6] += T(cz * cz) * wg;
                m[7] += T(cx * cy) * wg;
                m[8] += T(cx * cz) * wg;
                m[9] += T(cy * cz) * wg;
            }
#pragma unroll
            for (int j = 0; j < 10; j++) mo[j][my][mx] = m[j];
        }
        __syncthreads();
        const int mx = tx + 2, my = ty + 2;
        // history of sig_z* for the z-transpose
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int c = 0; c < 3; c++) hz[j][c] = hz[j + 1][c];
        hz[4][0] = mo[8][my][mx];
        hz[4][1] = mo[9][my][mx];
        hz[4][2] = mo[6][my][mx];
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int c = 0; c < 4; c++) part[j][c] = part[j + 1][c];
        part[2][0] = part[2][1] = part[2][2] = part[2][3] = 0;
        if (col_ok && s >= z0 && s < z1) {
            const long long id = (long long)x + (long long)nx * ((long long)y + (long long)ny * s);
            const T u0 = sprev[N + id], u1 = sprev[2 * N + id], u2 = sprev[3 * N + id];
            const T pi = mo[0][my][mx];
            const T sxx = mo[4][my][mx], syy = mo[5][my][mx], szz = mo[6][my][mx];
            const T sxy = mo[7][my][mx], sxz = mo[8][my][mx], syz = mo[9][my][mx];
            T o0 = T(3) * mo[1][my][mx] + T(9) * (sxx * u0 + sxy * u1 + sxz * u2) - T(3) * pi * u0;
            T o1 = T(3) * mo[2][my][mx] + T(9) * (sxy * u0 + syy * u1 + syz * u2) - T(3) * pi * u1;
            T o2 = T(3) * mo[3][my][mx] + T(9) * (sxz * u0 + syz * u1 + szz * u2) - T(3) * pi * u2;
            int off[5];
            T cf[5];
            int k = dT_stencil<T>(x, nx, g.per[0], off, cf);
            for (int j = 0; j < k; j++) {  // a = x: sig_xb -> u_b
                o0 += A2 * cf[j] * mo[4][my][mx + off[j]];
                o1 += A2 * cf[j] * mo[7][my][mx + off[j]];
                o2 += A2 * cf[j] * mo[8][my][mx + off[j]];
            }
            k = dT_stencil<T>(y, ny, g.per[1], off, cf);
            for (int j = 0; j < k; j++) {  // a = y: sig_yb -> u_b
                o0 += A2 * cf[j] * mo[7][my + off[j]][mx];
                o1 += A2 * cf[j] * mo[5][my + off[j]][mx];
                o2 += A2 * cf[j] * mo[9][my + off[j]][mx];
            }
            part[2][0] = T(3) * pi;
            part[2][1] = o0;
            part[2][2] = o1;
            part[2][3] = o2;
        }
        __syncthreads();
        const int zo = s - 2;
        if (col_ok && zo >= z0 && zo < z1) {
            int off[5];
            T cf[5];
            const int k = dT_stencil<T>(zo, nz, g.per[2], off, cf);
            T o[3] = {part[0][1], part[0][2], part[0][3]};
            for (int j = 0; j < k; j++) {  // a = z: sig_zb -> u_b, history index off + 2
                const int h = off[j] + 2;
                T hx = hz[0][0], hy = hz[0][1], hzz = hz[0][2];
#pragma unroll
                for (int q = 1; q < 5; q++)
                    if (q == h) {
                        hx = hz[q][0];
                        hy = hz[q][1];
                        hzz = hz[q][2];
                    }
                o[0] += A2 * cf[j] * hx;
                o[1] += A2 * cf[j] * hy;
                o[2] += A2 * cf[j] * hzz;
            }
            const long long id = (long long)x + (long long)nx * ((long long)y + (long long)ny * zo);
            out[id] = part[0][0];
            out[N + id] = o[0];
            out[2 * N + id] = o[1];
            out[3 * N + id] = o[2];
        }
    }
}

}  // namespace lks
