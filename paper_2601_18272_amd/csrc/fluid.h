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

// ===================================================================== lane shifts
// A register's value in lane l - 1 (from_left) or l + 1 (from_right) of the wave,
// through the DPP whole-wave shifts (wave_shr:1, wave_shl:1); lanes past either end of
// the wave read zero. FP64 values move as two 32-bit halves.
__device__ __forceinline__ float from_left(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double dpp64(double v, int ctrl_left) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    int lo, hi;
    if (ctrl_left) {
        lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x138, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x138, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x130, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x130, 0xf, 0xf, true);
    }
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_left(double v) { return dpp64(v, 1); }
__device__ __forceinline__ double from_right(double v) { return dpp64(v, 0); }

// ===================================================================== forward, 2D: column march
// The kernel of large grids (k_gather2d below serves those whose tiles fill the device
// only a few times over, where the march's serial rows cost more than they save).
// Column march. Each wave works alone: its lane l holds column x0 - 2 + l, and it
// writes the C2_W = 60 columns x0 .. x0+59 of a run of `rows` rows, marching along y.
// Neighbours along x are the wave's other lanes (DPP shifts), neighbours along y are rows
// the lane keeps in registers, so the kernel uses no LDS and no barriers. At iteration r
// the lane holds p, u of rows r-2 .. r+2 (a one-sided y derivative at a non-periodic end
// reaches two rows) and has rows r+3 .. r+5 in flight; it evaluates the f_i of row r,
// pushes them into the moments of rows r-1, r, r+1 and stores row r-1, now complete.
// Rows live in a ring of 8 register slots (row q in slot (q - Ya + 3) mod 8); the loop
// is unrolled by 8 so that every slot index is a compile-time constant.
//
// With fold, boundary nodes are read from the interior node they copy and their
// prescribed values replace what the face fixes (bc_resolve), as k_bc would have stored
// them; the replacement is applied when the row is first needed (as row r+2), long
// after its loads were issued.
constexpr int C2_W = 60, C2_NT = 256;

// Prescribed values of 2D node (x, y) as a fold applies them: mask (bit 0 p, bit 1 u)
// and the values (u as its deviation from U).
template <typename T>
__device__ __forceinline__ void fold_values2(const Grid &g, const Bc &bc, int x, int y, int &m, T &vp, T &vu,
                                             T &vv) {
    const int xx[3] = {x, y, 0};
    BcNode b;
    bc_resolve<2>(g, bc, xx, b);
    m = (b.p_fixed ? 1 : 0) | (b.u_fixed ? 2 : 0);
    vp = T(b.p);
    vu = T(b.u[0] - g.U[0]);
    vv = T(b.u[1] - g.U[1]);
}

template <typename T, bool SP>
__global__ __launch_bounds__(C2_NT) void k_gather2d_march(Grid g, T A, Bc bc, int fold, int rows, int nstrip, int nwave,
                                                    const T *__restrict__ sin_, T *__restrict__ sout,
                                                    unsigned long long *ts) {
    if (SP) span_begin(ts);
    // the grid as plain scalars: the march below is written without closures or
    // references, so that every per-lane value stays in a register
    const int nx = g.n[0], ny = g.n[1], perx = g.per[0], pery = g.per[1];
    const long long N = g.N;
    const T Ux = gU<T>(g, 0), Uy = gU<T>(g, 1);
    const int lane = threadIdx.x & 63;
    // the wave's index, in a scalar register (uniform over the wave)
    const int wv = (int)xcd_block() * (C2_NT / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wv < nwave) {
        // uniform over the wave: kept in scalar registers (readfirstlane), so that the row
        // logic below is scalar code and its branches are scalar branches
        const int strip = __builtin_amdgcn_readfirstlane(wv % nstrip);
        const int run = __builtin_amdgcn_readfirstlane(wv / nstrip);
        const int x0 = strip * C2_W, Ya = run * rows, Yb = min(Ya + rows, ny);
        // this lane's column; lanes off the grid (a non-periodic x axis) read a column on
        // the grid instead: their f_i reach only boundary nodes, which are not written
        const int x = x0 - 2 + lane;
        int xw = x;
        const bool colok = wrap_coord(xw, nx, perx);
        if (!colok) xw = x < 0 ? 0 : nx - 1;
        const int xcls = (!perx && colok) ? (xw == 0 ? 1 : (xw == nx - 1 ? 2 : 0)) : 0;
        const unsigned xl = (unsigned)((fold && xcls) ? (xcls == 1 ? 1 : nx - 2) : xw);
        const bool wave_xb = !perx && (x0 - 2 <= 0 || x0 + 61 >= nx - 1);
        const bool outc = lane >= 2 && lane < 2 + C2_W && x < nx && xcls == 0;
        // prescribed values of this lane's node (fold): on rows off the y faces (0, x faces
        // only), on the low and on the high y face (1, 2); resolved once here
        int fx0 = 0, fx1 = 0, fx2 = 0;
        T fp0 = 0, fp1 = 0, fp2 = 0, fu0 = 0, fu1 = 0, fu2 = 0, fv0 = 0, fv1 = 0, fv2 = 0;
        if (fold) {
            fold_values2<T>(g, bc, xw, pery ? 0 : 1, fx0, fp0, fu0, fv0);
            if (!pery) {
                fold_values2<T>(g, bc, xw, 0, fx1, fp1, fu1, fv1);
                fold_values2<T>(g, bc, xw, ny - 1, fx2, fp2, fu2, fv2);
            }
        }
        const T w0 = T(4.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
        const T A2 = T(2) * A;
        const int nit = Yb - Ya + 2;  // iterations r = Ya-1 .. Yb

// face class of a wrapped row (0 interior, 1 low face, 2 high face of a non-periodic y)
#define C2_YCLS(yw) (pery ? 0 : ((yw) == 0 ? 1 : ((yw) == ny - 1 ? 2 : 0)))
// p, u of row r into (p, u, v): rows Ya-2 .. Yb+1 are read (the f_i of rows Ya-1 .. Yb);
// a row off the grid reads a row on it, for the same reason as the columns; with fold a
// face row reads the interior row it copies
#define C2_LOAD(r, p, u, v)                                                          \
    do {                                                                             \
        const int r_ = (r);                                                          \
        if (r_ >= Ya - 2 && r_ <= Yb + 1) {                                          \
            int yw_ = r_;                                                            \
            if (!wrap_coord(yw_, ny, pery)) yw_ = r_ < 0 ? 0 : ny - 1;               \
            const int yc_ = C2_YCLS(yw_);                                            \
            const int yl_ = (fold && yc_) ? (yc_ == 1 ? 1 : ny - 2) : yw_;           \
            const T *rp_ = sin_ + (size_t)yl_ * (size_t)nx;                          \
            (p) = rp_[xl];                                                           \
            (u) = rp_[N + xl];                                                       \
            (v) = rp_[2 * N + xl];                                                   \
        }                                                                            \
    } while (0)
// the prescribed values of row r replace what its nodes' faces fix (fold)
#define C2_FIX(r, p, u, v)                                                           \
    do {                                                                             \
        int yw_ = (r);                                                               \
        if (fold && wrap_coord(yw_, ny, pery)) {                                     \
            const int yc_ = C2_YCLS(yw_);                                            \
            if (yc_ != 0 || wave_xb) {                                               \
                const bool s1_ = yc_ == 1, s2_ = yc_ == 2;                           \
                const int m_ = s1_ ? fx1 : (s2_ ? fx2 : fx0);                        \
                (p) = (m_ & 1) ? (s1_ ? fp1 : (s2_ ? fp2 : fp0)) : (p);              \
                (u) = (m_ & 2) ? (s1_ ? fu1 : (s2_ ? fu2 : fu0)) : (u);              \
                (v) = (m_ & 2) ? (s1_ ? fv1 : (s2_ ? fv2 : fv0)) : (v);              \
            }                                                                        \
        }                                                                            \
    } while (0)

        T P[8], U[8], V[8];     // rows, slot (q - Ya + 3) & 7
        T AP[8], AX[8], AY[8];  // moments being gathered, same slots
#pragma unroll
        for (int k = 0; k < 8; k++) {
            AP[k] = AX[k] = AY[k] = T(0);
            P[k] = U[k] = V[k] = T(0);
            C2_LOAD(Ya - 3 + k, P[k], U[k], V[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) C2_FIX(Ya - 3 + k, P[k], U[k], V[k]);

// Iteration r = Ya - 1 + i0 + J. BULK: every row it touches (r-1 .. r+6) lies inside the
// run, off the y faces and the periodic seam: no row checks, only the x-face values.
#define C2_STEP(J, BULK)                                                                            \
    {                                                                                               \
        constexpr int m2 = (J) & 7, m1 = ((J) + 1) & 7, c0 = ((J) + 2) & 7, p1 = ((J) + 3) & 7,      \
                      p2 = ((J) + 4) & 7;                                                           \
        const int r = Ya - 1 + i0 + (J);                                                            \
        int yc = 0;                                                                                 \
        if (BULK) {                                                                                 \
            if (fold && wave_xb) {                                                                  \
                P[p2] = (fx0 & 1) ? fp0 : P[p2];                                                    \
                U[p2] = (fx0 & 2) ? fu0 : U[p2];                                                    \
                V[p2] = (fx0 & 2) ? fv0 : V[p2];                                                    \
            }                                                                                       \
        } else {                                                                                    \
            C2_FIX(r + 2, P[p2], U[p2], V[p2]);                                                     \
            int yw = r;                                                                             \
            yc = wrap_coord(yw, ny, pery) ? C2_YCLS(yw) : 0;                                        \
        }                                                                                           \
        /* S_ab = d_a u_b: along x from the neighbouring lanes, along y from the rows */           \
        const T u = U[c0], v = V[c0];                                                               \
        const T uL = from_left(u), uR = from_right(u), vL = from_left(v), vR = from_right(v);       \
        T dxu = T(0.5) * (uR - uL), dxv = T(0.5) * (vR - vL);                                       \
        if (wave_xb) {                                                                              \
            /* one-sided on the end columns of a non-periodic x axis; the lanes two away are       \
               read with every lane active (DPP reads zero from inactive lanes) */                  \
            const T uRR = from_right(uR), vRR = from_right(vR), uLL = from_left(uL),                \
                    vLL = from_left(vL);                                                            \
            if (xcls == 1) {                                                                        \
                dxu = T(0.5) * (T(-3) * u + T(4) * uR - uRR);                                       \
                dxv = T(0.5) * (T(-3) * v + T(4) * vR - vRR);                                       \
            } else if (xcls == 2) {                                                                 \
                dxu = T(0.5) * (T(3) * u - T(4) * uL + uLL);                                        \
                dxv = T(0.5) * (T(3) * v - T(4) * vL + vLL);                                        \
            }                                                                                       \
        }                                                                                           \
        T dyu, dyv;                                                                                 \
        if (yc == 0) {                                                                              \
            dyu = T(0.5) * (U[p1] - U[m1]);                                                         \
            dyv = T(0.5) * (V[p1] - V[m1]);                                                         \
        } else if (yc == 1) {                                                                       \
            dyu = T(0.5) * (T(-3) * u + T(4) * U[p1] - U[p2]);                                      \
            dyv = T(0.5) * (T(-3) * v + T(4) * V[p1] - V[p2]);                                      \
        } else {                                                                                    \
            dyu = T(0.5) * (T(3) * u - T(4) * U[m1] + U[m2]);                                       \
            dyv = T(0.5) * (T(3) * v - T(4) * V[m1] + V[m2]);                                       \
        }                                                                                           \
        /* df_i = w_i (3p - 3 U.v - 3/2 v.v + 3 c.v + 9 (c.U)(c.v) + 9/2 (c.v)^2                    \
           + A c.(S + S^T).c) (u, v hold the deviation), formed for the pairs +-c at once: the      \
           even part is shared, the odd part 3 w c.v changes sign; evaluated on every lane (off     \
           the grid the values reach no written node) */                                            \
        const T base = T(3) * P[c0] - T(1.5) * (u * u + v * v) - T(3) * (Ux * u + Uy * v);          \
        const T axx = A2 * dxu, ayy = A2 * dyv, axy = A2 * (dxv + dyu);                             \
        const T f0 = w0 * base;                                                                     \
        const T e12 = w1 * (base + (T(9) * Ux + T(4.5) * u) * u + axx), o12 = T(3) * w1 * u;        \
        const T e34 = w1 * (base + (T(9) * Uy + T(4.5) * v) * v + ayy), o34 = T(3) * w1 * v;        \
        const T bd = base + axx + ayy;                                                              \
        const T cu56 = u + v, cu78 = u - v;                                                         \
        const T e56 = w2 * (bd + (T(9) * (Ux + Uy) + T(4.5) * cu56) * cu56 + axy),                  \
                o56 = T(3) * w2 * cu56;                                                             \
        const T e78 = w2 * (bd + (T(9) * (Ux - Uy) + T(4.5) * cu78) * cu78 - axy),                  \
                o78 = T(3) * w2 * cu78;                                                             \
        /* push: f_i of this node reaches node (x + c_ix, r + c_iy) */                              \
        const T a1 = from_left(e12 + o12), a2 = from_right(e12 - o12); /* row r */                 \
        const T a5 = from_left(e56 + o56), a8 = from_right(e78 - o78); /* row r+1 */               \
        const T a7 = from_left(e78 + o78), a6 = from_right(e56 - o56); /* row r-1 */               \
        const T s0 = f0 + (a1 + a2), sp = (e34 + o34) + (a5 + a8), sm = (e34 - o34) + (a6 + a7);    \
        AP[p1] = sp;                                                                                \
        AX[p1] = a5 - a8;                                                                           \
        AY[p1] = sp;                                                                                \
        AP[c0] += s0;                                                                               \
        AX[c0] += a1 - a2;                                                                          \
        AP[m1] += sm;                                                                               \
        AX[m1] += a7 - a6;                                                                          \
        AY[m1] -= sm;                                                                               \
        /* row r-1 is complete */                                                                   \
        const int yo = r - 1;                                                                       \
        if (((BULK) || (yo >= Ya && yo < Yb && C2_YCLS(yo) == 0)) && outc) {                         \
            T *op = sout + (size_t)yo * (size_t)nx + (unsigned)x;                                   \
            op[0] = AP[m1] * T(1.0 / 3.0);                                                          \
            op[N] = AX[m1];                                                                         \
            op[2 * N] = AY[m1];                                                                     \
        }                                                                                           \
        /* row r-2 is no longer needed: its slot takes row r+6 */                                   \
        if (BULK) {                                                                                 \
            const T *rp = sin_ + (size_t)(r + 6) * (size_t)nx;                                      \
            P[m2] = rp[xl];                                                                         \
            U[m2] = rp[N + xl];                                                                     \
            V[m2] = rp[2 * N + xl];                                                                 \
        } else {                                                                                    \
            C2_LOAD(r + 6, P[m2], U[m2], V[m2]);                                                    \
        }                                                                                           \
    }

        // Groups of 8 iterations (the slots follow the iteration index mod 8) whose rows
        // r-1 .. r+6 all lie in [lo, hi] run in bulk.
        const int lo = max(Ya, 1), hi = min(Yb + 1, ny - 2);
        for (int i0 = 0; i0 < nit; i0 += 8) {
            const int rf = Ya - 1 + i0;
            if (i0 + 8 <= nit && rf - 1 >= lo && rf + 13 <= hi) {
                C2_STEP(0, true) C2_STEP(1, true) C2_STEP(2, true) C2_STEP(3, true)
                C2_STEP(4, true) C2_STEP(5, true) C2_STEP(6, true) C2_STEP(7, true)
            } else {
                C2_STEP(0, false) if (i0 + 1 < nit) {
                    C2_STEP(1, false) if (i0 + 2 < nit) {
                        C2_STEP(2, false) if (i0 + 3 < nit) {
                            C2_STEP(3, false) if (i0 + 4 < nit) {
                                C2_STEP(4, false) if (i0 + 5 < nit) {
                                    C2_STEP(5, false) if (i0 + 6 < nit) {
                                        C2_STEP(6, false) if (i0 + 7 < nit) { C2_STEP(7, false) }
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
#undef C2_STEP
#undef C2_FIX
#undef C2_LOAD
#undef C2_YCLS
    }
    if (SP) span_end(ts);
}

// ===================================================================== forward, 2D: tiles
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
// 2.5D blocking. A block of TX x TY threads (one wave per row of 64 columns) is the tile
// of source columns (x, y) whose f_i it evaluates, one column per thread; it writes the
// columns of lanes 2 .. 61 of rows 1 .. TY-2 and marches along z over ZC output planes.
// Per source plane s each thread evaluates the 15 f_i of its node into LDS and pushes
// them (by the gather of its output column) to the destination planes s-1, s, s+1, whose
// moments it keeps in registers. The thread's own column of p, u for planes s-2..s+2
// lives in registers, loaded three planes ahead. The x derivatives take u from the
// neighbouring lanes (DPP shifts: the tile needs no ring columns, whose loads would each
// fetch a cache line for one value); u of plane s with a ring of two rows is staged in
// LDS for the y derivatives. The march is unrolled six planes deep, so the plane ring
// (six slots) and the destination ring (three) are addressed by constants. Derivatives
// are central; the second-order one-sided forms at the nodes of a non-periodic wall are
// applied in branches that are uniform over a wave (a y-wall row, a tile holding an
// x-wall column) or over the block (a z-wall plane). Loads and stores go through buffer
// resources: a lane off the grid reads zeros and writes nothing.
template <typename T> struct G3 {
    static constexpr int TX = 64, TY = 12, NT = TX * TY;
    static constexpr int OX = TX - 4, OY = TY - 2;  // output tile: lanes 2 .. 61, rows 1 .. TY-2
    static constexpr int WY = TY + 2;               // staged u plane: the tile's rows and one more each side
    static constexpr int RING = 2 * TX;             // staged nodes outside the tile (two rows)
};

// Component c of plane p of a field of N-node components, read at the byte offset `off`
// within the plane (zeros when p is off the grid). WHOLE (the field's bytes stay below
// BOFF_NONE, checked on the host): `rw` is one resource over the whole field, set up
// once per kernel, and the component and plane are chosen by the scalar offset; a plane
// off the grid switches every lane off through its vector offset. Otherwise a resource
// per plane of `base` (a plane's bytes stay below BOFF_NONE, checked on the host).
template <typename T, bool WHOLE>
__device__ __forceinline__ T pload(const T *base, __amdgpu_buffer_rsrc_t rw, long long N, int c, int p, int nz,
                                   int pz, unsigned plane, unsigned off) {
    int zw = p;
    const bool ok = wrap_coord(zw, nz, pz);
    if (WHOLE)
        return bload<T>(rw, ok ? off : BOFF_NONE,
                        ((unsigned)c * (unsigned)N + (unsigned)(ok ? zw : 0) * plane) * (unsigned)sizeof(T));
    return bload<T>(brsrc(base + (long long)c * N + (long long)(ok ? zw : 0) * plane,
                          ok ? plane * (unsigned)sizeof(T) : 0u),
                    off);
}
// Store to component c of plane p (on the grid) at the byte offset `off` within it.
template <typename T, bool WHOLE>
__device__ __forceinline__ void pstore(T v, T *base, __amdgpu_buffer_rsrc_t rw, long long N, int c, int p,
                                       unsigned plane, unsigned off) {
    if (WHOLE)
        bstore(v, rw, off, ((unsigned)c * (unsigned)N + (unsigned)p * plane) * (unsigned)sizeof(T));
    else
        bstore(v, brsrc(base + (long long)c * N + (long long)p * plane, plane * (unsigned)sizeof(T)), off);
}
// The whole-field resource of a field of nc components (WHOLE only).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const T *base, long long N, int nc) {
    return brsrc(base, (unsigned)nc * (unsigned)N * (unsigned)sizeof(T));
}

// Second-order one-sided doubled derivatives at the first (lo) and last (hi) node of a
// non-periodic axis: c the node, p1, p2 (m1, m2) the next (previous) nodes along the axis.
template <typename T> __device__ __forceinline__ T d2_lo(T c, T p1, T p2) { return T(-3) * c + T(4) * p1 - p2; }
template <typename T> __device__ __forceinline__ T d2_hi(T c, T m1, T m2) { return T(3) * c - T(4) * m1 + m2; }

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

template <typename T, bool SP, bool WHOLE>
__global__ __launch_bounds__(G3<T>::NT, sizeof(T) == 4 ? 6 : 2) void k_gather3d(Grid g, T A, FeqU<T> fu, int ZC,
                                                        const T *__restrict__ sin_, T *__restrict__ sout,
                                                        unsigned long long *ts) {
    using G = G3<T>;
    constexpr int TX = G::TX, TY = G::TY, WY = G::WY;
    // u of plane s for the y derivatives (one buffer: its readers pass the second barrier
    // of a plane before anyone stages the next one)
    __shared__ T wu[3][WY][TX];
    __shared__ T fb[15][TY][TX];
    if (SP) span_begin(ts);
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int px = g.per[0], py = g.per[1], pz = g.per[2];
    const uint3 tb = xcd_tile();
    const int x0 = tb.x * G::OX, y0 = tb.y * G::OY;
    const int z0 = tb.z * ZC, z1 = min(z0 + ZC, nz);
    // a wave is one row of the tile: ty is uniform over it
    const int tx = threadIdx.x, ty = __builtin_amdgcn_readfirstlane(threadIdx.y), tid = tx + TX * ty;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const __amdgpu_buffer_rsrc_t rin = field_rsrc(sin_, N, 4), rout = field_rsrc(sout, N, 4);

    // this thread's source column (x0 - 2 + tx, y0 - 1 + ty); the x neighbours of a node
    // are the neighbouring lanes of its wave, so the tile needs no ring columns
    int cx = x0 - 2 + tx, cy = y0 - 1 + ty;
    const bool colok = wrap_coord(cx, nx, px) && wrap_coord(cy, ny, py);
    const unsigned coff = colok ? ((unsigned)cx + (unsigned)nx * (unsigned)cy) * (unsigned)sizeof(T) : BOFF_NONE;
    // ring node of the staged plane handled by this thread (waves 0 and 1: the rows
    // y0 - 2 and y0 + TY - 1 of the tile's columns)
    const bool ring = tid < G::RING;
    const int ry = tid < TX ? 0 : WY - 1;
    int gx = x0 - 2 + tx, gy = ry == 0 ? y0 - 2 : y0 + TY - 1;
    const bool ringok = ring && wrap_coord(gx, nx, px) && wrap_coord(gy, ny, py);
    const unsigned roff = ringok ? ((unsigned)gx + (unsigned)nx * (unsigned)gy) * (unsigned)sizeof(T) : BOFF_NONE;
    // output node: the thread's own node for lanes 2 .. 61 and rows 1 .. TY-2, written
    // when it is an interior node of the x-y plane
    // (unwrapped: on a periodic axis a node past the end belongs to the first tile)
    const int ox = x0 - 2 + tx, oy = y0 - 1 + ty;
    const bool outrow = ty >= 1 && ty <= G::OY;
    const bool outlane = tx >= 2 && tx < 2 + G::OX;
    const bool outok = outlane && outrow && ox < nx && oy < ny && !(!px && (ox == 0 || ox == nx - 1)) &&
                       !(!py && (oy == 0 || oy == ny - 1));
    const unsigned ooff = outok ? ((unsigned)ox + (unsigned)nx * (unsigned)oy) * (unsigned)sizeof(T) : BOFF_NONE;
    // one-sided derivatives: the tile holds an x-wall column (block-uniform), the lane's
    // column is one (1 first, 2 last), the wave's row is a y-wall row (wave-uniform)
    const bool xw = !px && (x0 - 2 <= 0 || x0 + TX - 3 >= nx - 1);
    const T xlo = (!px && colok && cx == 0) ? T(1) : T(0), xhi = (!px && colok && cx == nx - 1) ? T(1) : T(0);
    const int ys = (!py && cy >= 0 && cy < ny) ? (cy == 0 ? 1 : (cy == ny - 1 ? 2 : 0)) : 0;

    T q[6][4];  // own column: plane s + k in slot (J + k + 2) mod 6 at unrolled step J
#pragma unroll
    for (int j = 0; j < 5; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) q[j][c] = pload<T, WHOLE>(sin_, rin, N, c, z0 - 3 + j, nz, pz, plane, coff);
    T rv[3];  // ring node of plane s (reloaded with plane s + 1 once staged)
    if (ring) {
#pragma unroll
        for (int c = 0; c < 3; c++) rv[c] = pload<T, WHOLE>(sin_, rin, N, 1 + c, z0 - 1, nz, pz, plane, roff);
    }
    T acc[3][4];  // destination plane s + k in slot (J + k + 1) mod 3
#pragma unroll
    for (int k = 0; k < 3; k++) acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = T(0);

    const int nsteps = z1 - z0 + 2;  // source planes z0 - 1 .. z1
    for (int jb = 0; jb < nsteps; jb += 6) {
#pragma unroll
        for (int J = 0; J < 6; J++) {
            if (jb + J < nsteps) {
            const int s = z0 - 1 + jb + J;
            const int qm2 = J % 6, qm1 = (J + 1) % 6, qc = (J + 2) % 6, qp1 = (J + 3) % 6, qp2 = (J + 4) % 6,
                      qp3 = (J + 5) % 6;
            // stage u of plane s: own node and ring node
#pragma unroll
            for (int c = 0; c < 3; c++) wu[c][ty + 1][tx] = q[qc][1 + c];
            if (ring) {
#pragma unroll
                for (int c = 0; c < 3; c++) wu[c][ry][tx] = rv[c];
            }
            // next planes in flight while this one is evaluated: the ring node first (it is
            // staged at the next plane, and the wait for it must not drain the own column's
            // loads, which run three planes ahead)
            if (s + 1 <= z1 && ring) {
#pragma unroll
                for (int c = 0; c < 3; c++)
                    rv[c] = pload<T, WHOLE>(sin_, rin, N, 1 + c, s + 1, nz, pz, plane, roff);
            }
            if (s + 3 <= z1 + 2) {
#pragma unroll
                for (int c = 0; c < 4; c++) q[qp3][c] = pload<T, WHOLE>(sin_, rin, N, c, s + 3, nz, pz, plane, coff);
            }
            __syncthreads();

            // Sources off the grid (non-periodic axes) only feed boundary nodes, which this
            // kernel does not write; their f_i are evaluated from zeros and never used.
            int zs = s;
            (void)wrap_coord(zs, nz, pz);
            T f[15];
            {
                const int ly = ty + 1;
                T D[3][3];  // D[a][b] = 2 d_a u_b
                T um[3], up[3];  // u at the lanes on either side (every lane active here)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    um[c] = from_left(q[qc][1 + c]);
                    up[c] = from_right(q[qc][1 + c]);
                }
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    D[0][c] = up[c] - um[c];
                    D[1][c] = wu[c][ly + 1][tx] - wu[c][ly - 1][tx];
                    D[2][c] = q[qp1][1 + c] - q[qm1][1 + c];
                }
                if (xw) {  // blend in the one-sided form on the wall lane (weights 0 or 1)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const T m2 = from_left(um[c]), p2 = from_right(up[c]);
                        const T lo = d2_lo(q[qc][1 + c], up[c], p2), hi = d2_hi(q[qc][1 + c], um[c], m2);
                        D[0][c] = D[0][c] + xlo * (lo - D[0][c]) + xhi * (hi - D[0][c]);
                    }
                }
                if (ys) {
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const T(*U)[TX] = wu[c];
                        D[1][c] = ys == 1 ? d2_lo(U[ly][tx], U[ly + 1][tx], U[ly + 2 >= WY ? WY - 1 : ly + 2][tx])
                                          : d2_hi(U[ly][tx], U[ly - 1][tx], U[ly - 2 < 0 ? 0 : ly - 2][tx]);
                    }
                }
                if (!pz && (zs == 0 || zs == nz - 1)) {
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        D[2][c] = zs == 0 ? d2_lo(q[qc][1 + c], q[qp1][1 + c], q[qp2][1 + c])
                                          : d2_hi(q[qc][1 + c], q[qm1][1 + c], q[qm2][1 + c]);
                }
                const T u[3] = {q[qc][1], q[qc][2], q[qc][3]};
                feq3(q[qc][0], u, fu, D, A, f);
            }
#pragma unroll
            for (int i = 0; i < 15; i++) fb[i][ty][tx] = f[i];
            __syncthreads();

            if (outrow && outlane) {
                const int km = J % 3, k0 = (J + 1) % 3, kp = (J + 2) % 3;
#pragma unroll
                for (int c = 0; c < 4; c++) acc[kp][c] = T(0);
#pragma unroll
                for (int i = 0; i < 15; i++) {
                    const int ex = Lat<3>::c(i, 0), ey = Lat<3>::c(i, 1), ez = Lat<3>::c(i, 2);
                    const int k = ez < 0 ? km : (ez == 0 ? k0 : kp);
                    const T v = fb[i][ty - ey][tx - ex];
                    acc[k][0] += v;
                    if (ex) acc[k][1] += T(ex) * v;
                    if (ey) acc[k][2] += T(ey) * v;
                    if (ez) acc[k][3] += T(ez) * v;
                }
                // destination plane s - 1 has received all its sources
                const int zd = s - 1;
                if (zd >= z0 && zd < z1 && !(!pz && (zd == 0 || zd == nz - 1))) {
                    pstore<T, WHOLE>(acc[km][0] * T(1.0 / 3.0), sout, rout, N, 0, zd, plane, ooff);
#pragma unroll
                    for (int a = 0; a < 3; a++) pstore<T, WHOLE>(acc[km][1 + a], sout, rout, N, 1 + a, zd, plane, ooff);
                }
            }
            }
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

// ===================================================================== adjoint, 2D: column march
// Column march like the forward (large grids; k_adjgather2d below serves the others): lane l of a wave holds column x0 - 2 + l (x0 = 60 s -
// off), the wave writes columns x0 .. x0+59 of a run of `rows` rows and marches along y
// with no LDS and no barriers. Per row r the lane forms the cotangent g of the
// post-streaming moments (p*bar / 3, u*bar; zero off the interior) from the raw adjoint
// state (the fold of the boundary copies by DPP shifts and the neighbouring rows, u*bar
// from ustb inside the body box), the moments (pi, ups, sig) of row r from g rows r-1 ..
// r+1, the part of the outputs of row r that needs only row r (with the x transpose of
// the gradient through the neighbouring lanes), and completes row r-2 with the y
// transpose from sig rows r-4 .. r. Rows live in rings of 8 register slots (row q in
// slot (q - Ya + 4) mod 8), the loop unrolled by 8 so the slots are compile-time
// constants; the raw rows are loaded 4 iterations ahead. off = 1 where a strip edge
// would cut the two-lane reach of the one-sided transpose next to a non-periodic x face.
constexpr int A2_W = 60, A2_NT = 256;

// Coefficients with which sig at offsets -2 .. 2 along an axis enters D^T sig at
// coordinate z (the transpose of the boundary-aware difference; dT_stencil's values).
template <typename T>
__device__ __forceinline__ void dT_coef(int z, int n, int per, T &cm2, T &cm1, T &c0, T &cp1, T &cp2) {
    if (per) {
        cm2 = c0 = cp2 = T(0);
        cm1 = T(0.5);
        cp1 = T(-0.5);
        return;
    }
    cm1 = z - 1 >= 0 ? (z - 1 == 0 ? T(2) : T(0.5)) : T(0);
    cp1 = z + 1 <= n - 1 ? (z + 1 == n - 1 ? T(-2) : T(-0.5)) : T(0);
    c0 = (z == 0 ? T(-1.5) : T(0)) + (z == n - 1 ? T(1.5) : T(0));
    cm2 = z - 2 == 0 ? T(-0.5) : T(0);
    cp2 = z + 2 == n - 1 ? T(0.5) : T(0);
}

// p fixed (bit 0) / u fixed (bit 1) at boundary node (x, y)
__device__ __forceinline__ int fix_mask2(const Grid &g, const Bc &bc, int x, int y) {
    const int xx[3] = {x, y, 0};
    BcNode b;
    bc_resolve<2>(g, bc, xx, b);
    return (b.p_fixed ? 1 : 0) | (b.u_fixed ? 2 : 0);
}

template <typename T, bool SP>
__global__ __launch_bounds__(A2_NT) void k_adjgather2d_march(Grid g, Bc bc, T A, int rows, int nstrip, int nwave, int off,
                                                       const T *__restrict__ ab, const T *__restrict__ ustb,
                                                       const double *__restrict__ Bprev, Design D, int has_box,
                                                       const T *__restrict__ sprev, T *__restrict__ out,
                                                       unsigned long long *ts, T *__restrict__ ups) {
    if (SP) span_begin(ts);
    const int nx = g.n[0], ny = g.n[1], perx = g.per[0], pery = g.per[1];
    const long long N = g.N;
    const T Ux = gU<T>(g, 0), Uy = gU<T>(g, 1);
    const int lane = threadIdx.x & 63;
    const int wv = (int)xcd_block() * (A2_NT / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wv < nwave) {
        const int strip = __builtin_amdgcn_readfirstlane(wv % nstrip);
        const int run = __builtin_amdgcn_readfirstlane(wv / nstrip);
        const int x0 = strip * A2_W - off, Ya = run * rows, Yb = min(Ya + rows, ny);
        // the body box (rows and columns of the box nodes, from the pose at t-1)
        int bo0 = 0, bo1 = 0, bl0 = 0, bl1 = 0;
        if (has_box) {
            int o[3];
            box_origin<2>(D, Bprev, o);
            bo0 = __builtin_amdgcn_readfirstlane(o[0]);
            bo1 = __builtin_amdgcn_readfirstlane(o[1]);
            bl0 = D.L[0];
            bl1 = D.L[1];
        }
        const long long bN = D.boxN;
        // this lane's column (lanes off the grid read column 0 or nx-1; g is zero there)
        const int x = x0 - 2 + lane;
        int xw = x;
        const bool colok = wrap_coord(xw, nx, perx);
        if (!colok) xw = x < 0 ? 0 : nx - 1;
        const bool xint = colok && (perx || (xw >= 1 && xw <= nx - 2));
        const unsigned xo = (unsigned)xw;
        const bool wave_xb = !perx && (x0 - 2 <= 1 || x0 + 61 >= nx - 2);
        const bool outc = lane >= 2 && lane < 2 + A2_W && x >= 0 && x < nx;
        const bool xbox = has_box && xint && xw - bo0 >= 0 && xw - bo0 < bl0;  // interior box column
        // fold of the boundary copies (transpose of the boundary treatment): which of the
        // neighbouring boundary nodes copy this node, and whether their p / u are free
        const bool isx1 = !perx && xw == 1, isxn = !perx && xw == nx - 2;
        const int mxl = perx ? 3 : fix_mask2(g, bc, 0, pery ? 0 : 1);
        const int mxh = perx ? 3 : fix_mask2(g, bc, nx - 1, pery ? 0 : 1);
        const int myl = pery ? 3 : fix_mask2(g, bc, perx ? 0 : 1, 0);
        const int myh = pery ? 3 : fix_mask2(g, bc, perx ? 0 : 1, ny - 1);
        const int mll = (perx || pery) ? 3 : fix_mask2(g, bc, 0, 0);
        const int mhl = (perx || pery) ? 3 : fix_mask2(g, bc, nx - 1, 0);
        const int mlh = (perx || pery) ? 3 : fix_mask2(g, bc, 0, ny - 1);
        const int mhh = (perx || pery) ? 3 : fix_mask2(g, bc, nx - 1, ny - 1);
        // per-lane weights of the x fold: the left / right neighbour is a boundary node
        // copying this one on rows off the y faces, and its p / u are free there
        const T fLp = (isx1 && !(mxl & 1)) ? T(1) : T(0), fLu = (isx1 && !(mxl & 2)) ? T(1) : T(0);
        const T fRp = (isxn && !(mxh & 1)) ? T(1) : T(0), fRu = (isxn && !(mxh & 2)) ? T(1) : T(0);
        // x transpose of the gradient at this column
        T xm2, xm1, x00, xp1, xp2;
        dT_coef<T>(xw, nx, perx, xm2, xm1, x00, xp1, xp2);
        const T w0 = T(4.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
        const T A2 = T(2) * A;
        const int nit = Yb - Ya + 4;  // iterations r = Ya-2 .. Yb+1

#define A2_INT(yw) (pery || ((yw) >= 1 && (yw) <= ny - 2))
// raw adjoint state of row r: rows Ya-4 .. Yb+3 are read, a row off the grid reads a
// row on it (its g is zero); inside the body box u*bar comes from ustb
#define A2_LOAD(r, p, u, v)                                                          \
    do {                                                                             \
        const int r_ = (r);                                                          \
        if (r_ >= Ya - 4 && r_ <= Yb + 3) {                                          \
            int yw_ = r_;                                                            \
            if (!wrap_coord(yw_, ny, pery)) yw_ = r_ < 0 ? 0 : ny - 1;               \
            const T *rp_ = ab + (size_t)yw_ * (size_t)nx;                            \
            (p) = rp_[xo];                                                           \
            const int by_ = yw_ - bo1;                                               \
            if (has_box && by_ >= 0 && by_ < bl1 && A2_INT(yw_)) {                   \
                if (xbox) {                                                          \
                    const T *bp_ = ustb + (size_t)by_ * (size_t)bl0 + (xw - bo0);    \
                    (u) = bp_[0];                                                    \
                    (v) = bp_[bN];                                                   \
                } else {                                                             \
                    (u) = rp_[N + xo];                                               \
                    (v) = rp_[2 * N + xo];                                           \
                }                                                                    \
            } else {                                                                 \
                (u) = rp_[N + xo];                                                   \
                (v) = rp_[2 * N + xo];                                               \
            }                                                                        \
        }                                                                            \
    } while (0)
#define A2_SPREV(r, a, b)                                                            \
    do {                                                                             \
        const int r_ = (r);                                                          \
        if (r_ >= Ya && r_ < Yb) {                                                   \
            const T *rp_ = sprev + (size_t)r_ * (size_t)nx;                          \
            (a) = rp_[N + xo];                                                       \
            (b) = rp_[2 * N + xo];                                                   \
        }                                                                            \
    } while (0)

        T RP[8], RU[8], RV[8];     // raw rows, slot (q - Ya + 4) & 7
        T GP[8], GU[8], GV[8];     // g rows
        T S0[8], S1[8];            // forward velocity at t-1 (deviation)
        T MXY[8], MYY[8];          // sig_xy, sig_yy rows
        T OP[8], OX[8], OY[8];     // outputs being completed
        T QX[8], QY[8];            // the moment ups (for the paper's variant)
#pragma unroll
        for (int k = 0; k < 8; k++) {
            RP[k] = RU[k] = RV[k] = GP[k] = GU[k] = GV[k] = T(0);
            S0[k] = S1[k] = MXY[k] = MYY[k] = OP[k] = OX[k] = OY[k] = QX[k] = QY[k] = T(0);
            A2_LOAD(Ya - 4 + k, RP[k], RU[k], RV[k]);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) A2_SPREV(Ya - 2 + k, S0[k + 2], S1[k + 2]);

// fold of a y-face row (raw values bp, bu, bv) into the row it copies: the node below /
// above, and the corner nodes beside it (masks my: face, ml / mh: the low / high x corner)
#define A2_YFOLD(bp, bu, bv, my, ml, mh)                                                            \
    {                                                                                               \
        const T bp_ = (bp), bu_ = (bu), bv_ = (bv);                                                 \
        const T yp_ = ((my) & 1) ? T(0) : T(1), yu_ = ((my) & 2) ? T(0) : T(1);                     \
        gp_ += yp_ * bp_;                                                                           \
        gu_ += yu_ * bu_;                                                                           \
        gv_ += yu_ * bv_;                                                                           \
        if (wave_xb) {                                                                              \
            const T lp_ = from_left(bp_), rq_ = from_right(bp_);                                    \
            const T lu_ = from_left(bu_), ru_ = from_right(bu_);                                    \
            const T lv_ = from_left(bv_), rv_ = from_right(bv_);                                    \
            const T cLp_ = (isx1 && !((ml) & 1)) ? T(1) : T(0), cLu_ = (isx1 && !((ml) & 2)) ? T(1) : T(0); \
            const T cRp_ = (isxn && !((mh) & 1)) ? T(1) : T(0), cRu_ = (isxn && !((mh) & 2)) ? T(1) : T(0); \
            gp_ += cLp_ * lp_ + cRp_ * rq_;                                                         \
            gu_ += cLu_ * lu_ + cRu_ * ru_;                                                         \
            gv_ += cLu_ * lv_ + cRu_ * rv_;                                                         \
        }                                                                                           \
    }
// g of row q (slot c) from the raw rows q-1 (slot m), q, q+1 (slot p): the raw values of
// an interior node plus, next to a non-periodic face, those of the boundary nodes that
// copy it (where they are not prescribed); zero off the interior
#define A2_G(q, m, c, p)                                                                            \
    {                                                                                               \
        int yw_ = (q);                                                                              \
        const bool rowok_ = wrap_coord(yw_, ny, pery);                                              \
        const bool yint_ = rowok_ && A2_INT(yw_);                                                   \
        T gp_ = RP[c], gu_ = RU[c], gv_ = RV[c];                                                    \
        if (wave_xb) {                                                                              \
            const T lp_ = from_left(RP[c]), rp_ = from_right(RP[c]);                                \
            const T lu_ = from_left(RU[c]), ru_ = from_right(RU[c]);                                \
            const T lv_ = from_left(RV[c]), rv_ = from_right(RV[c]);                                \
            gp_ += fLp * lp_ + fRp * rp_;                                                           \
            gu_ += fLu * lu_ + fRu * ru_;                                                           \
            gv_ += fLu * lv_ + fRu * rv_;                                                           \
        }                                                                                           \
        /* the rows on the y faces that copy this one, and their corners */                         \
        if (!pery && yw_ == 1) A2_YFOLD(RP[m], RU[m], RV[m], myl, mll, mhl)                         \
        if (!pery && yw_ == ny - 2) A2_YFOLD(RP[p], RU[p], RV[p], myh, mlh, mhh)                    \
        /* inside the body box u*bar is ustb itself (no fold) */                                    \
        const int by_ = yw_ - bo1;                                                                  \
        if (has_box && by_ >= 0 && by_ < bl1 && yint_ && xbox) {                                    \
            gu_ = RU[c];                                                                            \
            gv_ = RV[c];                                                                            \
        }                                                                                           \
        const bool in_ = yint_ && xint;                                                             \
        GP[c] = in_ ? gp_ * T(1.0 / 3.0) : T(0);                                                    \
        GU[c] = in_ ? gu_ : T(0);                                                                   \
        GV[c] = in_ ? gv_ : T(0);                                                                   \
    }

        // g rows Ya-3, Ya-2 (the first iteration forms row Ya-1)
        A2_G(Ya - 3, 0, 1, 2)
        A2_G(Ya - 2, 1, 2, 3)

// Iteration r = Ya - 2 + i0 + J (slot of row r + k: (J + 2 + k) & 7).
#define A2_STEP(J)                                                                                  \
    {                                                                                               \
        constexpr int sm4 = ((J) + 6) & 7, sm2 = (J) & 7, sm1 = ((J) + 1) & 7, s0 = ((J) + 2) & 7,   \
                      sp1 = ((J) + 3) & 7, sp2 = ((J) + 4) & 7, sp3 = ((J) + 5) & 7;                \
        constexpr int sm3 = ((J) + 7) & 7;                                                          \
        const int r = Ya - 2 + i0 + (J);                                                            \
        A2_G(r + 1, s0, sp1, sp2)                                                                   \
        /* moments of row r: g_i = (p*bar/3 + c_i.u*bar)(x + c_i), sum_i w_i g_i (1, c, cc) */      \
        const T g0 = GP[s0];                                                                        \
        const T g1 = from_right(GP[s0] + GU[s0]), g2 = from_left(GP[s0] - GU[s0]);                  \
        const T g3 = GP[sp1] + GV[sp1], g4 = GP[sm1] - GV[sm1];                                     \
        const T g5 = from_right(GP[sp1] + GU[sp1] + GV[sp1]);                                       \
        const T g8 = from_left(GP[sp1] - GU[sp1] + GV[sp1]);                                        \
        const T g6 = from_left(GP[sm1] - GU[sm1] - GV[sm1]);                                        \
        const T g7 = from_right(GP[sm1] + GU[sm1] - GV[sm1]);                                       \
        const T e1 = g1 + g2, e2 = g3 + g4, s56 = g5 + g6, s78 = g7 + g8, d56 = g5 - g6,            \
                d78 = g7 - g8;                                                                      \
        const T dd = w2 * (s56 + s78);                                                              \
        const T pi = w0 * g0 + w1 * (e1 + e2) + dd;                                                 \
        const T mux = w1 * (g1 - g2) + w2 * (d56 + d78);                                            \
        const T muy = w1 * (g3 - g4) + w2 * (d56 - d78);                                            \
        const T sxx = w1 * e1 + dd, syy = w1 * e2 + dd, sxy = w2 * (s56 - s78);                     \
        MXY[s0] = sxy;                                                                              \
        MYY[s0] = syy;                                                                              \
        /* outputs of row r except the y transpose: pbar = 3 pi, ubar = 3 ups + 9 sig u -          \
           3 pi u + 2A (D_x^T sig_x.) */                                                            \
        {                                                                                           \
            const T u0 = Ux + S0[s0], u1 = Uy + S1[s0];                                             \
            const T lxx = from_left(sxx), rxx = from_right(sxx), lxy = from_left(sxy),              \
                    rxy = from_right(sxy);                                                          \
            T tx = T(0.5) * (lxx - rxx), ty = T(0.5) * (lxy - rxy);                                 \
            if (wave_xb) {                                                                          \
                tx = xm2 * from_left(lxx) + xm1 * lxx + x00 * sxx + xp1 * rxx + xp2 * from_right(rxx); \
                ty = xm2 * from_left(lxy) + xm1 * lxy + x00 * sxy + xp1 * rxy + xp2 * from_right(rxy); \
            }                                                                                       \
            OP[s0] = T(3) * pi;                                                                     \
            OX[s0] = T(3) * mux + T(9) * (sxx * u0 + sxy * u1) - T(3) * pi * u0 + A2 * tx;          \
            OY[s0] = T(3) * muy + T(9) * (sxy * u0 + syy * u1) - T(3) * pi * u1 + A2 * ty;          \
            QX[s0] = mux;                                                                           \
            QY[s0] = muy;                                                                           \
        }                                                                                           \
        /* row r-2 is complete with the y transpose of sig rows r-4 .. r */                         \
        const int yo = r - 2;                                                                       \
        if (yo >= Ya && yo < Yb) {                                                                  \
            T cm2, cm1, c00, cp1, cp2;                                                              \
            dT_coef<T>(yo, ny, pery, cm2, cm1, c00, cp1, cp2);                                      \
            const T ox = OX[sm2] + A2 * (cm2 * MXY[sm4] + cm1 * MXY[sm3] + c00 * MXY[sm2] +          \
                                         cp1 * MXY[sm1] + cp2 * MXY[s0]);                           \
            const T oy = OY[sm2] + A2 * (cm2 * MYY[sm4] + cm1 * MYY[sm3] + c00 * MYY[sm2] +          \
                                         cp1 * MYY[sm1] + cp2 * MYY[s0]);                           \
            if (outc) {                                                                             \
                T *op = out + (size_t)yo * (size_t)nx + (unsigned)x;                                \
                op[0] = OP[sm2];                                                                    \
                op[N] = ox;                                                                         \
                op[2 * N] = oy;                                                                     \
                if (ups) {                                                                          \
                    T *uq = ups + (size_t)yo * (size_t)nx + (unsigned)x;                            \
                    uq[0] = QX[sm2];                                                                \
                    uq[N] = QY[sm2];                                                                \
                }                                                                                   \
            }                                                                                       \
        }                                                                                           \
        /* raw row r-2 is no longer needed (g rows up to r+1 are formed): its slot takes row       \
           r+6; the forward velocity of row r+3 */                                                  \
        A2_LOAD(r + 6, RP[sm2], RU[sm2], RV[sm2]);                                                  \
        A2_SPREV(r + 3, S0[sp3], S1[sp3]);                                                          \
    }

        for (int i0 = 0; i0 < nit; i0 += 8) {
            A2_STEP(0) if (i0 + 1 < nit) {
                A2_STEP(1) if (i0 + 2 < nit) {
                    A2_STEP(2) if (i0 + 3 < nit) {
                        A2_STEP(3) if (i0 + 4 < nit) {
                            A2_STEP(4) if (i0 + 5 < nit) {
                                A2_STEP(5) if (i0 + 6 < nit) {
                                    A2_STEP(6) if (i0 + 7 < nit) { A2_STEP(7) }
                                }
                            }
                        }
                    }
                }
            }
        }
#undef A2_STEP
#undef A2_G
#undef A2_YFOLD
#undef A2_SPREV
#undef A2_LOAD
#undef A2_INT
    }
    if (SP) span_end(ts);
}

// ===================================================================== adjoint, 2D: tiles
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
// Along x a wave's 64 lanes are the columns x0 - 2 .. x0 + 61: the g planes are staged
// for those columns only (plus a ring of two rows), so the moments are complete at lanes
// 1 .. 62 and the outputs at lanes 2 .. 61. The second-order one-sided difference on a
// wall node reaches two nodes inward, so the transpose at the node two away from a wall
// needs sig on the wall node. Tile origins are shifted by `off` (0 or 1 per axis, chosen
// on the host) so that no tile boundary falls where that reach would leave the tile's
// complete moments (node n-3 on a tile's last output column along x, nodes 2 and n-3 on
// a tile's first and last output row along y).
template <typename T> struct A3 {
    static constexpr int TX = 64, TY = 8, NT = TX * TY;
    static constexpr int OX = TX - 4, OY = TY - 2;
    static constexpr int WX = TX + 2, WY = TY + 2;  // LDS rows padded by a zero column each side
    static constexpr int RING = 2 * TX;             // the two ring rows
};

// g = (p*bar, u*bar) of plane p at the own column (v[0..3]) and, for ring threads, at the
// ring node (v[4..7]); zeros off the grid.
template <typename T, bool WHOLE>
__device__ __forceinline__ void a3_load(const T *ab, __amdgpu_buffer_rsrc_t rw, long long N, int p, int nz, int pz,
                                        unsigned plane, unsigned coff, unsigned roff, bool ring, T v[8]) {
#pragma unroll
    for (int c = 0; c < 4; c++) v[c] = pload<T, WHOLE>(ab, rw, N, c, p, nz, pz, plane, coff);
    if (ring) {
#pragma unroll
        for (int c = 0; c < 4; c++) v[4 + c] = pload<T, WHOLE>(ab, rw, N, c, p, nz, pz, plane, roff);
    }
}

// ab as prepared by k_adj_fold3d and k_adj_clear3d. The march is unrolled six planes
// deep: the sig history ring (six slots), the partial-output ring and the LDS plane ring
// (three) and the g registers (two) are addressed by constants. g is loaded two planes
// ahead, the previous state one plane ahead and first, so that waiting for it does not
// drain the g loads. Loads and stores go through buffer resources (a lane off the grid
// reads zeros and writes nothing). The transposes are central; the one-sided forms near
// a non-periodic wall are taken in branches uniform over the block (x), the wave (y) or
// the plane (z). UPS: also store the moment ups itself (the paper's u~*).
template <typename T, bool SP, bool UPS, bool WHOLE>
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
    const int px = g.per[0], py = g.per[1], pz = g.per[2];
    const T U0 = gU<T>(g, 0), U1 = gU<T>(g, 1), U2 = gU<T>(g, 2);
    const uint3 tb = xcd_tile();
    const int x0 = (int)tb.x * G::OX - offx, y0 = (int)tb.y * G::OY - offy;
    const int z0 = tb.z * ZC, z1 = min(z0 + ZC, nz);
    // a wave is one row of the tile: ty is uniform over it
    const int tx = threadIdx.x, ty = __builtin_amdgcn_readfirstlane(threadIdx.y), tid = tx + TX * ty;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const __amdgpu_buffer_rsrc_t rab = field_rsrc(ab, N, 4), rsp = field_rsrc(sprev, N, 4),
                                 rout = field_rsrc(out, N, 4), rups = field_rsrc(ups, N, UPS ? 3 : 0);
    // own column (x, y as the output node when inside the output tile)
    const int ox = x0 - 2 + tx, oy = y0 - 1 + ty;
    int cx = ox, cy = oy;
    const bool colok = wrap_coord(cx, nx, px) && wrap_coord(cy, ny, py);
    const unsigned coff = colok ? ((unsigned)cx + (unsigned)nx * (unsigned)cy) * (unsigned)sizeof(T) : BOFF_NONE;
    // ring node of the g planes handled by this thread (waves 0 and 1: the rows y0 - 2
    // and y0 + TY - 1 of the tile's columns)
    const bool ring = tid < G::RING;
    const int ry = tid < TX ? 0 : WY - 1;
    int gx = ox, gy = ry == 0 ? y0 - 2 : y0 + TY - 1;
    const bool ringok = ring && wrap_coord(gx, nx, px) && wrap_coord(gy, ny, py);
    const unsigned roff = ringok ? ((unsigned)gx + (unsigned)nx * (unsigned)gy) * (unsigned)sizeof(T) : BOFF_NONE;
    const bool outcol = tx >= 2 && tx < 2 + G::OX && ty >= 1 && ty <= G::OY && ox >= 0 && ox < nx && oy >= 0 &&
                        oy < ny;
    const unsigned ooff = outcol ? ((unsigned)ox + (unsigned)nx * (unsigned)oy) * (unsigned)sizeof(T) : BOFF_NONE;
    // some output column of the tile (x) / the wave's output row (y) lies within two
    // nodes of a non-periodic wall, where the transposes are one-sided
    const bool xnear = !px && (x0 <= 2 || x0 + G::OX - 1 >= nx - 3);
    const bool ynear = !py && (oy <= 2 || oy >= ny - 3);
    const T A2 = T(2) * A;
    constexpr T w0 = T(2.0 / 9.0), w1 = T(1.0 / 9.0), w2 = T(1.0 / 72.0);

    auto stage = [&](int sl, const T v[8]) {
        gr[sl][0][ty + 1][tx + 1] = v[0] * T(1.0 / 3.0);
#pragma unroll
        for (int c = 1; c < 4; c++) gr[sl][c][ty + 1][tx + 1] = v[c];
        if (ring) {
            gr[sl][0][ry][tx + 1] = v[4] * T(1.0 / 3.0);
#pragma unroll
            for (int c = 1; c < 4; c++) gr[sl][c][ry][tx + 1] = v[4 + c];
        }
    };
    // the pad columns stay zero (read only by lanes 0 and 63, whose moments no output uses)
    if (tid < 3 * 4 * WY * 2) {
        const int k = tid >> 1, side = tid & 1;
        gr[k / (4 * WY)][(k / WY) % 4][k % WY][side ? WX - 1 : 0] = T(0);
    }

    // planes z0-3, z0-2 staged (LDS slots 0, 1); z0-1, z0 in registers (slots 0, 1)
    T gv[2][8];
    a3_load<T, WHOLE>(ab, rab, N, z0 - 3, nz, pz, plane, coff, roff, ring, gv[0]);
    stage(0, gv[0]);
    a3_load<T, WHOLE>(ab, rab, N, z0 - 2, nz, pz, plane, coff, roff, ring, gv[1]);
    stage(1, gv[1]);
    a3_load<T, WHOLE>(ab, rab, N, z0 - 1, nz, pz, plane, coff, roff, ring, gv[0]);
    a3_load<T, WHOLE>(ab, rab, N, z0, nz, pz, plane, coff, roff, ring, gv[1]);
    T uc[3] = {0, 0, 0};  // U + v of the previous state at the output node of plane s
    T hz[6][3];           // sig_xz, sig_yz, sig_zz of plane s + k in slot (J + k + 6) mod 6
    T part[3][4];         // local + in-plane terms of plane s + k in slot (J + k + 3) mod 3
#pragma unroll
    for (int j = 0; j < 6; j++) hz[j][0] = hz[j][1] = hz[j][2] = T(0);
#pragma unroll
    for (int j = 0; j < 3; j++) part[j][0] = part[j][1] = part[j][2] = part[j][3] = T(0);

    const int nsteps = z1 - z0 + 4;  // planes s = z0 - 2 .. z1 + 1
    for (int jb = 0; jb < nsteps; jb += 6) {
#pragma unroll
        for (int J = 0; J < 6; J++) {
            if (jb + J < nsteps) {
            const int s = z0 - 2 + jb + J;
            const int sm = J % 3, s0 = (J + 1) % 3, sp = (J + 2) % 3;  // LDS slots of planes s-1, s, s+1
            stage(sp, gv[J & 1]);
            const T u0 = uc[0], u1 = uc[1], u2 = uc[2];
            {
                // (planes outside [z0, z1) are never output planes: read as off the grid)
                const int pu = s + 1 >= z0 && s + 1 < z1 ? s + 1 : -1;
                uc[0] = U0 + pload<T, WHOLE>(sprev, rsp, N, 1, pu, nz, 0, plane, ooff);
                uc[1] = U1 + pload<T, WHOLE>(sprev, rsp, N, 2, pu, nz, 0, plane, ooff);
                uc[2] = U2 + pload<T, WHOLE>(sprev, rsp, N, 3, pu, nz, 0, plane, ooff);
            }
            if (s + 3 <= z1 + 2) a3_load<T, WHOLE>(ab, rab, N, s + 3, nz, pz, plane, coff, roff, ring, gv[J & 1]);
            __syncthreads();
            // moments of plane s at the own node: g_i taken at the node + c_i
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
                    const int zl = ez > 0 ? sp : sm, zf = ez > 0 ? sm : sp;
                    const T gp = gr[zl][0][ly + ey][lx + 1] + gr[zl][1][ly + ey][lx + 1] +
                                 T(ey) * gr[zl][2][ly + ey][lx + 1] + T(ez) * gr[zl][3][ly + ey][lx + 1];
                    const T gm = gr[zf][0][ly - ey][lx - 1] - gr[zf][1][ly - ey][lx - 1] -
                                 T(ey) * gr[zf][2][ly - ey][lx - 1] - T(ez) * gr[zf][3][ly - ey][lx - 1];
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
            hz[J][0] = sxz;
            hz[J][1] = syz;
            hz[J][2] = szz;
            __syncthreads();
            if (outcol && s >= z0 && s < z1) {
                T o[3];
                o[0] = T(3) * up[0] + T(9) * (sxx * u0 + sxy * u1 + sxz * u2) - T(3) * pi * u0;
                o[1] = T(3) * up[1] + T(9) * (sxy * u0 + syy * u1 + syz * u2) - T(3) * pi * u1;
                o[2] = T(3) * up[2] + T(9) * (sxz * u0 + syz * u1 + szz * u2) - T(3) * pi * u2;
                if (xnear) {
                    dT_apply3<T>(ox, nx, px, A2, [&](int d, T v[3]) {  // a = x: sig_xb -> u_b
                        const int xi = min(max(tx + d, 0), TX - 1);
                        v[0] = sg[0][ty][xi];
                        v[1] = sg[1][ty][xi];
                        v[2] = sg[2][ty][xi];
                    }, o);
                } else {
                    const T km = A2 * T(0.5), kp = A2 * T(-0.5);
#pragma unroll
                    for (int c = 0; c < 3; c++) o[c] += km * sg[c][ty][tx - 1];
#pragma unroll
                    for (int c = 0; c < 3; c++) o[c] += kp * sg[c][ty][tx + 1];
                }
                if (ynear) {
                    dT_apply3<T>(oy, ny, py, A2, [&](int d, T v[3]) {  // a = y: sig_yb -> u_b
                        const int yi = min(max(ty + d, 0), TY - 1);
                        v[0] = sg[1][yi][tx];
                        v[1] = sg[3][yi][tx];
                        v[2] = sg[4][yi][tx];
                    }, o);
                } else {
                    const T km = A2 * T(0.5), kp = A2 * T(-0.5);
                    o[0] += km * sg[1][ty - 1][tx];
                    o[1] += km * sg[3][ty - 1][tx];
                    o[2] += km * sg[4][ty - 1][tx];
                    o[0] += kp * sg[1][ty + 1][tx];
                    o[1] += kp * sg[3][ty + 1][tx];
                    o[2] += kp * sg[4][ty + 1][tx];
                }
                const int ps = J % 3;
                part[ps][0] = T(3) * pi;
                part[ps][1] = o[0];
                part[ps][2] = o[1];
                part[ps][3] = o[2];
                if (UPS) {  // the moment ups itself (the paper's u~*), for its adjoint variant
#pragma unroll
                    for (int c = 0; c < 3; c++) pstore<T, WHOLE>(up[c], ups, rups, N, c, s, plane, ooff);
                }
            }
            const int zo = s - 2;
            if (outcol && zo >= z0 && zo < z1) {
                const int ps = (J + 1) % 3;
                T o[3] = {part[ps][1], part[ps][2], part[ps][3]};
                // a = z: sig_zb -> u_b from the history (plane zo + d in slot (J + d + 4) mod 6)
                if (!pz && (zo <= 2 || zo >= nz - 3)) {
                    dT_apply3<T>(zo, nz, pz, A2, [&](int d, T v[3]) {
                        const int h = (J + d + 4) % 6;
                        v[0] = hz[h][0];
                        v[1] = hz[h][1];
                        v[2] = hz[h][2];
                    }, o);
                } else {
                    const T km = A2 * T(0.5), kp = A2 * T(-0.5);
                    const int hm = (J + 3) % 6, hp = (J + 5) % 6;
#pragma unroll
                    for (int c = 0; c < 3; c++) o[c] += km * hz[hm][c];
#pragma unroll
                    for (int c = 0; c < 3; c++) o[c] += kp * hz[hp][c];
                }
                pstore<T, WHOLE>(part[ps][0], out, rout, N, 0, zo, plane, ooff);
#pragma unroll
                for (int c = 0; c < 3; c++) pstore<T, WHOLE>(o[c], out, rout, N, 1 + c, zo, plane, ooff);
            }
            }
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
