// body.h -- rigid body <-> fluid coupling on gfx950 (Secs. 2.3, 2.4, 3.1) and its
// exact reverse.
//
// Forward, per fluid <-> body iteration k of a step:
//   spread   kappa(x) = sum_m W kappa_ref_m, u^S(x) = sum_m W u^S,ref_m (Eqs.
//            kappa_mapping, us_mapping) in GATHER form: every node of the footprint box
//            inverts the pose once (FP64) and visits its candidate design points with
//            small FP32 body-frame offsets -- no atomics, bitwise-reproducible sums;
//            fused with the Brinkman correction u = (u* + kappa u^S)/(1 + kappa) (Eq. u).
//   interp   u^ref_m = sum_x W u(x) (Eq. u_mapping) over branch-free clamped taps,
//            force/torque contributions in FP64, wave shuffles -> LDS -> per-block
//            partials; the last block to finish sums the partials in a fixed order and
//            applies the Euler update of Sec. 2.4 to the body state of t-1.
// The footprint box of a step is fixed from x^G(t-1): origin floor(x^G) - H, size L,
// wide enough for any rotation and a drift of `margin` nodes within the step.
#pragma once
#include "fluid.h"

namespace lks {

// Threads per block of the design-point kernels: 128 in 2D (more blocks, more CUs for
// small designs), 512 in 3D (fewer block partials for the fixed-order final sums).
template <int DIM> struct Dblk {
    static constexpr int v = DIM == 3 ? 512 : 128;
};

struct BodyParams {
    double kmax, q, mass, inertia;
    int dof;  // LKS_DOF_* bits
};

// ------------------------------------------------------------------ kappa_ref(gamma)
template <typename T>
__global__ __launch_bounds__(256) void k_kappa_ref(long long ND, double kmax, double q,
                                                   const T *__restrict__ gamma, T *__restrict__ krT,
                                                   double *__restrict__ krD) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ND) return;
    const double k = kappa_of(kmax, q, (double)gamma[m]);
    krT[m] = T(k);
    krD[m] = k;
}

__device__ __forceinline__ void body_finish(double *B) {
    double s, c;
    sincos(B[B_TH], &s, &c);
    B[B_COS] = c;
    B[B_SIN] = s;
    B[10] = 0.0;
    B[11] = 0.0;
}

template <int DIM>
__global__ void k_body_init(const double *__restrict__ body, double *__restrict__ B0) {
    if (threadIdx.x != 0) return;
    for (int j = 0; j < 8; j++) B0[j] = body[j];
    body_finish(B0);
}

// Euler update (Sec. 2.4) from the state at t-1 and the force/torque; an inactive DOF
// keeps its previous position and velocity.
template <int DIM>
__device__ __forceinline__ void body_update(const BodyParams &bp, const double *Bp, const double FT[4],
                                            double *Bn) {
    for (int j = 0; j < 8; j++) Bn[j] = Bp[j];
#pragma unroll
    for (int a = 0; a < DIM; a++)
        if (bp.dof & (1 << a)) {
            Bn[B_UG + a] = Bp[B_UG + a] + FT[a] / bp.mass;
            Bn[B_XG + a] = Bp[B_XG + a] + Bn[B_UG + a];
        }
    if (bp.dof & 8) {
        Bn[B_OM] = Bp[B_OM] + FT[3] / bp.inertia;
        Bn[B_TH] = Bp[B_TH] + Bn[B_OM];
    }
    body_finish(Bn);
}

// Transpose of body_update: cotangent Bb of the updated state -> cotangent of the
// force/torque, and the part that flows directly to the state at t-1 (added to acc).
template <int DIM>
__device__ __forceinline__ void body_update_rev(const BodyParams &bp, const double *Bb, double FTb[4],
                                                double *acc) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a < DIM && (bp.dof & (1 << a))) {
            const double ut = Bb[B_UG + a] + Bb[B_XG + a];
            FTb[a] = ut / bp.mass;
            acc[B_XG + a] += Bb[B_XG + a];
            acc[B_UG + a] += ut;
        } else {
            FTb[a] = 0.0;
            acc[B_XG + a] += Bb[B_XG + a];
            acc[B_UG + a] += Bb[B_UG + a];
        }
    }
    if (bp.dof & 8) {
        const double wt = Bb[B_OM] + Bb[B_TH];
        FTb[3] = wt / bp.inertia;
        acc[B_TH] += Bb[B_TH];
        acc[B_OM] += wt;
    } else {
        FTb[3] = 0.0;
        acc[B_TH] += Bb[B_TH];
        acc[B_OM] += Bb[B_OM];
    }
}

// ------------------------------------------------------------------ gather form
// Design points within the support of node x at pose B. The node's body-frame
// position xi0 = R^T (x - x^G) is formed once in FP64 and split into an integer design
// index ib and a fraction f in [0, 1); a candidate ib + delta then has the body-frame
// offset e = delta - f and the lab-frame offset r = x - x^ref = -R e, both small and
// accurate in T. Window: delta in [-1, 2] along the rotation axis (|r| < 2) and in
// the plane [-1, 2] without rotation, [-2, 3] with (|r| < 2 spans 2(|cos| + |sin|) <=
// 2 sqrt 2 design spacings). Calls f(m, W, r) for every candidate with W != 0; also
// returns d = x - x^G (FP64) for callers that rebuild lab-frame arms.
// With LPN > 1, lane q of a group of LPN consecutive lanes visits the candidates
// q, q + LPN, ... of the flattened plane window; callers combine the groups with
// lane_sum (a fixed xor tree: deterministic).
template <int DIM, typename T, bool ROT, int LPN = 1, typename F>
__device__ __forceinline__ void gather_design(const Design &D, const double *B, const int x[3], double d[3],
                                              int q, F &&f) {
    const double c = B[B_COS], s = B[B_SIN];
    d[0] = d[1] = d[2] = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; a++) d[a] = (double)x[a] - B[B_XG + a];
    double xi0[3];
    xi0[D.axis] = d[D.axis];
    xi0[D.pi] = c * d[D.pi] + s * d[D.pj];
    xi0[D.pj] = -s * d[D.pi] + c * d[D.pj];
    int ib[3] = {0, 0, 0};
    T fr[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a >= DIM) continue;
        const double i0 = xi0[a] + D.half[a];
        const double fl = floor(i0);
        ib[a] = (int)fmax(fmin(fl, 1.0e9), -1.0e9);
        fr[a] = T(i0 - fl);
    }
    const T cc = T(c), ss = T(s);
    // along the rotation axis (3D): up to 4 candidates, weight depends on delta only
    constexpr int NA = DIM == 3 ? 4 : 1;
    T wa[NA];
    int ia[NA];
#pragma unroll
    for (int t = 0; t < NA; t++) {
        if (DIM == 3) {
            const int i = ib[D.axis] + t - 1;
            const bool ok = i >= 0 && i < D.nd[D.axis];
            wa[t] = ok ? wk(T(t - 1) - fr[D.axis]) : T(0);  // w is even: w(-e) = w(e)
            ia[t] = ok ? i : 0;
        } else {
            wa[t] = T(1);
            ia[t] = 0;
        }
    }
    constexpr int PW = ROT ? 6 : 4, P0 = ROT ? -2 : -1;
    const int ni = D.nd[D.pi], nj = D.nd[D.pj];
    for (int cidx = q; cidx < PW * PW; cidx += LPN) {
        const int u = cidx / PW, v = cidx - u * PW;
        const int ii = ib[D.pi] + P0 + u;
        const int jj = ib[D.pj] + P0 + v;
        if (ii < 0 || ii >= ni || jj < 0 || jj >= nj) continue;
        const T ei = T(P0 + u) - fr[D.pi];
        const T ej = T(P0 + v) - fr[D.pj];
        T r[3];
        r[D.pi] = -(cc * ei - ss * ej);
        r[D.pj] = -(ss * ei + cc * ej);
        if (!(fabs(r[D.pi]) < T(2) && fabs(r[D.pj]) < T(2))) continue;
        const T wp = wk(r[D.pi]) * wk(r[D.pj]);
#pragma unroll
        for (int t = 0; t < NA; t++) {
            const T W = wp * wa[t];
            if (W == T(0)) continue;
            r[D.axis] = DIM == 3 ? fr[D.axis] - T(t - 1) : T(0);
            int idx[3];
            idx[D.axis] = ia[t];
            idx[D.pi] = ii;
            idx[D.pj] = jj;
            const long long m = idx[0] + (long long)D.nd[0] * (idx[1] + (long long)D.nd[1] * idx[2]);
            f(m, W, r, idx);
        }
    }
}

// 2D form of gather_design (rotation about z: plane axes 0, 1) for sums over design
// arrays: the NC candidates of lane q are listed first (index m and weight w; w = 0 and
// m = 0 for the candidates gather_design skips), so that the caller can issue all their
// loads at once. Summed in list order, zero terms included, the result equals
// gather_design's.
// With WR the offsets r (lab frame, as gather_design passes them), the design indices
// (ci, cj) and d = x - x^G are kept.
template <typename T, bool ROT, int LPN, bool WR = false> struct Cand2 {
    static constexpr int PW = ROT ? 6 : 4, P0 = ROT ? -2 : -1, NC = (PW * PW + LPN - 1) / LPN;
    long long m[NC];
    T w[NC];
    T r0[WR ? NC : 1], r1[WR ? NC : 1];
    int ci[WR ? NC : 1], cj[WR ? NC : 1];
    double d[2];
    __device__ __forceinline__ void init(const Design &D, const double *B, const int x[3], int q) {
        const double c = B[B_COS], s = B[B_SIN];
        const double d0 = (double)x[0] - B[B_XG + 0], d1 = (double)x[1] - B[B_XG + 1];
        d[0] = d0;
        d[1] = d1;
        const double xi0[2] = {c * d0 + s * d1, -s * d0 + c * d1};
        int ib[2];
        T fr[2];
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const double i0 = xi0[a] + D.half[a];
            const double fl = floor(i0);
            ib[a] = (int)fmax(fmin(fl, 1.0e9), -1.0e9);
            fr[a] = T(i0 - fl);
        }
        const T cc = T(c), ss = T(s);
#pragma unroll
        for (int it = 0; it < NC; it++) {
            const int cidx = q + it * LPN;
            const int u = cidx / PW, v = cidx - u * PW;
            const int ii = ib[0] + P0 + u, jj = ib[1] + P0 + v;
            const T ei = T(P0 + u) - fr[0], ej = T(P0 + v) - fr[1];
            const T ri = -(cc * ei - ss * ej), rj = -(ss * ei + cc * ej);
            const bool ok = cidx < PW * PW && ii >= 0 && ii < D.nd[0] && jj >= 0 && jj < D.nd[1] &&
                            fabs(ri) < T(2) && fabs(rj) < T(2);
            w[it] = ok ? wk(ri) * wk(rj) : T(0);
            m[it] = ok ? ii + (long long)D.nd[0] * jj : 0;
            if constexpr (WR) {
                r0[it] = ri;
                r1[it] = rj;
                ci[it] = ii;
                cj[it] = jj;
            }
        }
    }
};

// Sum over the LPN lanes of a group (xor tree, identical result in every lane).
template <int LPN, typename V> __device__ __forceinline__ V lane_sum(V v) {
    if (LPN >= 2) v += __shfl_xor(v, 1, 64);
    if (LPN >= 4) v += __shfl_xor(v, 2, 64);
    if (LPN >= 8) v += __shfl_xor(v, 4, 64);
    return v;
}

template <int DIM>
__device__ __forceinline__ bool box_node(const Grid &g, const Design &D, const int o[3], long long l,
                                         int x[3]) {
    unsigned r = (unsigned)l;  // boxN < 2^31 (checked on the host): 32-bit division
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a < DIM) {
            const unsigned L = (unsigned)D.L[a], q = r / L;
            x[a] = o[a] + (int)(r - q * L);
            r = q;
        } else {
            x[a] = 0;
        }
    }
#pragma unroll
    for (int a = 0; a < DIM; a++)
        if (x[a] < 0 || x[a] >= g.n[a]) return false;
    return is_interior<DIM>(g, x);
}

// kappa(x) and u^S(x) at node x: sum W kappa_ref, and u^G phi + omega a x (sum W (x^ref - x^G))
// with phi = sum W and sum W (x^ref - x^G) = phi d - sum W r formed in FP64. us returns
// u^S(x) - Uref (the fields' reference velocity; Uref null: u^S itself), subtracted in
// FP64 before the rounding to T: a body moving with the flow has u^S close to U, whose
// difference in T would lose the digits that drive the Brinkman term.
// kr(m, idx) returns kappa^ref of design point m (design index idx).
template <int DIM, typename T, bool ROT, int LPN = 1, typename KR>
__device__ __forceinline__ void spread_node_kr(const Design &D, const double *B, KR &&kr, const int x[3], int q,
                                               T &kap, T us[3], const double *Uref) {
    double d[3];
    T k = 0, phi = 0, wr[3] = {0, 0, 0};
    gather_design<DIM, T, ROT, LPN>(D, B, x, d, q, [&](long long m, T W, const T r[3], const int *idx) {
        k += W * kr(m, idx);
        phi += W;
#pragma unroll
        for (int a = 0; a < DIM; a++) wr[a] += W * r[a];
    });
    k = lane_sum<LPN>(k);
    phi = lane_sum<LPN>(phi);
#pragma unroll
    for (int a = 0; a < DIM; a++) wr[a] = lane_sum<LPN>(wr[a]);
    double arm[3];
#pragma unroll
    for (int a = 0; a < 3; a++) arm[a] = a < DIM ? (double)phi * d[a] - (double)wr[a] : 0.0;
    const double armp = pick3(arm, D.pi), armq = pick3(arm, D.pj);
    double axa[3];
#pragma unroll
    for (int a = 0; a < 3; a++) axa[a] = a == D.axis ? 0.0 : (a == D.pi ? -armq : armp);
    const double om = B[B_OM];
    kap = k;
#pragma unroll
    for (int a = 0; a < 3; a++)
        us[a] = a < DIM ? T((B[B_UG + a] * (double)phi - (Uref ? Uref[a] : 0.0)) + om * axa[a]) : T(0);
}

// 2D spread_node_kr with the candidates listed first (Cand2) and all their kappa_ref
// values requested at once; kr(m, ii, jj) returns kappa_ref of design point m = (ii, jj)
// (called for skipped candidates too, with weight 0). The sums, zero terms included,
// equal spread_node_kr's.
template <typename T, bool ROT, int LPN, typename KR>
__device__ __forceinline__ void spread_node2(const Design &D, const double *B, KR &&kr, const int x[3], int q,
                                             T &kap, T us[3], const double *Uref) {
    using C2 = Cand2<T, ROT, LPN, true>;
    C2 cd;
    cd.init(D, B, x, q);
    T kv[C2::NC];
#pragma unroll
    for (int it = 0; it < C2::NC; it++) kv[it] = kr(cd.m[it], cd.ci[it], cd.cj[it]);
    T k = 0, phi = 0, wr[2] = {0, 0};
#pragma unroll
    for (int it = 0; it < C2::NC; it++) {
        const T W = cd.w[it];
        k += W * kv[it];
        phi += W;
        wr[0] += W * cd.r0[it];
        wr[1] += W * cd.r1[it];
    }
    k = lane_sum<LPN>(k);
    phi = lane_sum<LPN>(phi);
    wr[0] = lane_sum<LPN>(wr[0]);
    wr[1] = lane_sum<LPN>(wr[1]);
    const double armp = (double)phi * cd.d[0] - (double)wr[0], armq = (double)phi * cd.d[1] - (double)wr[1];
    const double om = B[B_OM];
    kap = k;
    us[0] = T((B[B_UG + 0] * (double)phi - (Uref ? Uref[0] : 0.0)) + om * (-armq));
    us[1] = T((B[B_UG + 1] * (double)phi - (Uref ? Uref[1] : 0.0)) + om * armp);
    us[2] = T(0);
}

template <int DIM, typename T, bool ROT, int LPN = 1>
__device__ __forceinline__ void spread_node(const Design &D, const double *B, const T *__restrict__ krT,
                                            const int x[3], int q, T &kap, T us[3], const double *Uref) {
    if constexpr (DIM == 2)
        spread_node2<T, ROT, LPN>(D, B, [&](long long m, int, int) { return krT[m]; }, x, q, kap, us, Uref);
    else
        spread_node_kr<DIM, T, ROT, LPN>(D, B, [&](long long m, const int *) { return krT[m]; }, x, q, kap, us,
                                         Uref);
}

// ------------------------------------------------------------------ 3D axial sums
// In 3D the body rotates about a fixed axis, so the position of design point m along the
// axis is x^G_a + xi_a(m) and the mapping weight of node x and point m factors into an
// axial weight and a weight in the rotation plane. The axial offset of node x from point
// m is (x_a - ia) + frac part shared by every node: with c = half_a - x^G_a, the axial base
// index of node x is ib = x_a + floor(c) and its four axial weights w(t - 1 - frac(c)),
// t = 0..3, are the same for all nodes. Sums over the design points therefore take the
// axial sum first, once per pose, on an array the size of the design grid:
//   A[ib][p] = sum_t w(t - 1 - frac(c)) F[ib + t - 1][p]   (ib = -2 .. nd_a + 1),
// and a node then visits only the candidates in the plane (one value each).
struct Axial {
    int fl;     // ib = x_a + fl
    double fr;  // frac(half_a - x^G_a)
};

__device__ __forceinline__ Axial axial_of(const Design &D, const double *B) {
    const double c = D.half[D.axis] - B[B_XG + D.axis];
    const double fl = floor(c);
    return {(int)fmax(fmin(fl, 1.0e9), -1.0e9), c - fl};
}

// The sum of the valid axial weights of base ib.
template <typename T> __device__ __forceinline__ T axial_sum(const Design &D, const Axial &ax, int ib) {
    T s = 0;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int ia = ib + t - 1;
        if (ia >= 0 && ia < D.nd[D.axis]) s += wk(T(t - 1) - T(ax.fr));
    }
    return s;
}

// Axial sums of NC design fields (stride sstride) at the poses B^(k0 + blockIdx.y):
// dst[(y * NC + c) * NA * NP + (ib + 2) + NA * p], NA = nd_a + 4, p = ii + nd_pi * jj.
template <int NC, typename T>
__global__ __launch_bounds__(256) void k_axial(Design D, const double *__restrict__ Bk, int k0,
                                               const T *__restrict__ src, long long sstride, T *__restrict__ dst) {
    const int na = D.nd[D.axis], NA = na + 4;
    const long long NP = (long long)D.nd[D.pi] * D.nd[D.pj];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NA * NP) return;
    const Axial ax = axial_of(D, Bk + (k0 + blockIdx.y) * B_REC);
    // NA * NP < 2^31 (checked on the host): 32-bit division
    const unsigned tu = (unsigned)t, pu = tu / (unsigned)NA, ni = (unsigned)D.nd[D.pi];
    const int ib = (int)(tu - pu * (unsigned)NA) - 2;
    int idx[3];
    idx[D.pi] = (int)(pu % ni);
    idx[D.pj] = (int)(pu / ni);
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) acc[c] = T(0);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int ia = ib + q - 1;
        if (ia < 0 || ia >= na) continue;
        idx[D.axis] = ia;
        const long long m = idx[0] + (long long)D.nd[0] * (idx[1] + (long long)D.nd[1] * idx[2]);
        const T w = wk(T(q - 1) - T(ax.fr));
#pragma unroll
        for (int c = 0; c < NC; c++) acc[c] += w * src[c * sstride + m];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) dst[((long long)blockIdx.y * NC + c) * NA * NP + t] = acc[c];
}

// Plane candidates of node x (3D, gather form, LPN lanes; axis-aligned window: rotated
// windows go through box rows, PlaneRow): f(W, plane index p, r_pi, r_pj) for every design
// column (ii, jj) of the window, with W = 0 at p = 0 for those outside the support (their
// terms vanish). Returns the node's axial base ib and fills d = x - x^G. Plane indices and
// axial-sum offsets fit in int (checked on the host).
template <typename T, bool ROT, int LPN, typename F>
__device__ __forceinline__ int gather_plane(const Design &D, const double *B, const Axial &ax, const int x[3],
                                            double d[3], int q, F &&f) {
    const double c = B[B_COS], s = B[B_SIN];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = (double)x[a] - B[B_XG + a];
    const double xp = c * pick3(d, D.pi) + s * pick3(d, D.pj);
    const double xq = -s * pick3(d, D.pi) + c * pick3(d, D.pj);
    const double i0 = xp + D.half[D.pi], j0 = xq + D.half[D.pj];
    const double fi = floor(i0), fj = floor(j0);
    const int bi = (int)fmax(fmin(fi, 1.0e9), -1.0e9), bj = (int)fmax(fmin(fj, 1.0e9), -1.0e9);
    const T fri = T(i0 - fi), frj = T(j0 - fj);
    const int ib = x[D.axis] + ax.fl;
    if (ib < -2 || ib > D.nd[D.axis] + 1) return ib;  // no design point along the axis
    const T cc = T(c), ss = T(s);
    constexpr int PW = ROT ? 6 : 4, P0 = ROT ? -2 : -1, NC = (PW * PW + LPN - 1) / LPN;
    const int ni = D.nd[D.pi], nj = D.nd[D.pj];
    static_assert(!ROT, "rotated windows: box rows (PlaneRow)");
    // without branches, unrolled by rows, so that the callers' loads of a row are in
    // flight together (the sums are unchanged by the zero terms)
#pragma unroll PW
    for (int it = 0; it < NC; it++) {
        const int cidx = q + it * LPN;
        const int u = cidx / PW, v = cidx - u * PW;
        const int ii = bi + P0 + u, jj = bj + P0 + v;
        const T ei = T(P0 + u) - fri, ej = T(P0 + v) - frj;
        const T rp = -(cc * ei - ss * ej), rq = -(ss * ei + cc * ej);
        const bool ok = cidx < PW * PW && ii >= 0 && ii < ni && jj >= 0 && jj < nj && fabs(rp) < T(2) &&
                        fabs(rq) < T(2);
        f(ok ? wk(rp) * wk(rq) : T(0), ok ? ii + ni * jj : 0, rp, rq);
    }
    return ib;
}

// kappa, u^S at node x (3D) from the axial sums K1 of kappa_ref at pose B (see k_axial).
template <typename T, bool ROT, int LPN>
__device__ __forceinline__ void spread_node_ax(const Design &D, const double *B, const Axial &ax,
                                               const T *__restrict__ K1, const int x[3], int q, T &kap, T us[3],
                                               const double *Uref) {
    const int NA = D.nd[D.axis] + 4;
    double d[3];
    T k = 0, phi = 0, wp = 0, wq = 0;
    const int ib = x[D.axis] + ax.fl;
    gather_plane<T, ROT, LPN>(D, B, ax, x, d, q, [&](T W, int p, T rp, T rq) {
        k += W * K1[(ib + 2) + NA * p];
        phi += W;
        wp += W * rp;
        wq += W * rq;
    });
    k = lane_sum<LPN>(k);
    phi = lane_sum<LPN>(phi);
    wp = lane_sum<LPN>(wp);
    wq = lane_sum<LPN>(wq);
    const T sa = axial_sum<T>(D, ax, ib);
    phi *= sa;
    wp *= sa;
    wq *= sa;
    // u^S(x) = sum_m W (u^G + omega a x (x^ref_m - x^G)) = u^G phi + omega a x (phi d - sum W r)
    const double armp = (double)phi * pick3(d, D.pi) - (double)wp;
    const double armq = (double)phi * pick3(d, D.pj) - (double)wq;
    const double om = B[B_OM];
    kap = k;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double axa = a == D.axis ? 0.0 : (a == D.pi ? -armq : armp);
        us[a] = T((B[B_UG + a] * (double)phi - (Uref ? Uref[a] : 0.0)) + om * axa);
    }
}

// ------------------------------------------------------------------ 3D box rows
// The footprint-box nodes along the rotation axis (a box row) share their plane
// coordinates, hence their plane candidates and weights (only the axial base ib
// differs). The 3D node-side mapping kernels therefore give each box row to one wave:
// the wave forms the row's candidates once, one per lane, into its slot of LDS, and its
// lanes then sweep the row's nodes, reading each candidate (weight, plane index, offsets)
// from LDS at a wave-uniform index, in gather_plane's order, so the sums are the same.
// (LDS, not cross-lane reads of registers: the compiler may recompute a register value
// inside the sweep, where some lanes are inactive.)
template <typename T> struct RowSlot {
    T w[36], rp[36], rq[36];
    int p[36];
};

template <typename T, bool ROT> struct PlaneRow {
    RowSlot<T> *sl;             // this wave's slot
    unsigned long long valid;   // candidates in the support (wave-uniform)
    double dp, dq;              // x - x^G along the plane axes
    // every lane of the wave calls it (the whole wave, no lane inactive)
    __device__ __forceinline__ void init(const Design &D, const double *B, int xi, int xj, RowSlot<T> *slot) {
        sl = slot;
        const double c = B[B_COS], s = B[B_SIN];
        dp = (double)xi - B[B_XG + D.pi];
        dq = (double)xj - B[B_XG + D.pj];
        const double xp = c * dp + s * dq, xq = -s * dp + c * dq;
        const double i0 = xp + D.half[D.pi], j0 = xq + D.half[D.pj];
        const double fi = floor(i0), fj = floor(j0);
        const int bi = (int)fmax(fmin(fi, 1.0e9), -1.0e9), bj = (int)fmax(fmin(fj, 1.0e9), -1.0e9);
        const T fri = T(i0 - fi), frj = T(j0 - fj);
        const T cc = T(c), ss = T(s);
        constexpr int PW = ROT ? 6 : 4, P0 = ROT ? -2 : -1;
        const int lane = threadIdx.x & 63;
        const int u = lane / PW, v = lane - u * PW;
        const int ii = bi + P0 + u, jj = bj + P0 + v;
        const T ei = T(P0 + u) - fri, ej = T(P0 + v) - frj;
        const T rp = -(cc * ei - ss * ej);
        const T rq = -(ss * ei + cc * ej);
        const bool ok = lane < PW * PW && ii >= 0 && ii < D.nd[D.pi] && jj >= 0 && jj < D.nd[D.pj] &&
                        fabs(rp) < T(2) && fabs(rq) < T(2);
        if (lane < PW * PW) {
            sl->w[lane] = ok ? wk(rp) * wk(rq) : T(0);
            sl->rp[lane] = rp;
            sl->rq[lane] = rq;
            sl->p[lane] = ok ? ii + D.nd[D.pi] * jj : 0;
        }
        valid = __ballot(ok);
        // the slot is this wave's alone: order its stores before the sweep's loads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // f(W, p, r_pi, r_pj) for the row's candidates in order (wave-uniform loop), NB at a
    // time without branches between them, so that their loads are in flight together (a
    // batch's missing tail is visited with W = 0 at p = 0: its terms vanish)
    template <int NB, typename F> __device__ __forceinline__ void visit(F &&f) const {
        unsigned long long m = valid;
        while (m) {
            int jb[NB];
            bool on[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                on[b] = m != 0;
                jb[b] = on[b] ? __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1) : 0;
                m &= m - 1;
            }
#pragma unroll
            for (int b = 0; b < NB; b++)
                f(on[b] ? sl->w[jb[b]] : T(0), on[b] ? sl->p[jb[b]] : 0, sl->rp[jb[b]], sl->rq[jb[b]]);
        }
    }
};

// The box row of wave `row`: plane box coordinates and, per node, the grid node.
struct BoxRow {
    int row, bp, bq;  // row index; its box coordinates along the plane axes
    __device__ __forceinline__ static int count(const Design &D) { return D.L[D.pi] * D.L[D.pj]; }
    __device__ __forceinline__ void init(const Design &D, int r) {
        row = r;
        bq = r / D.L[D.pi];
        bp = r - bq * D.L[D.pi];
    }
    // box index l and grid node x of the row's node at axial box coordinate ba; returns
    // whether x is a box node (on the grid and interior), as box_node
    __device__ __forceinline__ bool node(const Grid &g, const Design &D, const int o[3], int ba, long long &l,
                                         int x[3]) const {
        int b[3];
        b[D.axis] = ba;
        b[D.pi] = bp;
        b[D.pj] = bq;
        l = b[0] + (long long)D.L[0] * (b[1] + (long long)D.L[1] * b[2]);
#pragma unroll
        for (int a = 0; a < 3; a++) x[a] = o[a] + b[a];
#pragma unroll
        for (int a = 0; a < 3; a++)
            if (x[a] < 0 || x[a] >= g.n[a]) return false;
        return is_interior<3>(g, x);
    }
};

// spread_node_ax for a node of a box row (candidates from the row's PlaneRow).
template <typename T, bool ROT>
__device__ __forceinline__ void spread_node_row(const Design &D, const double *B, const Axial &ax,
                                                const T *__restrict__ K1, int xa, const PlaneRow<T, ROT> &pr,
                                                T &kap, T us[3], const double *Uref) {
    const int NA = D.nd[D.axis] + 4;
    T k = 0, phi = 0, wp = 0, wq = 0;
    const int ib = xa + ax.fl;
    if (ib >= -2 && ib <= D.nd[D.axis] + 1)
        pr.template visit<8>([&](T W, int p, T rp, T rq) {
            k += W * K1[(ib + 2) + NA * p];
            phi += W;
            wp += W * rp;
            wq += W * rq;
        });
    const T sa = axial_sum<T>(D, ax, ib);
    phi *= sa;
    wp *= sa;
    wq *= sa;
    const double armp = (double)phi * pr.dp - (double)wp;
    const double armq = (double)phi * pr.dq - (double)wq;
    const double om = B[B_OM];
    kap = k;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double axa = a == D.axis ? 0.0 : (a == D.pi ? -armq : armp);
        us[a] = T((B[B_UG + a] * (double)phi - (Uref ? Uref[a] : 0.0)) + om * axa);
    }
}

// Forward spread (k_spread_fwd) in 3D over box rows: 4 waves per block, one row each.
template <typename T, bool ROT>
__global__ __launch_bounds__(256) void k_spread_fwd_rows(Grid g, Design D, const double *__restrict__ Bk, int k,
                                                         const T *__restrict__ K1, T *__restrict__ u,
                                                         T *__restrict__ ustar) {
    const int r = (int)xcd_block() * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= BoxRow::count(D)) return;  // whole waves
    BoxRow br;
    br.init(D, r);
    int o[3];
    box_origin<3>(D, Bk, o);
    const double *B = Bk + k * B_REC;
    __shared__ RowSlot<T> slots[4];
    PlaneRow<T, ROT> pr;
    pr.init(D, B, o[D.pi] + br.bp, o[D.pj] + br.bq, &slots[threadIdx.x >> 6]);
    const Axial ax = axial_of(D, B);
    const long long N = g.N, bN = D.boxN;
    for (int ba = lane; ba < D.L[D.axis]; ba += 64) {
        long long l;
        int x[3];
        if (!br.node(g, D, o, ba, l, x)) continue;
        T kap, us[3];
        spread_node_row<T, ROT>(D, B, ax, K1, x[D.axis], pr, kap, us, g.U);
        const long long id = node_id(g, x[0], x[1], x[2]);
        const T inv = T(1) / (T(1) + kap);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            T s;
            if (k == 0) {
                s = u[a * N + id];
                ustar[a * bN + l] = s;
            } else {
                s = ustar[a * bN + l];
            }
            u[a * N + id] = (s + kap * us[a]) * inv;
        }
    }
}

// ------------------------------------------------------------------ forward spread
// Iteration k of a step: footprint nodes get kappa, u^S at pose B^(k) and the Brinkman
// correction of u* (read from the state at k = 0 and kept in ustar; from ustar after).
template <int DIM, typename T, bool ROT, int LPN>
__global__ __launch_bounds__(256) void k_spread_fwd(Grid g, Design D, const double *__restrict__ Bk, int k,
                                                    const T *__restrict__ krT, const T *__restrict__ K1,
                                                    T *__restrict__ u, T *__restrict__ ustar) {
    const long long t = (long long)xcd_block() * blockDim.x + threadIdx.x;
    const long long l = t / LPN;
    const int q = (int)(t % LPN);
    if (l >= D.boxN) return;
    int o[3], x[3];
    box_origin<DIM>(D, Bk, o);
    if (!box_node<DIM>(g, D, o, l, x)) return;
    T kap, us[3];
    if constexpr (DIM == 3)  // axial sums of kappa_ref at B^(k) in K1 (k_axial)
        spread_node_ax<T, ROT, LPN>(D, Bk + k * B_REC, axial_of(D, Bk + k * B_REC), K1, x, q, kap, us, g.U);
    else
        spread_node<DIM, T, ROT, LPN>(D, Bk + k * B_REC, krT, x, q, kap, us, g.U);
    if (q != 0) return;
    const long long N = g.N;
    const long long id = node_id(g, x[0], x[1], x[2]);
    const T inv = T(1) / (T(1) + kap);
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        T s;
        if (k == 0) {
            s = u[a * N + id];
            ustar[a * D.boxN + l] = s;
        } else {
            s = ustar[a * D.boxN + l];
        }
        u[a * N + id] = (s + kap * us[a]) * inv;
    }
}

// map_design: kappa, u^S on every interior node of the grid at one pose (an ABI body
// state; cos/sin of theta are formed here).
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_spread_map(Grid g, Design D, const double *__restrict__ body,
                                                    const T *__restrict__ krT, T *__restrict__ kap_out,
                                                    T *__restrict__ us_out) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.N) return;
    double B[B_REC];
    for (int j = 0; j < 8; j++) B[j] = body[j];
    body_finish(B);
    int x[3];
    x[0] = (int)(id % g.n[0]);
    x[1] = (int)((id / g.n[0]) % g.n[1]);
    x[2] = (int)(id / ((long long)g.n[0] * g.n[1]));
    T kap = 0, us[3] = {0, 0, 0};
    if (is_interior<DIM>(g, x)) spread_node<DIM, T, true>(D, B, krT, x, 0, kap, us, nullptr);
    kap_out[id] = kap;
#pragma unroll
    for (int a = 0; a < DIM; a++) us_out[a * g.N + id] = us[a];
}

// ------------------------------------------------------------------ taps of a point
// The 4^d nodes around x^ref (floor(X) - 1 .. floor(X) + 2 per axis). Per-axis weights
// are zero for coordinates off the grid or on a boundary layer (the sums run over
// interior nodes) and the coordinates are clamped, so the tap loops have no branches.
// Box-relative variant: coordinates relative to the footprint box, zero weight outside.
template <int DIM, typename T>
//
// S[a] = sum_t w[a][t] and dS[a] = sum_t dw[a][t] are the per-axis weight sums in FP64:
// the sum of W over the taps is S[0] S[1] S[2]. The cosine kernel is a partition of
// unity, so where all four taps of an axis lie on the interior grid S = 1 and dS = 0
// exactly; only an axis with a masked tap (next to a wall) sums its weights, in FP64.
// The interpolation of u = U + v uses them for its U part, U S[0] S[1] S[2], which in
// the weights' own precision would add their rounding times |U| to every force term.
struct Taps {
    int c[3][4];
    T w[3][4], dw[3][4];
    double S[3], dS[3];
    __device__ __forceinline__ void init(const Grid &g, const double X[3], bool want_dw, const int *bo = nullptr,
                                         const int *bl = nullptr) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int base = a < DIM ? (int)fmax(fmin(floor(X[a]), 1.0e9), -1.0e9) - 1 : 0;
            S[a] = 1.0;
            dS[a] = 0.0;
            int okm = 0;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                if (a >= DIM) {
                    c[a][t] = 0;
                    w[a][t] = t == 0 ? T(1) : T(0);
                    dw[a][t] = T(0);
                    continue;
                }
                const int v = base + t;
                bool ok = v >= 0 && v < g.n[a] && (g.per[a] || (v >= 1 && v <= g.n[a] - 2));
                int cv = v;
                if (bo) {
                    cv = v - bo[a];
                    ok = ok && cv >= 0 && cv < bl[a];
                    cv = cv < 0 ? 0 : (cv >= bl[a] ? bl[a] - 1 : cv);
                } else {
                    cv = v < 0 ? 0 : (v >= g.n[a] ? g.n[a] - 1 : v);
                }
                c[a][t] = cv;
                const T r = T((double)v - X[a]);
                w[a][t] = ok ? wk(r) : T(0);
                dw[a][t] = (ok && want_dw) ? dwk(r) : T(0);
                okm |= ok ? 1 << t : 0;
            }
            if (a < DIM && okm != 15) {
                double s = 0.0, ds = 0.0;
#pragma unroll
                for (int t = 0; t < 4; t++)
                    if (okm & (1 << t)) {
                        const double r = (double)(base + t) - X[a];
                        s += wk(r);
                        ds += dwk(r);
                    }
                S[a] = s;
                dS[a] = want_dw ? ds : 0.0;
            }
        }
    }
    // sum of W over the taps
    __device__ __forceinline__ double wsum() const { return S[0] * S[1] * S[2]; }
};

template <typename V> __device__ __forceinline__ V sel4(const V v[4], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// ------------------------------------------------------------------ block reduction
// Thread j < NV stores the block's sum of v[j] (plus its `add`, when given).
template <int NV, int NTHR>
__device__ __forceinline__ void block_reduce_store(double v[NV], double *__restrict__ out, const double *add = nullptr,
                                                   long long slot = -1) {
    __shared__ double red[NV][NTHR / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; j++) v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; j++) red[j][wid] = v[j];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NTHR / 64; w++) s += red[threadIdx.x][w];
        out[(slot < 0 ? (long long)blockIdx.x : slot) * NV + threadIdx.x] = add ? *add + s : s;
    }
}

// Returns true in the one block that arrives last (all partials visible to it). The
// partials of a block are stored by its first wave, so only that wave needs the
// release fence before the arrival counter, and only it (which reads the partials in
// reduce_partials) the acquire fence after.
__device__ __forceinline__ bool last_block(unsigned *counter) {
    __shared__ bool is_last;
    if (threadIdx.x < 64) {
        __threadfence();
        if (threadIdx.x == 0) is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (is_last && threadIdx.x < 64) __threadfence();
    return is_last;
}

// Fixed-order, compensated sum of nb partial vectors of NV doubles (plus a second set
// p2 when given) by all NTHR threads of a block: thread t adds (Neumaier) the vectors
// t, t + NTHR, t + 2 NTHR, ... with two vectors' loads in flight, then the threads'
// sums meet in a fixed xor tree per wave and a fixed-order sum over the waves. The
// same inputs give the same bits in every block. Result in out[NV] (shared memory),
// valid after the call (it ends with a barrier).
template <int NV, int NTHR>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ p1, const double *__restrict__ p2,
                                                unsigned nb, double *out) {
    constexpr int NW = NTHR / 64;
    __shared__ double red[NV][NW];
    Kahan s[NV];
    for (unsigned b0 = threadIdx.x; b0 < nb; b0 += 2 * NTHR) {
        double v[2][NV];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const unsigned b = b0 + u * NTHR;
#pragma unroll
            for (int j = 0; j < NV; j++) {
                v[u][j] = b < nb ? p1[(long long)b * NV + j] : 0.0;
                if (p2) v[u][j] += b < nb ? p2[(long long)b * NV + j] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 2; u++)
#pragma unroll
            for (int j = 0; j < NV; j++) s[j].add(v[u][j]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        const double w = wave_sum(s[j].value());
        if (lane == 0) red[j][wid] = w;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++) t += red[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ forward interp
template <int DIM, int NTHR>
__device__ __forceinline__ void interp_finish(const Design &D, const BodyParams &bp, double *Bk, int k, int K,
                                              double *Bnext0, const double *part, unsigned nb, int *flag);

// flag bits: 1 non-finite body state, 2 drift beyond the footprint margin. With
// last = 0 the kernel only writes its partials (k_interp_finish follows).
// ------------------------------------------------------------------ 3D design tiles
// In 3D (FP32) the interpolation reverse (R1), which reads the 64 taps of a point twice,
// runs one 512-thread block per 8x8x8 tile of design points and stages in LDS the
// analysis-grid patch the tile's stencils touch, so the taps are read from LDS instead
// of L2. pose_point rounds
// monotonically in each design index (see k_iter2d), so the stencil floors of a tile are
// extreme at its eight corners and the patch floor(X) - 1 .. floor(X) + 2 over the corners
// holds every tap of nonzero weight; it spans at most 12 nodes along the rotation axis
// (corners 7 apart) and 14 across it (7 sqrt 2 + 4).
struct Tile3 {
    static constexpr int E = 8, SA = 12, SP = 14, PN = SA * SP * SP, NT = 512;
    static constexpr int CH = (PN + NT - 1) / NT;  // patch nodes per thread
    long long m;  // this thread's design point
    bool own;     // the point exists (ragged tiles)
    int lo[3], s[3];  // patch origin (grid coordinates) and extent
};

// Tile of this block, the thread's point and the patch; false if the patch exceeds its
// bound (excluded above; the extents are then clamped so every access stays in range).
// Every thread of the block must call it (it has a barrier).
__device__ __forceinline__ bool tile3_setup(const Grid &g, const Design &D, const double *B, Tile3 &t) {
    constexpr int E = Tile3::E;
    const int ntx = (D.nd[0] + E - 1) / E, nty = (D.nd[1] + E - 1) / E;
    const int b = (int)xcd_block();
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    const int tid = (int)threadIdx.x;
    const int i = tx * E + tid % E, j = ty * E + (tid / E) % E, kz = tz * E + tid / (E * E);
    t.own = i < D.nd[0] && j < D.nd[1] && kz < D.nd[2];
    t.m = t.own ? i + (long long)D.nd[0] * (j + (long long)D.nd[1] * kz) : 0;
    // the eight corner poses, one per thread, shared through LDS
    __shared__ int cfl[8][3];
    if (tid < 8) {
        const int cc = tid;
        const int ci = tx * E + ((cc & 1) ? min(E, D.nd[0] - tx * E) - 1 : 0);
        const int cj = ty * E + ((cc & 2) ? min(E, D.nd[1] - ty * E) - 1 : 0);
        const int ck = tz * E + ((cc & 4) ? min(E, D.nd[2] - tz * E) - 1 : 0);
        double xi[3];
        design_xi<3>(D, ci + (long long)D.nd[0] * (cj + (long long)D.nd[1] * ck), xi);
        Pose P;
        pose_point(D, B, xi, P);
#pragma unroll
        for (int a = 0; a < 3; a++) cfl[cc][a] = (int)fmax(fmin(floor(P.X[a]), 1.0e9), -1.0e9);
    }
    __syncthreads();
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = cfl[0][a];
        hi[a] = cfl[0][a];
#pragma unroll
        for (int cc = 1; cc < 8; cc++) {
            lo[a] = min(lo[a], cfl[cc][a]);
            hi[a] = max(hi[a], cfl[cc][a]);
        }
        lo[a] -= 1;
        hi[a] += 2;
    }
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = min(max(lo[a], 0), g.n[a] - 1);
        hi[a] = min(max(hi[a], 0), g.n[a] - 1);
        const int cap = a == D.axis ? Tile3::SA : Tile3::SP;
        t.lo[a] = lo[a];
        t.s[a] = hi[a] - lo[a] + 1;
        if (t.s[a] > cap) {
            ok = false;
            t.s[a] = cap;
        }
    }
    return ok;
}

// Stage NC components of a field on the patch: get(x, v) fills v at grid node x. All of
// a thread's loads are issued before its LDS stores. Ends with a barrier.
template <int NC, typename T, typename Get>
__device__ __forceinline__ void tile3_stage(const Tile3 &t, T (*pt)[Tile3::PN], Get &&get) {
    const int n = t.s[0] * t.s[1] * t.s[2];
    T v[Tile3::CH][NC];
#pragma unroll
    for (int r = 0; r < Tile3::CH; r++) {
        const int l = (int)threadIdx.x + r * Tile3::NT;
#pragma unroll
        for (int c = 0; c < NC; c++) v[r][c] = T(0);
        if (l < n) {
            const int x[3] = {t.lo[0] + l % t.s[0], t.lo[1] + (l / t.s[0]) % t.s[1], t.lo[2] + l / (t.s[0] * t.s[1])};
            get(x, v[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < Tile3::CH; r++) {
        const int l = (int)threadIdx.x + r * Tile3::NT;
        if (l < n)
#pragma unroll
            for (int c = 0; c < NC; c++) pt[c][l] = v[r][c];
    }
    __syncthreads();
}

// Patch offsets of a point's taps (clamped: taps outside the patch have weight zero).
template <typename T> struct TapIdx3 {
    int x[4], y[4], z[4];
    __device__ __forceinline__ TapIdx3(const Tile3 &t, const Taps<3, T> &tp) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            x[q] = min(max(tp.c[0][q] - t.lo[0], 0), t.s[0] - 1);
            y[q] = t.s[0] * min(max(tp.c[1][q] - t.lo[1], 0), t.s[1] - 1);
            z[q] = t.s[0] * t.s[1] * min(max(tp.c[2][q] - t.lo[2], 0), t.s[2] - 1);
        }
    }
};

template <int DIM, typename T>
__global__ __launch_bounds__(Dblk<DIM>::v) void k_interp_force(Grid g, Design D, BodyParams bp,
                                                       const T *__restrict__ u, const double *__restrict__ krD,
                                                       double *__restrict__ Bk, int k, int K,
                                                       double *__restrict__ Bnext0, double *__restrict__ part,
                                                       unsigned *__restrict__ counter, int *__restrict__ flag,
                                                       int last) {
    const long long N = g.N;
    const unsigned lb = xcd_block();
    const long long m = (long long)lb * blockDim.x + threadIdx.x;
    const double *B = Bk + k * B_REC;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (m < D.ND) {
        double xi[3];
        design_xi<DIM>(D, m, xi);
        Pose P;
        pose_point(D, B, xi, P);
        Taps<DIM, T> tp;
        tp.init(g, P.X, false);
        T ur[3] = {0, 0, 0};
        constexpr int TZ = DIM == 3 ? 4 : 1;
#pragma unroll 1
        for (int c = 0; c < TZ; c++) {
            const T wz = sel4(tp.w[2], c);
            const int cz = sel4(tp.c[2], c);
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const T wyz = tp.w[1][b] * wz;
                const long long row = (long long)g.n[0] * (tp.c[1][b] + (long long)g.n[1] * cz);
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const T W = tp.w[0][a] * wyz;
                    const long long id = row + tp.c[0][a];
#pragma unroll
                    for (int e = 0; e < DIM; e++) ur[e] += W * u[e * N + id];
                }
            }
        }
        const double kr = krD[m];
        double Dv[3] = {0.0, 0.0, 0.0};
        // u^ref = sum W v + U sum W (the state holds v = u - U)
        const double sw = tp.wsum();
#pragma unroll
        for (int e = 0; e < DIM; e++) {
            Dv[e] = ((double)ur[e] + g.U[e] * sw) - P.US[e];
            v[e] = kr * Dv[e];
        }
        v[3] = kr * (pick3(P.r, D.pi) * pick3(Dv, D.pj) - pick3(P.r, D.pj) * pick3(Dv, D.pi));
    }
    block_reduce_store<4, Dblk<DIM>::v>(v, part, nullptr, lb);
    if (!last) return;
    if (!last_block(counter)) return;
    interp_finish<DIM, Dblk<DIM>::v>(D, bp, Bk, k, K, Bnext0, part, gridDim.x, flag);
    if (threadIdx.x == 0) *counter = 0u;
}

// Fixed-order sum of the force/torque partials and the Euler update of Sec. 2.4:
// B^(k+1) from B(t-1) (plus, after the last iteration, the next step's first record).
template <int DIM, int NTHR>
__device__ __forceinline__ void interp_finish(const Design &D, const BodyParams &bp, double *Bk, int k, int K,
                                              double *Bnext0, const double *part, unsigned nb, int *flag) {
    __shared__ double FT[4];
    reduce_partials<4, NTHR>(part, nullptr, nb, FT);
    if (threadIdx.x == 0) {
        double ft[4] = {FT[0], FT[1], FT[2], FT[3]};
        double *Bn = Bk + (k + 1) * B_REC;
        body_update<DIM>(bp, Bk, ft, Bn);
        bool bad = false;
        for (int j = 0; j < 8; j++) bad = bad || !isfinite(Bn[j]);
        if (bad) atomicOr(flag, 1);
        if (k + 1 < K) {
            for (int a = 0; a < DIM; a++)
                if (!(fabs(Bn[B_XG + a] - Bk[B_XG + a]) <= (double)D.margin)) atomicOr(flag, 2);
        } else if (Bnext0) {
            for (int j = 0; j < B_REC; j++) Bnext0[j] = Bn[j];
        }
    }
}

// One block: the same finish for grids too large for the last-block pattern (one
// arrival counter shared by thousands of blocks serialises them).
template <int DIM>
__global__ __launch_bounds__(1024) void k_interp_finish(Design D, BodyParams bp, double *__restrict__ Bk, int k,
                                                       int K, double *__restrict__ Bnext0,
                                                       const double *__restrict__ part, unsigned nb,
                                                       int *__restrict__ flag) {
    interp_finish<DIM, 1024>(D, bp, Bk, k, K, Bnext0, part, nb, flag);
}

// ------------------------------------------------------------------ fused 2D iteration
// One kernel per fluid <-> body iteration in 2D. Every block first sums the
// force/torque partials of iteration k-1 in a fixed order (the same bits in every
// block) and applies the Euler update, so B^(k) needs no grid-wide fence; block 0
// keeps the record. Each block then owns a TT x TT tile of design points: it forms
// kappa, u^S and the Brinkman-corrected velocity on the patch of nodes touched by the
// tile's interpolation stencils (in LDS; the spread is evaluated again where patches
// overlap), interpolates at its points and stores its force/torque partial. The state
// is left untouched (it holds u* throughout); the step's last spread writes it.
template <int TT> struct It2 {
    static constexpr int NT = 1024;
    static constexpr int HE = TT + 12;  // design halo edge: spread candidates of patch nodes
    // patch edge: the floors of TT points along a rotated lattice line span at most
    // ceil((TT - 1) sqrt 2) + 1 nodes, the stencil adds 3
    static constexpr int PE = TT == 8 ? 14 : 26;
    static constexpr int NW = (TT * TT + 63) / 64;  // waves holding design points
};

template <typename T, bool ROT, int TT>
__global__ __launch_bounds__(It2<TT>::NT) void k_iter2d(Grid g, Design D, BodyParams bp, double *__restrict__ Bk,
                                                         int k, const T *__restrict__ krT,
                                                         const double *__restrict__ krD, const T *__restrict__ u,
                                                         const double *__restrict__ part_in, unsigned nb,
                                                         double *__restrict__ part_out, int *__restrict__ flag) {
    constexpr int NT = It2<TT>::NT, PE = It2<TT>::PE, NW = It2<TT>::NW, HE = It2<TT>::HE;
    __shared__ double B0s[B_REC];
    __shared__ double FT[4];
    __shared__ double red[4][NW];
    __shared__ T up[2][PE][PE];
    __shared__ T kh[HE * HE];
    const int tid = threadIdx.x;
    // Every load is requested first, into registers: the previous iteration's partials
    // (wave 0; nb <= 256), B(t-1), the point's kappa^ref, the kappa^ref halo. Stores into
    // LDS come after, so that no load waits behind another's store.
    double pv[4][4];
    if (k > 0 && tid < 64) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const unsigned b = tid + 64u * u;
#pragma unroll
            for (int j = 0; j < 4; j++) pv[u][j] = b < nb ? part_in[(size_t)b * 4 + j] : 0.0;
        }
    }
    const double b0v = tid < B_REC ? Bk[tid] : 0.0;
    const int tilesX = (D.nd[0] + TT - 1) / TT;
    const int ti = (int)blockIdx.x % tilesX, tj = (int)blockIdx.x / tilesX;
    const int mi = ti * TT + tid % TT, mj = tj * TT + tid / TT;
    const bool own = tid < TT * TT && mi < D.nd[0] && mj < D.nd[1];
    const long long m = own ? mi + (long long)D.nd[0] * mj : 0;
    const double kr = own ? krD[m] : 0.0;
    // kappa^ref of the tile and a six-point halo. A patch node x lies within 2 grid
    // spacings (per axis) of a tile point p, so its body-frame position is within 2 sqrt 2
    // of xi_p, its window base within 3 of xi_p and its gather-form candidates (base - 2 ..
    // base + 3) within 5 of xi_p.
    const int hi0 = ti * TT - 6, hj0 = tj * TT - 6;
    constexpr int KHT = (HE * HE + NT - 1) / NT;
    T khv[KHT];
#pragma unroll
    for (int r = 0; r < KHT; r++) {
        const int l = tid + r * NT;
        const int i = hi0 + l % HE, j = hj0 + l / HE;
        khv[r] = (l < HE * HE && i >= 0 && i < D.nd[0] && j >= 0 && j < D.nd[1]) ? krT[i + (long long)D.nd[0] * j]
                                                                               : T(0);
    }
#pragma unroll
    for (int r = 0; r < KHT; r++)
        if (tid + r * NT < HE * HE) kh[tid + r * NT] = khv[r];
    if (tid < B_REC) B0s[tid] = b0v;
    // the fixed-order sum of iteration k-1's partials by wave 0 (lane l adds the vectors
    // l, l + 64, l + 128, l + 192 compensated, then a fixed xor tree)
    if (k > 0 && tid < 64) {
        Kahan sk[4];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < 4; j++) sk[j].add(pv[u][j]);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const double f = wave_sum(sk[j].value());
            if (tid == 0) FT[j] = f;
        }
    }
    __syncthreads();
    // B^(k) in every thread's registers: B(t-1) at k = 0, else the Euler update
    double Bs[B_REC];
    if (k == 0) {
#pragma unroll
        for (int j = 0; j < B_REC; j++) Bs[j] = B0s[j];
    } else {
        const double ft[4] = {FT[0], FT[1], FT[2], FT[3]};
        double B0[B_REC];
#pragma unroll
        for (int j = 0; j < B_REC; j++) B0[j] = B0s[j];
        body_update<2>(bp, B0, ft, Bs);
        if (blockIdx.x == 0 && tid == 0) {
            bool bad = false;
            for (int j = 0; j < B_REC; j++) Bk[k * B_REC + j] = Bs[j];
            for (int j = 0; j < 8; j++) bad = bad || !isfinite(Bs[j]);
            if (bad) atomicOr(flag, 1);
            for (int a = 0; a < 2; a++)
                if (!(fabs(Bs[B_XG + a] - B0[B_XG + a]) <= (double)D.margin)) atomicOr(flag, 2);
        }
    }
    // Patch: the nodes of the tile points' stencils, floor(X) - 1 .. floor(X) + 2 per
    // axis (clamped to the grid like the taps). pose_point rounds c xi_p, s xi_q, their
    // difference and the sum with x^G, each monotone in its operands, so the computed X
    // is monotone in each design index and its floors are extreme at the tile's corners
    // (exactly, not only up to rounding); threads 0..3 form one corner each.
    __shared__ int cfl[4][2];
    if (tid < 4) {
        const int i0 = ti * TT, i1 = min(i0 + TT, D.nd[0]) - 1;
        const int j0 = tj * TT, j1 = min(j0 + TT, D.nd[1]) - 1;
        const long long mc = ((tid & 1) ? i1 : i0) + (long long)D.nd[0] * ((tid & 2) ? j1 : j0);
        double xi[3];
        design_xi<2>(D, mc, xi);
        Pose Pc;
        pose_point(D, Bs, xi, Pc);
#pragma unroll
        for (int a = 0; a < 2; a++) cfl[tid][a] = (int)fmax(fmin(floor(Pc.X[a]), 1.0e9), -1.0e9);
    }
    __syncthreads();
    int lo[2] = {0x7fffffff, 0x7fffffff}, hi[2] = {-0x7fffffff, -0x7fffffff};
    {
#pragma unroll
        for (int cc = 0; cc < 4; cc++)
#pragma unroll
            for (int a = 0; a < 2; a++) {
                lo[a] = min(lo[a], cfl[cc][a] - 1);
                hi[a] = max(hi[a], cfl[cc][a] + 2);
            }
#pragma unroll
        for (int a = 0; a < 2; a++) {
            lo[a] = min(max(lo[a], 0), g.n[a] - 1);
            hi[a] = min(max(hi[a], 0), g.n[a] - 1);
        }
    }
    const int ox = lo[0], oy = lo[1], sx = hi[0] - lo[0] + 1, sy = hi[1] - lo[1] + 1;
    if (sx > PE || sy > PE) {  // excluded by the bound on PE; keeps LDS accesses in range
        if (tid == 0) atomicOr(flag, 4);
        return;
    }
    // patch: kappa, u^S at pose B^(k), Brinkman correction of u* (LPN lanes per node).
    // The tasks start at the waves after those holding design points, so that these
    // waves get the fewest tasks (none for TT = 8) and form their points' pose and
    // stencil meanwhile.
    int bo[3];
    box_origin<2>(D, B0s, bo);
    const long long N = g.N;
    constexpr int LPN = 4;
    const int pt = (tid + NT - NW * 64) % NT;
    for (int task = pt; task < PE * PE * LPN; task += NT) {
        const int node = task / LPN, q = task % LPN;
        const int px = node % PE, py = node / PE;
        const int x[3] = {ox + px, oy + py, 0};
        const bool in = px < sx && py < sy && x[0] >= 0 && x[0] < g.n[0] && x[1] >= 0 && x[1] < g.n[1] &&
                        is_interior<2>(g, x);
        T v0 = 0, v1 = 0;
        if (in) {
            const long long id = x[0] + (long long)g.n[0] * x[1];
            v0 = u[id];
            v1 = u[N + id];
            const int lx = x[0] - bo[0], ly = x[1] - bo[1];
            if (lx >= 0 && lx < D.L[0] && ly >= 0 && ly < D.L[1]) {
                T kap, us[3];
                spread_node2<T, ROT, LPN>(
                    D, Bs,
                    [&](long long, int ii, int jj) {
                        // always inside the halo (see kh); the clamp only keeps the read in range
                        const int li = min(max(ii - hi0, 0), HE - 1), lj = min(max(jj - hj0, 0), HE - 1);
                        return kh[lj * HE + li];
                    },
                    x, q, kap, us, g.U);
                const T inv = T(1) / (T(1) + kap);
                v0 = (v0 + kap * us[0]) * inv;
                v1 = (v1 + kap * us[1]) * inv;
            }
        }
        if (q == 0 && px < sx && py < sy) {
            up[0][py][px] = v0;
            up[1][py][px] = v1;
        }
    }
    // own point's pose and stencil
    Pose P;
    Taps<2, T> tp;
    if (own) {
        double xi[3];
        design_xi<2>(D, m, xi);
        pose_point(D, Bs, xi, P);
        tp.init(g, P.X, false);
    }
    __syncthreads();
    // interpolation at the tile's points, force and torque terms
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (own) {
        T ur[2] = {0, 0};
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const T wyz = tp.w[1][b] * tp.w[2][0];
            const int yy = min(max(tp.c[1][b] - oy, 0), PE - 1);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                const T W = tp.w[0][a] * wyz;
                const int xx = min(max(tp.c[0][a] - ox, 0), PE - 1);
                ur[0] += W * up[0][yy][xx];
                ur[1] += W * up[1][yy][xx];
            }
        }
        // u^ref = sum W v + U sum W (the patch holds v = u - U)
        const double sw = tp.wsum();
        double Dv[3] = {((double)ur[0] + g.U[0] * sw) - P.US[0], ((double)ur[1] + g.U[1] * sw) - P.US[1], 0.0};
        v[0] = kr * Dv[0];
        v[1] = kr * Dv[1];
        v[3] = kr * (pick3(P.r, D.pi) * pick3(Dv, D.pj) - pick3(P.r, D.pj) * pick3(Dv, D.pi));
    }
    // fixed-order block sum of the waves holding points
    const int lane = tid & 63, wid = tid >> 6;
    if (wid < NW) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const double s = wave_sum(v[j]);
            if (lane == 0) red[j][wid] = s;
        }
    }
    __syncthreads();
    if (tid < 4) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++) s += red[tid][w];
        part_out[(long long)blockIdx.x * 4 + tid] = s;
    }
}

// Last step of the 2D loop: the last block (one beyond the box's) forms B^(K) from the
// partials of iteration K-1 (record, next step's first record, finiteness flag), in
// parallel with the others, which spread at pose B^(K-1) over the footprint box and write
// u <- (u* + kappa u^S) / (1 + kappa) into the state, keeping u* in ustar.
template <typename T, bool ROT, int LPN>
__global__ __launch_bounds__(256) void k_iter_final2d(Grid g, Design D, BodyParams bp, double *__restrict__ Bk,
                                                      int K, const T *__restrict__ krT, T *__restrict__ u,
                                                      T *__restrict__ ustar, const double *__restrict__ part_in,
                                                      unsigned nb, double *__restrict__ Bnext0,
                                                      int *__restrict__ flag) {
    if (blockIdx.x == gridDim.x - 1) {
        // wave 0: the fixed-order sum of the nb <= 256 partials (lane l adds l, l + 64,
        // l + 128, l + 192 compensated, then a fixed xor tree), all loads requested first
        if (threadIdx.x >= 64) return;
        double pv[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const unsigned b = threadIdx.x + 64u * u;
#pragma unroll
            for (int j = 0; j < 4; j++) pv[u][j] = b < nb ? part_in[(size_t)b * 4 + j] : 0.0;
        }
        Kahan sk[4];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < 4; j++) sk[j].add(pv[u][j]);
        double ft[4];
#pragma unroll
        for (int j = 0; j < 4; j++) ft[j] = wave_sum(sk[j].value());
        if (threadIdx.x == 0) {
            double B0[B_REC], Bs[B_REC];
            for (int j = 0; j < B_REC; j++) B0[j] = Bk[j];
            body_update<2>(bp, B0, ft, Bs);
            bool bad = false;
            for (int j = 0; j < B_REC; j++) Bk[K * B_REC + j] = Bs[j];
            for (int j = 0; j < 8; j++) bad = bad || !isfinite(Bs[j]);
            if (bad) atomicOr(flag, 1);
            if (Bnext0)
                for (int j = 0; j < B_REC; j++) Bnext0[j] = Bs[j];
        }
        return;
    }
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long l = t / LPN;
    const int q = (int)(t % LPN);
    if (l >= D.boxN) return;
    int o[3], x[3];
    box_origin<2>(D, Bk, o);
    if (!box_node<2>(g, D, o, l, x)) return;
    T kap, us[3];
    spread_node<2, T, ROT, LPN>(D, Bk + (K - 1) * B_REC, krT, x, q, kap, us, g.U);
    if (q != 0) return;
    const long long N = g.N;
    const long long id = node_id(g, x[0], x[1], x[2]);
    const T inv = T(1) / (T(1) + kap);
#pragma unroll
    for (int a = 0; a < 2; a++) {
        const T s = u[a * N + id];
        ustar[a * D.boxN + l] = s;
        u[a * N + id] = (s + kap * us[a]) * inv;
    }
}

// Standalone Euler update (body_step entry point).
template <int DIM>
__global__ void k_body_step(BodyParams bp, const double *__restrict__ ft, const double *__restrict__ bprev,
                            double *__restrict__ bout) {
    if (threadIdx.x != 0) return;
    double Bp[B_REC], Bn[B_REC], f[4];
    for (int j = 0; j < 8; j++) Bp[j] = bprev[j];
    for (int j = 8; j < B_REC; j++) Bp[j] = 0.0;
    for (int j = 0; j < 4; j++) f[j] = ft[j];
    body_update<DIM>(bp, Bp, f, Bn);
    for (int j = 0; j < 8; j++) bout[j] = Bn[j];
    for (int j = 8; j < 12; j++) bout[j] = bprev[j];
}

// Objective: x^G component or theta at the end minus at the start.
__global__ void k_objective(const double *__restrict__ B0, const double *__restrict__ B1, int obj,
                            double *__restrict__ J, double *__restrict__ body_out) {
    if (threadIdx.x != 0) return;
    const int j = obj == 3 ? B_TH : obj;
    *J = B1[j] - B0[j];
    if (body_out)
        for (int i = 0; i < 8; i++) body_out[i] = B1[i];
}

// =================================================================== reverse sweep
// Device record of the body adjoint (FP64):
//   Bbar[12]  cotangent of B(t) of the step being reversed (B^(K))
//   acc[12]   accumulating cotangent of B(t-1)
//   FTb[4]    force/torque cotangent of the current iteration
enum { AR_BBAR = 0, AR_ACC = 12, AR_FTB = 24, AR_SIZE = 32 };

template <int DIM>
__global__ void k_adj_init(BodyParams bp, int obj, double seed, const double *__restrict__ dbody_T,
                           double *__restrict__ rec) {
    if (threadIdx.x != 0) return;
    for (int j = 0; j < AR_SIZE; j++) rec[j] = 0.0;
    if (dbody_T)
        for (int j = 0; j < 8; j++) rec[AR_BBAR + j] = dbody_T[j];
    rec[AR_BBAR + (obj == 3 ? B_TH : obj)] += seed;
    body_update_rev<DIM>(bp, rec + AR_BBAR, rec + AR_FTB, rec + AR_ACC);
}

// Recompute, for all iterations of a step at once (blockIdx.y = k), the footprint
// fields kappa^(k), u^S^(k), u^(k) from u* and the stored iterates B^(k). These depend
// on forward data only (the cotangent of u* on the box needs no clearing: k_adj_r2
// starts it at the first reverse iteration).
template <int DIM, typename T, bool ROT, int LPN>
__global__ __launch_bounds__(256) void k_adj_recompute(Grid g, Design D, const double *__restrict__ Bk,
                                                       const T *__restrict__ krT, const T *__restrict__ K1,
                                                       const T *__restrict__ ustar, T *__restrict__ kapk,
                                                       T *__restrict__ usk, T *__restrict__ uk) {
    const unsigned lb = xcd_block();
    const long long t = (long long)(lb % gridDim.x) * blockDim.x + threadIdx.x;
    const long long l = t / LPN;
    const int q = (int)(t % LPN);
    const int k = (int)(lb / gridDim.x);
    if (l >= D.boxN) return;
    const long long bN = D.boxN;
    int o[3], x[3];
    box_origin<DIM>(D, Bk, o);
    T kap = 0, us[3] = {0, 0, 0};
    const bool ok = box_node<DIM>(g, D, o, l, x);
    if (ok) {
        if constexpr (DIM == 3)  // axial sums of kappa_ref at B^(k) in K1 + k NA NP (k_axial)
            spread_node_ax<T, ROT, LPN>(D, Bk + k * B_REC, axial_of(D, Bk + k * B_REC),
                                        K1 + (long long)k * (D.nd[D.axis] + 4) * D.nd[D.pi] * D.nd[D.pj], x, q,
                                        kap, us, g.U);
        else
            spread_node<DIM, T, ROT, LPN>(D, Bk + k * B_REC, krT, x, q, kap, us, g.U);
    }
    if (q != 0) return;
    kapk[k * bN + l] = kap;
    const T inv = T(1) / (T(1) + kap);
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        usk[(k * DIM + a) * bN + l] = us[a];
        uk[(k * DIM + a) * bN + l] = ok ? (ustar[a * bN + l] + kap * us[a]) * inv : T(0);
    }
}

// k_adj_recompute in 3D over box rows (4 waves per block, one row each; blockIdx.y = k).
template <typename T, bool ROT>
__global__ __launch_bounds__(256) void k_adj_recompute_rows(Grid g, Design D, const double *__restrict__ Bk,
                                                            const T *__restrict__ K1, const T *__restrict__ ustar,
                                                            T *__restrict__ kapk, T *__restrict__ usk,
                                                            T *__restrict__ uk) {
    const unsigned lb = xcd_block();
    const int r = (int)(lb % gridDim.x) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int k = (int)(lb / gridDim.x);
    if (r >= BoxRow::count(D)) return;  // whole waves
    BoxRow br;
    br.init(D, r);
    int o[3];
    box_origin<3>(D, Bk, o);
    const double *B = Bk + k * B_REC;
    __shared__ RowSlot<T> slots[4];
    PlaneRow<T, ROT> pr;
    pr.init(D, B, o[D.pi] + br.bp, o[D.pj] + br.bq, &slots[threadIdx.x >> 6]);
    const Axial ax = axial_of(D, B);
    const T *K1k = K1 + (long long)k * (D.nd[D.axis] + 4) * D.nd[D.pi] * D.nd[D.pj];
    const long long bN = D.boxN;
    for (int ba = lane; ba < D.L[D.axis]; ba += 64) {
        long long l;
        int x[3];
        const bool ok = br.node(g, D, o, ba, l, x);
        T kap = 0, us[3] = {0, 0, 0};
        if (ok) spread_node_row<T, ROT>(D, B, ax, K1k, x[D.axis], pr, kap, us, g.U);
        kapk[k * bN + l] = kap;
        const T inv = T(1) / (T(1) + kap);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            usk[(k * 3 + a) * bN + l] = us[a];
            uk[(k * 3 + a) * bN + l] = ok ? (ustar[a * bN + l] + kap * us[a]) * inv : T(0);
        }
    }
}

// Per-point pose cotangents -> (x^G, u^G, theta, omega) contributions.
// Xb: cotangent of x^ref, USb: of u^S,ref, rb: of r = R xi used by the torque.
__device__ __forceinline__ void pose_rev(const Design &D, const double *B, const Pose &P, const double Xb[3],
                                         const double USb[3], const double rb[3], double v[8]) {
    const int i = D.pi, j = D.pj;
    const double om = B[B_OM];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        v[a] += Xb[a];
        v[3 + a] += USb[a];
    }
    const double ri = pick3(P.r, i), rj = pick3(P.r, j);
    const double ui = pick3(USb, i), uj = pick3(USb, j);
    // d r / d theta = a x r = (-r_j, r_i) in the plane; d(a x r)/d theta = -(r_i, r_j)
    v[6] += (pick3(Xb, i) + pick3(rb, i)) * (-rj) + (pick3(Xb, j) + pick3(rb, j)) * ri +
            om * (ui * (-ri) + uj * (-rj));
    v[7] += ui * (-rj) + uj * ri;
}

template <int DIM, int NTHR>
__device__ __forceinline__ void rec_finish(const BodyParams &bp, int k, const double *parts, unsigned nb,
                                           const double *rin, double *rs);

// Record step of iteration k by one wave: the same as rec_finish, with the partials summed
// by the wave alone (lane l adds the blocks l, l + 64, ... compensated, four blocks' loads
// in flight, then a fixed xor tree), so the other waves of the block need not wait. rs
// complete after a barrier.
template <int DIM>
__device__ __forceinline__ void wave_rec_finish(const BodyParams &bp, int k, const double *parts, unsigned nb,
                                                const double *rin, double *rs) {
    const unsigned lane = threadIdx.x & 63;
    Kahan s[8];
    for (unsigned b0 = lane; b0 < nb; b0 += 256) {
        double v[4][8];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const unsigned b = b0 + u * 64;
#pragma unroll
            for (int j = 0; j < 8; j++) v[u][j] = b < nb ? parts[(size_t)b * 8 + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < 8; j++) s[j].add(v[u][j]);
    }
    double bb[B_REC];
#pragma unroll
    for (int j = 0; j < B_REC; j++) bb[j] = j < 8 ? wave_sum(s[j].value()) : 0.0;
    if (lane == 0) {
        for (int j = 0; j < AR_SIZE; j++) rs[j] = rin[j];
        if (k > 0) {
            body_update_rev<DIM>(bp, bb, rs + AR_FTB, rs + AR_ACC);
        } else {
            double *acc = rs + AR_ACC;
            for (int j = 0; j < 8; j++) acc[j] += bb[j];
            for (int j = 0; j < B_REC; j++) {
                rs[AR_BBAR + j] = acc[j];
                acc[j] = 0.0;
            }
            body_update_rev<DIM>(bp, rs + AR_BBAR, rs + AR_FTB, acc);
        }
    }
}

// Threads of an R1 block: one per design point, plus in 2D a wave that steps the record.
template <int DIM> struct R1blk {
    static constexpr int pts = Dblk<DIM>::v, v = pts + (DIM == 2 ? 64 : 0);
};

// R1: reverse of the force/torque and of the interpolation at iteration k. The
// force/torque cotangent comes from the record rin, or, with pnb > 0, every block first
// finishes the previous iteration kfin from its pnb partials pp (R1's and R3's summed by
// R3; the same fixed-order sum and record step in every block, so the same bits) and block 0
// stores the stepped record in rout (rin and rout are distinct, since other blocks may
// still read rin). In 2D the block's extra wave does that while the others interpolate.
template <int DIM, typename T, bool TL = false>
__global__ __launch_bounds__(R1blk<DIM>::v) void k_adj_r1(Grid g, Design D, BodyParams bp, const double *__restrict__ Bk,
                                                 int k,
                                                 const T *__restrict__ uk, const double *__restrict__ krD,
                                                 const double *__restrict__ rin, double *__restrict__ rout,
                                                 const double *__restrict__ pp, unsigned pnb, int kfin, T *__restrict__ URb,
                                                 double *__restrict__ krb, double *__restrict__ part,
                                                 int *__restrict__ flag) {
    __shared__ double rs[AR_SIZE];
    // The record step runs first in 3D (keeps the registers of the long tap loops
    // free) and after the interpolation in 2D (overlaps its loads).
    constexpr bool EARLY = DIM == 3;
    const double *FTb = rin + AR_FTB;
    if (EARLY && pnb > 0) {
        rec_finish<DIM, Dblk<DIM>::v>(bp, kfin, pp, pnb, rin, rs);
        FTb = rs + AR_FTB;
        if (blockIdx.x == 0 && threadIdx.x < AR_SIZE) rout[threadIdx.x] = rs[threadIdx.x];
    }
    const long long bN = D.boxN;
    const double *B = Bk + k * B_REC;
    const T *u = uk + (long long)k * DIM * bN;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int o[3];
    box_origin<DIM>(D, Bk, o);
    __shared__ T pt[TL ? 3 : 1][TL ? Tile3::PN : 1];
    Tile3 t;
    long long m;
    bool own;
    if constexpr (TL) {
        // a patch beyond its bound would clamp taps onto its edge: report it (flag 4)
        if (!tile3_setup(g, D, B, t) && threadIdx.x == 0) atomicOr(flag, 4);
        tile3_stage<3>(t, pt, [&](const int x[3], T *vv) {
            const int bx = x[0] - o[0], by = x[1] - o[1], bz = x[2] - o[2];
            if (bx >= 0 && bx < D.L[0] && by >= 0 && by < D.L[1] && bz >= 0 && bz < D.L[2]) {
                const long long bi = bx + (long long)D.L[0] * (by + (long long)D.L[1] * bz);
#pragma unroll
                for (int e = 0; e < 3; e++) vv[e] = u[e * bN + bi];
            }
        });
        m = t.m;
        own = t.own;
    } else {
        m = (long long)xcd_block() * R1blk<DIM>::pts + threadIdx.x;
        own = threadIdx.x < R1blk<DIM>::pts && m < D.ND;
    }
    // interpolation of u^(k) at the point (independent of the record)
    Pose P;
    Taps<DIM, T> tp;
    constexpr int TZ = DIM == 3 ? 4 : 1;
    T ur[3] = {0, 0, 0};
    // offsets of the taps: in the staged patch (TL) or in the box arrays
    int ox[4], oy[4], oz[4];
    const T *src[3];
    double kr = 0.0, kb0 = 0.0;  // kappa_ref and its running cotangent, requested early
    if (own) {
        kr = krD[m];
        kb0 = krb[m];
        double xi[3];
        design_xi<DIM>(D, m, xi);
        pose_point(D, B, xi, P);
        if (TL) tp.init(g, P.X, true);
        else tp.init(g, P.X, true, o, D.L);
        if constexpr (TL) {
            const TapIdx3<T> ti(t, tp);
#pragma unroll
            for (int q = 0; q < 4; q++) ox[q] = ti.x[q], oy[q] = ti.y[q], oz[q] = ti.z[q];
#pragma unroll
            for (int e = 0; e < 3; e++) src[e] = pt[e];
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                ox[q] = tp.c[0][q];
                oy[q] = D.L[0] * tp.c[1][q];
                oz[q] = D.L[0] * D.L[1] * tp.c[2][q];
            }
#pragma unroll
            for (int e = 0; e < 3; e++) src[e] = u + (e < DIM ? e : 0) * bN;
        }
#pragma unroll 1
        for (int c = 0; c < TZ; c++) {
            const T wz = sel4(tp.w[2], c);
            const int cz = sel4(oz, c);
#pragma unroll
            for (int b = 0; b < 4; b++) {
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const T W = tp.w[0][a] * tp.w[1][b] * wz;
                    const int l = ox[a] + oy[b] + cz;
#pragma unroll
                    for (int e = 0; e < DIM; e++) ur[e] += W * src[e][l];
                }
            }
        }
    }
    if (!EARLY && pnb > 0) {
        if (threadIdx.x >= R1blk<DIM>::pts) wave_rec_finish<DIM>(bp, kfin, pp, pnb, rin, rs);
        __syncthreads();
        FTb = rs + AR_FTB;
        if (blockIdx.x == 0 && threadIdx.x < AR_SIZE) rout[threadIdx.x] = rs[threadIdx.x];
    }
    if (own) {
        double Dv[3] = {0, 0, 0}, Db[3] = {0, 0, 0};
#pragma unroll
        for (int e = 0; e < DIM; e++) Dv[e] = ((double)ur[e] + g.U[e] * tp.wsum()) - P.US[e];
        double gsum = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; e++) {
            Db[e] = kr * (FTb[e] + FTb[3] * P.axr[e]);
            gsum += FTb[e] * Dv[e];
        }
        const double dp = pick3(Dv, D.pi), dq = pick3(Dv, D.pj);
        gsum += FTb[3] * (pick3(P.r, D.pi) * dq - pick3(P.r, D.pj) * dp);
        krb[m] = kb0 + gsum;
        double rb[3], USb[3] = {0, 0, 0}, Xb[3] = {0, 0, 0};
#pragma unroll
        for (int e = 0; e < 3; e++)
            rb[e] = e == D.pi ? FTb[3] * kr * dq : (e == D.pj ? -FTb[3] * kr * dp : 0.0);
#pragma unroll
        for (int e = 0; e < DIM; e++) {
            USb[e] = -Db[e];
            URb[e * D.ND + m] = T(Db[e]);
        }
        // x^ref cotangent from the interpolation: sum_x dW/dX (Db . u(x)), u = U + v; the
        // U part, (Db . U) d(S0 S1 S2)/dX, from the FP64 weight sums (zero away from walls)
        T xb[3] = {0, 0, 0};
        const T db[3] = {T(Db[0]), T(Db[1]), T(Db[2])};
        double dbU = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; e++) dbU += Db[e] * g.U[e];
#pragma unroll 1
        for (int c = 0; c < TZ; c++) {
            const T wz = sel4(tp.w[2], c), dwz = sel4(tp.dw[2], c);
            const int cz = sel4(oz, c);
#pragma unroll
            for (int b = 0; b < 4; b++) {
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    T dot = 0;
                    const int l = ox[a] + oy[b] + cz;
#pragma unroll
                    for (int e = 0; e < DIM; e++) dot += db[e] * src[e][l];
                    xb[0] -= tp.dw[0][a] * tp.w[1][b] * wz * dot;
                    xb[1] -= tp.w[0][a] * tp.dw[1][b] * wz * dot;
                    if (DIM == 3) xb[2] -= tp.w[0][a] * tp.w[1][b] * dwz * dot;
                }
            }
        }
        Xb[0] = (double)xb[0] - dbU * (tp.dS[0] * tp.S[1] * tp.S[2]);
        Xb[1] = (double)xb[1] - dbU * (tp.S[0] * tp.dS[1] * tp.S[2]);
        if (DIM == 3) Xb[2] = (double)xb[2] - dbU * (tp.S[0] * tp.S[1] * tp.dS[2]);
        pose_rev(D, B, P, Xb, USb, rb, v);
    }
    block_reduce_store<8, R1blk<DIM>::v>(v, part, nullptr, xcd_block());
}

// R2: box nodes. u^(k) cotangent = (k = last: the step's velocity cotangent, with the
// boundary fold) + sum_m W URb_m (transpose of the interpolation, gather form);
// Brinkman correction reversed.
template <int DIM, typename T, bool ROT, int LPN>
__global__ __launch_bounds__(256) void k_adj_r2(Grid g, Bc bc, Design D, const double *__restrict__ Bk, int k,
                                                int K, const T *__restrict__ ab, const T *__restrict__ URb,
                                                const T *__restrict__ AU, const T *__restrict__ kapk,
                                                const T *__restrict__ usk, const T *__restrict__ uk,
                                                T *__restrict__ ustb, T *__restrict__ kb, T *__restrict__ usb) {
    const long long t = (long long)xcd_block() * blockDim.x + threadIdx.x;
    const long long l = t / LPN;
    const int q = (int)(t % LPN);
    if (l >= D.boxN) return;
    const long long bN = D.boxN;
    int o[3], x[3];
    box_origin<DIM>(D, Bk, o);
    if (!box_node<DIM>(g, D, o, l, x)) {
        if (q != 0) return;
        kb[l] = T(0);
#pragma unroll
        for (int a = 0; a < DIM; a++) usb[a * bN + l] = T(0);
        return;
    }
    // the node's own fields, requested before the gather; the cotangent of u* starts
    // at the first reverse iteration (k = K - 1), which writes every node of the grid
    T kap = 0, ust[3] = {0, 0, 0}, dus[3] = {0, 0, 0};
    if (q == 0) {
        kap = kapk[k * bN + l];
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            ust[a] = k == K - 1 ? T(0) : ustb[a * bN + l];
            dus[a] = usk[(k * DIM + a) * bN + l] - uk[(k * DIM + a) * bN + l];
        }
    }
    T ub[3] = {0, 0, 0};
    double d[3];
    if constexpr (DIM == 3) {  // axial sums of URb at B^(k) in AU (k_axial, 3 components)
        const Axial ax = axial_of(D, Bk + k * B_REC);
        const int NA = D.nd[D.axis] + 4;
        const long long NANP = (long long)NA * D.nd[D.pi] * D.nd[D.pj];
        const int ib = x[D.axis] + ax.fl;
        gather_plane<T, ROT, LPN>(D, Bk + k * B_REC, ax, x, d, q, [&](T W, int p, T, T) {
            const int i = (ib + 2) + NA * p;
#pragma unroll
            for (int a = 0; a < 3; a++) ub[a] += W * AU[a * NANP + i];
        });
    } else {
        // candidates listed first, then all their loads in flight together
        Cand2<T, ROT, LPN> cd;
        cd.init(D, Bk + k * B_REC, x, q);
        T v[2][Cand2<T, ROT, LPN>::NC];
#pragma unroll
        for (int it = 0; it < Cand2<T, ROT, LPN>::NC; it++)
#pragma unroll
            for (int a = 0; a < 2; a++) v[a][it] = URb[a * D.ND + cd.m[it]];
#pragma unroll
        for (int it = 0; it < Cand2<T, ROT, LPN>::NC; it++)
#pragma unroll
            for (int a = 0; a < 2; a++) ub[a] += cd.w[it] * v[a][it];
        (void)d;
    }
#pragma unroll
    for (int a = 0; a < DIM; a++) ub[a] = lane_sum<LPN>(ub[a]);
    if (q != 0) return;
    if (k == K - 1) {
        const long long id = node_id(g, x[0], x[1], x[2]);
        T pdummy, uf[3];
        fold_bc<DIM, T>(g, bc, ab, x, id, pdummy, uf, true);
#pragma unroll
        for (int a = 0; a < DIM; a++) ub[a] += uf[a];
    }
    const T inv = T(1) / (T(1) + kap);
    T kbar = 0;
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        ustb[a * bN + l] = ust[a] + ub[a] * inv;
        kbar += ub[a] * dus[a] * inv;
        usb[a * bN + l] = ub[a] * kap * inv;
    }
    kb[l] = kbar;
}

// R3: transpose of the spread at iteration k (design-point parallel), the pose
// reversed. Block b stores its partial plus R1's partial b (part1) in part3: their sum
// over the blocks is the body cotangent B^(k)bar (rec_finish, in the next R1 or in
// k_r3_finish).
template <int DIM, typename T>
__global__ __launch_bounds__(Dblk<DIM>::v) void k_adj_r3(Grid g, Design D, const double *__restrict__ Bk, int k,
                                                 const T *__restrict__ kb, const T *__restrict__ usb,
                                                 const double *__restrict__ krD, double *__restrict__ krb,
                                                 const double *__restrict__ part1, double *__restrict__ part3) {
    const unsigned lb = xcd_block();
    const long long m = (long long)lb * blockDim.x + threadIdx.x;
    // R1's partial of this (logical) block, added to this block's at the end: requested
    // first in 2D; in 3D, held across the tap loop, the early load slowed the kernel
    const bool p1t = threadIdx.x < 8;
    double p1v = (DIM == 2 && p1t) ? part1[(long long)lb * 8 + threadIdx.x] : 0.0;
    const long long bN = D.boxN;
    const double *B = Bk + k * B_REC;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (m < D.ND) {
        int o[3];
        box_origin<DIM>(D, Bk, o);
        double xi[3];
        design_xi<DIM>(D, m, xi);
        Pose P;
        pose_point(D, B, xi, P);
        Taps<DIM, T> tp;
        tp.init(g, P.X, true, o, D.L);
        const T kr = T(krD[m]);
        const T US[3] = {T(P.US[0]), T(P.US[1]), T(P.US[2])};
        T ksum = 0, uss[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
        constexpr int TZ = DIM == 3 ? 4 : 1;
#pragma unroll 1
        for (int c = 0; c < TZ; c++) {
            const T wz = sel4(tp.w[2], c), dwz = sel4(tp.dw[2], c);
            const int cz = sel4(tp.c[2], c);
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const long long row = (long long)D.L[0] * (tp.c[1][b] + (long long)D.L[1] * cz);
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const long long bi = row + tp.c[0][a];
                    const T W = tp.w[0][a] * tp.w[1][b] * wz;
                    const T kv = kb[bi];
                    T dot = kv * kr;
                    ksum += W * kv;
#pragma unroll
                    for (int e = 0; e < DIM; e++) {
                        const T s = usb[e * bN + bi];
                        uss[e] += W * s;
                        dot += s * US[e];
                    }
                    xb[0] -= tp.dw[0][a] * tp.w[1][b] * wz * dot;
                    xb[1] -= tp.w[0][a] * tp.dw[1][b] * wz * dot;
                    if (DIM == 3) xb[2] -= tp.w[0][a] * tp.w[1][b] * dwz * dot;
                }
            }
        }
        krb[m] += (double)ksum;
        double Xb[3] = {0, 0, 0}, USb[3] = {0, 0, 0}, rb[3] = {0, 0, 0};
#pragma unroll
        for (int e = 0; e < DIM; e++) {
            Xb[e] = (double)xb[e];
            USb[e] = (double)uss[e];
        }
        pose_rev(D, B, P, Xb, USb, rb, v);
    }
    if (DIM == 3 && p1t) p1v = part1[(long long)lb * 8 + threadIdx.x];
    block_reduce_store<8, Dblk<DIM>::v>(v, part3, &p1v, lb);
}

// k_adj_r2 in 3D over box rows (4 waves per block, one row each).
template <typename T, bool ROT>
__global__ __launch_bounds__(256) void k_adj_r2_rows(Grid g, Bc bc, Design D, const double *__restrict__ Bk, int k,
                                                     int K, const T *__restrict__ ab, const T *__restrict__ AU,
                                                     const T *__restrict__ kapk, const T *__restrict__ usk,
                                                     const T *__restrict__ uk, T *__restrict__ ustb,
                                                     T *__restrict__ kb, T *__restrict__ usb) {
    const int r = (int)xcd_block() * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= BoxRow::count(D)) return;  // whole waves
    BoxRow br;
    br.init(D, r);
    int o[3];
    box_origin<3>(D, Bk, o);
    const double *B = Bk + k * B_REC;
    __shared__ RowSlot<T> slots[4];
    PlaneRow<T, ROT> pr;
    pr.init(D, B, o[D.pi] + br.bp, o[D.pj] + br.bq, &slots[threadIdx.x >> 6]);
    const Axial ax = axial_of(D, B);
    const int NA = D.nd[D.axis] + 4;
    const long long NANP = (long long)NA * D.nd[D.pi] * D.nd[D.pj];
    const long long bN = D.boxN;
    for (int ba = lane; ba < D.L[D.axis]; ba += 64) {
        long long l;
        int x[3];
        if (!br.node(g, D, o, ba, l, x)) {
            kb[l] = T(0);
#pragma unroll
            for (int a = 0; a < 3; a++) usb[a * bN + l] = T(0);
            continue;
        }
        // the node's own fields, requested before the gather; the cotangent of u* starts
        // at the first reverse iteration (k = K - 1)
        const T kap = kapk[k * bN + l];
        T ust[3], dus[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            ust[a] = k == K - 1 ? T(0) : ustb[a * bN + l];
            dus[a] = usk[(k * 3 + a) * bN + l] - uk[(k * 3 + a) * bN + l];
        }
        T ub[3] = {0, 0, 0};
        const int ib = x[D.axis] + ax.fl;
        if (ib >= -2 && ib <= D.nd[D.axis] + 1)
            pr.template visit<8>([&](T W, int p, T, T) {
                const int i = (ib + 2) + NA * p;
#pragma unroll
                for (int a = 0; a < 3; a++) ub[a] += W * AU[a * NANP + i];
            });
        if (k == K - 1) {
            const long long id = node_id(g, x[0], x[1], x[2]);
            T pdummy, uf[3];
            fold_bc<3, T>(g, bc, ab, x, id, pdummy, uf, true);
#pragma unroll
            for (int a = 0; a < 3; a++) ub[a] += uf[a];
        }
        const T inv = T(1) / (T(1) + kap);
        T kbar = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            ustb[a * bN + l] = ust[a] + ub[a] * inv;
            kbar += ub[a] * dus[a] * inv;
            usb[a * bN + l] = ub[a] * kap * inv;
        }
        kb[l] = kbar;
    }
}

// Body cotangent B^(k)bar from the partials of iteration k (fixed order), then
// the record step on a copy of rin in rs (shared or global memory; rs may be rin): the
// force/torque cotangent of iteration k-1, or at k = 0 the cotangent of B(t-1) and the
// force/torque cotangent of the previous step's last iteration. Every thread of the
// block calls it; rs is complete on return.
template <int DIM, int NTHR>
__device__ __forceinline__ void rec_finish(const BodyParams &bp, int k, const double *parts, unsigned nb,
                                           const double *rin, double *rs) {
    __shared__ double Bkb[8];
    if (rs != rin && threadIdx.x < AR_SIZE) rs[threadIdx.x] = rin[threadIdx.x];  // published by the barriers below
    reduce_partials<8, NTHR>(parts, nullptr, nb, Bkb);
    if (threadIdx.x == 0) {
        double bb[B_REC];
        for (int j = 0; j < B_REC; j++) bb[j] = j < 8 ? Bkb[j] : 0.0;
        if (k > 0) {
            body_update_rev<DIM>(bp, bb, rs + AR_FTB, rs + AR_ACC);
        } else {
            double *acc = rs + AR_ACC;
            for (int j = 0; j < 8; j++) acc[j] += bb[j];
            for (int j = 0; j < B_REC; j++) {
                rs[AR_BBAR + j] = acc[j];
                acc[j] = 0.0;
            }
            body_update_rev<DIM>(bp, rs + AR_BBAR, rs + AR_FTB, acc);
        }
    }
    __syncthreads();
}

// One block: the record step of iteration k in place (rec_finish), for grids whose R1
// would read too many partials per block, and after the last iteration.
template <int DIM>
__global__ __launch_bounds__(1024) void k_r3_finish(BodyParams bp, int k, const double *__restrict__ parts,
                                                   unsigned nb, double *__restrict__ rec) {
    rec_finish<DIM, 1024>(bp, k, parts, nb, rec, rec);
}

// grad = krb * d kappa_ref / d gamma; optional body cotangent of t = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_final(long long ND, double kmax, double q, const T *__restrict__ gamma,
                                                    const double *__restrict__ krb, double *__restrict__ grad,
                                                    const double *__restrict__ rec, int obj, double seed,
                                                    double *__restrict__ dbody0) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m < ND) grad[m] = krb[m] * dkappa_of(kmax, q, (double)gamma[m]);
    if (m == 0 && dbody0) {
        for (int j = 0; j < 12; j++) dbody0[j] = j < 8 ? rec[AR_BBAR + j] : 0.0;
        dbody0[obj == 3 ? B_TH : obj] -= seed;
    }
}

// ------------------------------------------------------------------ coupling constants
// The fluid <-> body iteration of Sec. 3.1 (u^G,(k+1) = u^G(t-1) + F(u^G,(k))/M at a
// frozen pose and u*) contracts when K/M < 1, K = -dF/du^G (and K_theta/I < 1,
// K_theta = -dT/domega). F and T are affine in u^G and omega, and the spread, the
// Brinkman factor and the interpolation give, with phi = sum_m W, kappa = sum_m W kappa_m,
// s_m = a x (x^ref_m - x^G), S = sum_m W s_m, S_k = sum_m W kappa_m s_m over interior nodes:
//   K       = sum_m kappa_m - sum_x kappa^2 phi / (1 + kappa)           (every axis)
//   K_theta = sum_m kappa_m |s_m|^2 - sum_x kappa / (1 + kappa) S . S_k
// Threads [0, boxN) take the footprint box nodes (gather form, FP64), threads [boxN,
// boxN + ND) the design points; grid-stride, fixed order, one partial per block.
template <int DIM, bool ROT>
__global__ __launch_bounds__(256) void k_coupling(Grid g, Design D, const double *__restrict__ B,
                                                  const double *__restrict__ krD, double *__restrict__ part) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // node sums (K, K_theta), design sums (K, K_theta)
    int o[3];
    box_origin<DIM>(D, B, o);
    const long long total = D.boxN + D.ND;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        if (t < D.boxN) {
            int x[3];
            if (!box_node<DIM>(g, D, o, t, x)) continue;
            double d[3];
            double kap = 0.0, phi = 0.0, S[3] = {0, 0, 0}, Sk[3] = {0, 0, 0};
            gather_design<DIM, double, ROT, 1>(D, B, x, d, 0, [&](long long m, double W, const double r[3], const int *) {
                const double km = krD[m];
                // s_m = a x (x^ref - x^G), x^ref - x^G = d - r (r = x - x^ref)
                const double rp = pick3(d, D.pi) - r[D.pi], rq = pick3(d, D.pj) - r[D.pj];
                kap += W * km;
                phi += W;
                S[D.pi] += W * -rq;
                S[D.pj] += W * rp;
                Sk[D.pi] += W * km * -rq;
                Sk[D.pj] += W * km * rp;
            });
            const double f = kap / (1.0 + kap);
            v[0] += f * kap * phi;
            v[1] += f * (S[0] * Sk[0] + S[1] * Sk[1] + S[2] * Sk[2]);
        } else {
            const long long m = t - D.boxN;
            double xi[3];
            design_xi<DIM>(D, m, xi);
            Pose P;
            pose_point(D, B, xi, P);
            const double km = krD[m], rp = pick3(P.r, D.pi), rq = pick3(P.r, D.pj);
            v[2] += km;
            v[3] += km * (rp * rp + rq * rq);
        }
    }
    block_reduce_store<4, 256>(v, part);
}

// One block: K[0..2] (zero beyond dim), K[3] from the nb partials (fixed order).
template <int DIM>
__global__ __launch_bounds__(1024) void k_coupling_finish(const double *__restrict__ part, unsigned nb,
                                                          double *__restrict__ K) {
    __shared__ double s[4];
    reduce_partials<4, 1024>(part, nullptr, nb, s);
    if (threadIdx.x == 0) {
        const double kt = s[2] - s[0];
        for (int a = 0; a < 3; a++) K[a] = a < DIM ? kt : 0.0;
        K[3] = s[3] - s[1];
    }
}

}  // namespace lks
