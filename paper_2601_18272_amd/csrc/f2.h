// f2.h -- the paper's adjoint variant on gfx950 (Sec. 2.5, App. A, Algorithm 1's adjoint loop).
//
// The paper differentiates the continuous equations and discretises the adjoint like the
// forward; lks_adjoint with LKS_FLAG_PAPER_ADJOINT computes that variant instead of the
// exact reverse of the discrete map. Objective J = sum_t J_I(t) with J_I = omega
// (Eq. objective2) or u^G_a (Eq. objective1). Per time level t, backwards:
//  - ALKS (Eqs. ap_tmp..as_tmp): the adjoint LKS kernels with the paper's variables,
//    carrying (3 p~, V = 3 u~ + 9 s~ u - 3 p~ u - 2A div s~); they also return the
//    moment u~* (here "ups") on the whole grid;
//  - N_itr iterations at the pose B(t): Eq. au on the footprint box,
//      u~ = (u~* + (u~G kappa + w~ S_k) / 3) / (1 + kappa),
//    then Eqs. axg, aug, atheta, aomega for the body adjoints (k_f2_node, k_f2_design,
//    k_f2_update), the right-hand sides taken with the u~G, w~ of the iteration's start;
//  - Eq. design_sensitivity into the kappa_ref cotangent, and V on the box from the last
//    iteration's u~ for the next ALKS step.
// Readings: adjoint zero at level N_t + 1 (the sources -dJ_I/d. enter at every level);
// the iteration starts from the values of level t+1; the sensitivity uses the final ones;
// Eq. au's u* read as u~*; boundary values through the transpose of the forward copies;
// an inactive degree of freedom has zero adjoints.
//
// Notation per design point m at the pose: r_m = x^ref - x^G, s_m = a x r_m (the
// direction of dx^ref/dtheta), u^S,ref = u^G + omega s_m; on the box: kappa, phi = sum W,
// S = sum W s_m, S_k = sum W kappa_m s_m, R = sum W r_m across the axis, u^S.
#pragma once
#include "body.h"

namespace lks {

// Record of the body adjoints of one time level (FP64, device): values of level t+1, the
// iterate of level t, and the level's x~G, theta~.
enum {
    F2_XN = 0, F2_UN = 3, F2_THN = 6, F2_OMN = 7,  // level t+1
    F2_UC = 8, F2_OMC = 11,                         // u~G, w~ of the current iteration
    F2_XT = 12, F2_THT = 15,                        // x~G, theta~ of level t
    F2_REC = 16
};
// Box fields of a level: kappa, phi, S[3], S_k[3], R[3], u^S[3], u[3] (forward velocity).
enum { F2F_K = 0, F2F_PHI = 1, F2F_S = 2, F2F_SK = 5, F2F_R = 8, F2F_US = 11, F2F_U = 14, F2F_N = 17 };
// Node partial sums: 3 kappa u~ phi (3), 3 kappa u~.S, 3 kappa u~.(-omega R).
constexpr int F2_NNODE = 5;
// Design partial sums: axg (3), atheta, sum kappa, sum kappa s (3), sum kappa |s|^2.
constexpr int F2_NDES = 9;
constexpr int F2_NT = 256;

// Fields of level t on the footprint box at the pose B (gather form, FP64 arms); block 0
// also starts the level's iteration from the values of level t+1.
template <int DIM, typename T, bool ROT>
__global__ __launch_bounds__(F2_NT) void k_f2_fields(Grid g, Design D, const double *__restrict__ Bprev,
                                                     const double *__restrict__ B, const T *__restrict__ krT,
                                                     const T *__restrict__ state, T *__restrict__ F,
                                                     double *__restrict__ rec) {
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        const int j = threadIdx.x;
        if (j < 3) rec[F2_UC + j] = rec[F2_UN + j];
        else rec[F2_OMC] = rec[F2_OMN];
    }
    if (l >= D.boxN) return;
    const long long bN = D.boxN;
    int o[3], x[3];
    box_origin<DIM>(D, Bprev, o);
    double f[F2F_N];
#pragma unroll
    for (int i = 0; i < F2F_N; i++) f[i] = 0.0;
    if (box_node<DIM>(g, D, o, l, x)) {
        double d[3];
        T k = 0, phi = 0, wr[3] = {0, 0, 0}, wkr[3] = {0, 0, 0};
        gather_design<DIM, T, ROT, 1>(D, B, x, d, 0, [&](long long m, T W, const T r[3], const int *) {
            const T km = krT[m];
            k += W * km;
            phi += W;
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                wr[a] += W * r[a];
                wkr[a] += W * km * r[a];
            }
        });
        // sum W r_m = phi d - sum W r, sum W kappa_m r_m = kappa d - sum W kappa_m r (r = x - x^ref)
        double arm[3] = {0, 0, 0}, armk[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            arm[a] = (double)phi * d[a] - (double)wr[a];
            armk[a] = (double)k * d[a] - (double)wkr[a];
        }
        const int ip = D.pi, jq = D.pj;
        f[F2F_K] = (double)k;
        f[F2F_PHI] = (double)phi;
        f[F2F_S + ip] = -pick3(arm, jq);
        f[F2F_S + jq] = pick3(arm, ip);
        f[F2F_SK + ip] = -pick3(armk, jq);
        f[F2F_SK + jq] = pick3(armk, ip);
        f[F2F_R + ip] = pick3(arm, ip);
        f[F2F_R + jq] = pick3(arm, jq);
        const long long id = node_id(g, x[0], x[1], x[2]);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            f[F2F_US + a] = a < DIM ? B[B_UG + a] * (double)phi + B[B_OM] * f[F2F_S + a] : 0.0;
            f[F2F_U + a] = a < DIM ? (double)(gU<T>(g, a) + state[(1 + a) * g.N + id]) : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < F2F_N; i++) F[i * bN + l] = T(f[i]);
}

// Eq. au on the box from the iteration's u~G, w~ (record) and u~* (ups, whole grid); h =
// (u - u^S).u~ and q = kappa u~ for the design pass; node sums of Eqs. aug, aomega,
// atheta. With last, also V = (the ALKS combination at the node, boundary-folded) +
// 3 (u~ - u~*) into ustb, the box input of the next ALKS step.
template <int DIM, typename T>
__global__ __launch_bounds__(F2_NT) void k_f2_node(Grid g, Bc bc, Design D, const double *__restrict__ Bprev,
                                                   const double *__restrict__ B, const T *__restrict__ F,
                                                   const T *__restrict__ ups, const double *__restrict__ rec,
                                                   T *__restrict__ hq, double *__restrict__ part, int last,
                                                   const T *__restrict__ ab, T *__restrict__ ustb) {
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long bN = D.boxN;
    double v[F2_NNODE] = {0, 0, 0, 0, 0};
    if (l < bN) {
        int o[3], x[3];
        box_origin<DIM>(D, Bprev, o);
        T h = 0, q[3] = {0, 0, 0};
        if (box_node<DIM>(g, D, o, l, x)) {
            const long long id = node_id(g, x[0], x[1], x[2]);
            const double kp = (double)F[F2F_K * bN + l], om = B[B_OM];
            T ubf[3] = {0, 0, 0};
            if (last) {
                T pdummy;
                fold_bc<DIM, T>(g, bc, ab, x, id, pdummy, ubf, true);
            }
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                const double us = (double)ups[a * g.N + id];
                const double ut = (us + (rec[F2_UC + a] * kp + rec[F2_OMC] * (double)F[(F2F_SK + a) * bN + l]) / 3.0) /
                                  (1.0 + kp);
                h += T((double)F[(F2F_U + a) * bN + l] - (double)F[(F2F_US + a) * bN + l]) * T(ut);
                q[a] = T(kp * ut);
                v[a] = 3.0 * kp * ut * (double)F[F2F_PHI * bN + l];
                v[3] += 3.0 * kp * ut * (double)F[(F2F_S + a) * bN + l];
                v[4] += 3.0 * kp * ut * (-om * (double)F[(F2F_R + a) * bN + l]);
                if (last) ustb[a * bN + l] = T((double)ubf[a] + 3.0 * (ut - us));
            }
        }
        hq[l] = h;
#pragma unroll
        for (int a = 0; a < 3; a++) hq[(1 + a) * bN + l] = q[a];
    }
    block_reduce_store<F2_NNODE, F2_NT>(v, part);
}

// Design pass at the pose B: with s = a x r and derivatives of the stencil weights,
//   Dh_g = sum dW/dX_g h, Dq_gb = sum dW/dX_g q_b, Du_gb = sum dW/dX_g u_b,
//   Dv = sum W u - u^S,ref. Sums of Eq. axg (a) and Eq. atheta, and the level's
// constants sum kappa, sum kappa s, sum kappa |s|^2. With sens, instead: the kappa_ref
// cotangent += 3 sum W h - (u~G + w~ s).Dv (Eq. design_sensitivity) from the final
// record values.
template <int DIM, typename T>
__global__ __launch_bounds__(F2_NT) void k_f2_design(Grid g, Design D, const double *__restrict__ Bprev,
                                                     const double *__restrict__ B, const double *__restrict__ krD,
                                                     const T *__restrict__ F, const T *__restrict__ hq,
                                                     const double *__restrict__ rec, double *__restrict__ part,
                                                     int sens, double *__restrict__ krb) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long bN = D.boxN;
    double v[F2_NDES];
#pragma unroll
    for (int i = 0; i < F2_NDES; i++) v[i] = 0.0;
    if (m < D.ND) {
        int o[3];
        box_origin<DIM>(D, Bprev, o);
        double xi[3];
        design_xi<DIM>(D, m, xi);
        Pose P;
        pose_point(D, B, xi, P);
        Taps<DIM, T> tp;
        tp.init(g, P.X, true, o, D.L);
        T Dh[3] = {0, 0, 0}, Dq[3][3] = {{0}}, Du[3][3] = {{0}}, ur[3] = {0, 0, 0}, H = 0;
        constexpr int TZ = DIM == 3 ? 4 : 1;
        for (int c = 0; c < TZ; c++) {
            const T wz = sel4(tp.w[2], c), dwz = sel4(tp.dw[2], c);
            const int cz = sel4(tp.c[2], c);
            for (int b = 0; b < 4; b++) {
                for (int a = 0; a < 4; a++) {
                    const long long bi = tp.c[0][a] + (long long)D.L[0] * (tp.c[1][b] + (long long)D.L[1] * cz);
                    const T W = tp.w[0][a] * tp.w[1][b] * wz;
                    // dW/dX_g = -w'(x_g - X_g) times the other axes' weights
                    const T dW[3] = {-tp.dw[0][a] * tp.w[1][b] * wz, -tp.w[0][a] * tp.dw[1][b] * wz,
                                     DIM == 3 ? -tp.w[0][a] * tp.w[1][b] * dwz : T(0)};
                    const T hv = hq[bi];
                    H += W * hv;
#pragma unroll
                    for (int e = 0; e < DIM; e++) {
                        const T qv = hq[(1 + e) * bN + bi], uv = F[(F2F_U + e) * bN + bi];
                        ur[e] += W * uv;
#pragma unroll
                        for (int gg = 0; gg < DIM; gg++) {
                            Dq[gg][e] += dW[gg] * qv;
                            Du[gg][e] += dW[gg] * uv;
                        }
                    }
#pragma unroll
                    for (int gg = 0; gg < DIM; gg++) Dh[gg] += dW[gg] * hv;
                }
            }
        }
        const double km = krD[m], om = B[B_OM];
        const double *s = P.axr;
        double Dv[3] = {0, 0, 0};
#pragma unroll
        for (int e = 0; e < DIM; e++) Dv[e] = (double)ur[e] - P.US[e];
        const double Uc[3] = {rec[F2_UC], rec[F2_UC + 1], rec[F2_UC + 2]}, Oc = rec[F2_OMC];
        if (sens) {
            double gs = 3.0 * (double)H;
#pragma unroll
            for (int e = 0; e < DIM; e++) gs -= (Uc[e] + Oc * s[e]) * Dv[e];
            krb[m] += gs;
        } else {
            double w[3] = {0, 0, 0};  // w_b = sum_g s_g Du_gb
#pragma unroll
            for (int b = 0; b < DIM; b++)
#pragma unroll
                for (int gg = 0; gg < DIM; gg++) w[b] += s[gg] * (double)Du[gg][b];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                double t = -3.0 * km * (double)Dh[a];
#pragma unroll
                for (int b = 0; b < DIM; b++)
                    t += 3.0 * P.US[b] * (double)Dq[a][b] + km * (Uc[b] + Oc * s[b]) * (double)Du[a][b];
                v[a] = t;
            }
            double th = 0.0;
            const int ip = D.pi, jq = D.pj;
#pragma unroll
            for (int gg = 0; gg < DIM; gg++) th -= 3.0 * km * s[gg] * (double)Dh[gg];
#pragma unroll
            for (int b = 0; b < DIM; b++)
#pragma unroll
                for (int gg = 0; gg < DIM; gg++) th += 3.0 * P.US[b] * (double)Dq[gg][b] * s[gg];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                const double rp = a == D.axis ? 0.0 : P.r[a];  // r across the axis
                th += km * Uc[a] * (w[a] + om * rp);
            }
            th += Oc * km * (pick3(s, ip) * pick3(Dv, jq) - pick3(s, jq) * pick3(Dv, ip));
            th += Oc * km * (pick3(P.r, ip) * pick3(w, jq) - pick3(P.r, jq) * pick3(w, ip));
            v[3] = th;
            v[4] = km;
#pragma unroll
            for (int a = 0; a < 3; a++) v[5 + a] = km * s[a];
            v[8] = km * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        }
    }
    if (!sens) block_reduce_store<F2_NDES, F2_NT>(v, part);
}

// One block: the fixed-order sums of the node and design partials, then Eqs. axg, aug
// (active translations) and atheta, aomega (rotation) into the record; with last, the
// level's final values become the "level t+1" values of the next level.
// seed: dL/dJ, the weight of the sources dJ_I/du^G, dJ_I/domega.
template <int DIM>
__global__ __launch_bounds__(1024) void k_f2_update(BodyParams bp, int obj, double seed, const double *__restrict__ pn,
                                                    unsigned nbn, const double *__restrict__ pd, unsigned nbd,
                                                    double *__restrict__ rec, int last) {
    __shared__ double sn[F2_NNODE], sd[F2_NDES];
    reduce_partials<F2_NNODE, 1024>(pn, nullptr, nbn, sn);
    reduce_partials<F2_NDES, 1024>(pd, nullptr, nbd, sd);
    if (threadIdx.x != 0) return;
    double dJdU[3] = {0, 0, 0}, dJdOm = 0.0;
    if (obj == 3) dJdOm = seed;
    else dJdU[obj] = seed;
    const double Uc[3] = {rec[F2_UC], rec[F2_UC + 1], rec[F2_UC + 2]}, Oc = rec[F2_OMC];
    double Un[3] = {0, 0, 0}, Om = 0.0;
    for (int a = 0; a < 3; a++) {
        if (a < DIM && (bp.dof & (1 << a))) {
            rec[F2_XT + a] = rec[F2_XN + a] + sd[a];
            Un[a] = rec[F2_UN + a] +
                    (rec[F2_XT + a] + sn[a] - Uc[a] * sd[4] - Oc * sd[5 + a] - dJdU[a]) / bp.mass;
        } else {
            rec[F2_XT + a] = 0.0;
        }
    }
    if (bp.dof & 8) {
        rec[F2_THT] = rec[F2_THN] + sd[3] + sn[4];
        double us = 0.0;
        for (int a = 0; a < DIM; a++) us += Uc[a] * sd[5 + a];
        Om = rec[F2_OMN] + (rec[F2_THT] + sn[3] - us - Oc * sd[8] - dJdOm) / bp.inertia;
    } else {
        rec[F2_THT] = 0.0;
    }
    for (int a = 0; a < 3; a++) rec[F2_UC + a] = Un[a];
    rec[F2_OMC] = Om;
    if (last) {
        for (int a = 0; a < 3; a++) {
            rec[F2_XN + a] = rec[F2_XT + a];
            rec[F2_UN + a] = Un[a];
        }
        rec[F2_THN] = rec[F2_THT];
        rec[F2_OMN] = Om;
    }
}

}  // namespace lks
