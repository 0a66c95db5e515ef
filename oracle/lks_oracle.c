/*
 * lks_oracle.c -- plain serial FP64 CPU oracle (test infrastructure only).
 *
 * Written from the paper, section by section:
 *   Sec. 2.2  lattice kinetic scheme: local equilibrium (Eq. local_equilibrium_function),
 *             viscosity relation, moments p*, u* (Eqs. p_tmp, u_tmp), Brinkman
 *             correction (Eqs. p, u); macroscopic values prescribed on boundaries.
 *   Sec. 2.3  grid separation: kappa / u^S mapping (Eqs. kappa_mapping, us_mapping),
 *             weight function (Eq. weight_function), u^ref (Eq. u_mapping), rigid-body
 *             position and velocity (Eqs. rigid_body_position, rigid_body_velocity).
 *   Sec. 2.4  explicit Euler update of the body (Eqs. equation_of_motion_*_discretized).
 *   Sec. 3.1  N_itr fluid <-> body iterations per step (Algorithm 1, time loop).
 *   Eq. brinkman_coefficient  kappa_ref(gamma).
 *   Sec. 2.5 / App. A  adjoint. The oracle differentiates the discrete forward map
 *             exactly (reverse mode). In the fluid interior this is the ALKS of
 *             Eqs. ap_tmp..as with (p~, u~, s~) the moments of the adjoint
 *             distribution; at boundaries, in the Brinkman / body terms and through
 *             the unrolled N_itr loop it is the exact transpose of the forward code.
 *             orc_gradient_paper is the paper's own variant instead (the continuous
 *             adjoint discretised like the forward; Eqs. au, axg..aomega).
 *
 * Readings where the paper is silent or garbled (each is listed in the design notes):
 *   - the -3/2 u.u sign of the equilibrium (printed with +);
 *   - w(r) = (1 + cos(pi r / 2)) / 4 (printed with 1 - cos);
 *   - velocity gradients: central differences, second-order one-sided differences
 *     along the normal on non-periodic boundary nodes;
 *   - boundary nodes are the outermost layer of non-periodic faces; a prescribed
 *     value is imposed, anything not prescribed is copied from the nearest interior
 *     node; WALL (u = 0) beats VELOCITY for u;
 *   - mapping sums run over interior nodes only, no wrap-around;
 *   - each N_itr iteration restarts the body update from the state at t-1 and uses
 *     the pose of the previous iterate; u(t) is the last iteration's fluid;
 *   - an inactive degree of freedom keeps its position and velocity from t-1.
 *
 * Everything is plain loops in the order the paper states them; no blocking, fusion
 * or reordering beyond the obvious (f_eq is evaluated once per node, then gathered).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "lks_oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define MAXQ 15

typedef struct {
    const orc_problem *P;
    int dim;
    int n[3];
    int per[3];          /* axis is periodic */
    long N;              /* analysis nodes */
    long ND;             /* design points */
    int q;
    int c[MAXQ][3];
    double w[MAXQ];
    double A;
    int axis, pi, pj;    /* rotation axis and the two axes of the rotation plane */
    int has_body;
} ctx_t;

/* ------------------------------------------------------------------ lattices */

/* D2Q9 / D3Q15 velocity sets and weights, Sec. 2.2 (weight equations). */
static void lattice_make(ctx_t *C)
{
    memset(C->c, 0, sizeof C->c);
    if (C->dim == 2) {
        static const int c2[9][2] = {{0, 0},  {1, 0},   {-1, 0}, {0, 1}, {0, -1},
                                     {1, 1},  {-1, -1}, {1, -1}, {-1, 1}};
        C->q = 9;
        for (int i = 0; i < 9; i++) {
            C->c[i][0] = c2[i][0];
            C->c[i][1] = c2[i][1];
            C->w[i] = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else {
        int k = 0;
        C->w[k++] = 2.0 / 9.0;
        for (int a = 0; a < 3; a++)
            for (int s = 1; s >= -1; s -= 2) {
                C->c[k][a] = s;
                C->w[k++] = 1.0 / 9.0;
            }
        for (int sx = 1; sx >= -1; sx -= 2)
            for (int sy = 1; sy >= -1; sy -= 2)
                for (int sz = 1; sz >= -1; sz -= 2) {
                    C->c[k][0] = sx;
                    C->c[k][1] = sy;
                    C->c[k][2] = sz;
                    C->w[k++] = 1.0 / 72.0;
                }
        C->q = 15;
    }
}

static int ctx_init(ctx_t *C, const orc_problem *P)
{
    if (!P || (P->dim != 2 && P->dim != 3)) return -1;
    memset(C, 0, sizeof *C);
    C->P = P;
    C->dim = P->dim;
    for (int a = 0; a < 3; a++) C->n[a] = P->n[a];
    if (C->dim == 2 && C->n[2] != 1) return -1;
    C->N = 1;
    for (int a = 0; a < 3; a++) {
        if (C->n[a] < 1) return -1;
        C->N *= C->n[a];
    }
    for (int a = 0; a < C->dim; a++) {
        int lo = P->bc[2 * a], hi = P->bc[2 * a + 1];
        if ((lo == ORC_PERIODIC) != (hi == ORC_PERIODIC)) return -1;
        C->per[a] = lo == ORC_PERIODIC;
        if (C->n[a] < 3) return -1;
    }
    C->per[2] = C->dim == 2 ? 1 : C->per[2];
    C->A = (1.0 / 6.0 - P->nu) * 4.5; /* nu = (1/6 - 2A/9) dx, Sec. 2.2 */
    lattice_make(C);
    C->ND = 1;
    for (int a = 0; a < 3; a++) C->ND *= P->nd[a] > 0 ? P->nd[a] : 0;
    C->has_body = C->ND > 0;
    if (C->dim == 2 && C->has_body && P->nd[2] != 1) return -1;
    C->axis = C->dim == 2 ? 2 : P->axis;
    if (C->axis < 0 || C->axis > 2) return -1;
    C->pi = (C->axis + 1) % 3;
    C->pj = (C->axis + 2) % 3;
    if (C->has_body && (P->n_itr < 1 || P->mass <= 0 || P->inertia <= 0)) return -1;
    return 0;
}

/* ---------------------------------------------------------------- grid helpers */

static long nid(const ctx_t *C, const int x[3])
{
    return x[0] + (long)C->n[0] * (x[1] + (long)C->n[1] * x[2]);
}

static void coords(const ctx_t *C, long id, int x[3])
{
    x[0] = (int)(id % C->n[0]);
    x[1] = (int)((id / C->n[0]) % C->n[1]);
    x[2] = (int)(id / ((long)C->n[0] * C->n[1]));
}

/* Interior node: not on the outermost layer of a non-periodic face. */
static int interior(const ctx_t *C, const int x[3])
{
    for (int a = 0; a < C->dim; a++)
        if (!C->per[a] && (x[a] == 0 || x[a] == C->n[a] - 1)) return 0;
    return 1;
}

/* y = x + s*c (c a lattice vector); wraps periodic axes; 0 if it leaves the grid. */
static int shifted(const ctx_t *C, const int x[3], const int c[3], int s, int y[3])
{
    for (int a = 0; a < 3; a++) {
        int v = x[a] + s * c[a];
        if (a < C->dim && C->per[a]) {
            v %= C->n[a];
            if (v < 0) v += C->n[a];
        } else if (v < 0 || v >= C->n[a]) {
            return 0;
        }
        y[a] = v;
    }
    return 1;
}

static long along(const ctx_t *C, const int x[3], int a, int d)
{
    int y[3] = {x[0], x[1], x[2]};
    int v = x[a] + d;
    if (C->per[a]) {
        v %= C->n[a];
        if (v < 0) v += C->n[a];
    }
    y[a] = v;
    return nid(C, y);
}

/* Stencil of the derivative along axis a at node x: up to 3 (node, coefficient)
 * pairs. Central differences; second-order one-sided on non-periodic boundary
 * nodes (reading of the unstated discretisation of du/dx in Sec. 2.2). */
static int deriv_stencil(const ctx_t *C, const int x[3], int a, long nodes[3], double coef[3])
{
    if (C->per[a] || (x[a] > 0 && x[a] < C->n[a] - 1)) {
        nodes[0] = along(C, x, a, 1);
        coef[0] = 0.5;
        nodes[1] = along(C, x, a, -1);
        coef[1] = -0.5;
        return 2;
    }
    if (x[a] == 0) {
        nodes[0] = along(C, x, a, 0);
        coef[0] = -1.5;
        nodes[1] = along(C, x, a, 1);
        coef[1] = 2.0;
        nodes[2] = along(C, x, a, 2);
        coef[2] = -0.5;
        return 3;
    }
    nodes[0] = along(C, x, a, 0);
    coef[0] = 1.5;
    nodes[1] = along(C, x, a, -1);
    coef[1] = -2.0;
    nodes[2] = along(C, x, a, -2);
    coef[2] = 0.5;
    return 3;
}

/* ------------------------------------------------------------ LKS (Sec. 2.2) */

/* f_eq_i at every node, Eq. local_equilibrium_function:
 *   f_i = w_i (3p + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) + w_i A sum_ab (du_b/dx_a + du_a/dx_b) c_a c_b */
static void equilibrium_all(const ctx_t *C, const double *s, double *feq)
{
    const int d = C->dim;
    const double *p = s;
    for (long id = 0; id < C->N; id++) {
        int x[3];
        coords(C, id, x);
        double u[3] = {0, 0, 0};
        for (int b = 0; b < d; b++) u[b] = s[(1 + b) * C->N + id];
        double S[3][3] = {{0}}; /* S[a][b] = du_b/dx_a */
        for (int a = 0; a < d; a++) {
            long nodes[3];
            double coef[3];
            int k = deriv_stencil(C, x, a, nodes, coef);
            for (int b = 0; b < d; b++) {
                double v = 0;
                for (int j = 0; j < k; j++) v += coef[j] * s[(1 + b) * C->N + nodes[j]];
                S[a][b] = v;
            }
        }
        double uu = 0;
        for (int b = 0; b < d; b++) uu += u[b] * u[b];
        for (int i = 0; i < C->q; i++) {
            double cu = 0, cSc = 0;
            for (int a = 0; a < d; a++) cu += C->c[i][a] * u[a];
            for (int a = 0; a < d; a++)
                for (int b = 0; b < d; b++) cSc += (S[a][b] + S[b][a]) * C->c[i][a] * C->c[i][b];
            feq[(long)i * C->N + id] =
                C->w[i] * (3.0 * p[id] + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) + C->w[i] * C->A * cSc;
        }
    }
}

/* p*(x) = 1/3 sum_i f_i(x - c_i), u*(x) = sum_i c_i f_i(x - c_i), Eqs. p_tmp, u_tmp,
 * at interior nodes (tau = 1 streaming). Non-interior nodes of s_out are untouched. */
static void lks_gather(const ctx_t *C, const double *s_in, double *s_out, double *feq)
{
    const int d = C->dim;
    equilibrium_all(C, s_in, feq);
    for (long id = 0; id < C->N; id++) {
        int x[3];
        coords(C, id, x);
        if (!interior(C, x)) continue;
        double ps = 0, us[3] = {0, 0, 0};
        for (int i = 0; i < C->q; i++) {
            int y[3];
            shifted(C, x, C->c[i], -1, y); /* always inside for an interior node */
            double f = feq[(long)i * C->N + nid(C, y)];
            ps += f / 3.0;
            for (int a = 0; a < d; a++) us[a] += C->c[i][a] * f;
        }
        s_out[id] = ps;
        for (int a = 0; a < d; a++) s_out[(1 + a) * C->N + id] = us[a];
    }
}

/* Boundary treatment of a non-interior node: which of p, u are prescribed, their
 * values, and the nearest interior node that supplies the others. */
typedef struct {
    int p_fixed, u_fixed;
    double p, u[3];
    long inward;
} bcnode_t;

static void bc_resolve(const ctx_t *C, const int x[3], bcnode_t *r)
{
    const orc_problem *P = C->P;
    int wall = 0, vel = -1, pres = -1;
    int y[3] = {x[0], x[1], x[2]};
    for (int a = 0; a < C->dim; a++) {
        if (C->per[a]) continue;
        int f = -1;
        if (x[a] == 0) {
            f = 2 * a;
            y[a] = 1;
        } else if (x[a] == C->n[a] - 1) {
            f = 2 * a + 1;
            y[a] = C->n[a] - 2;
        }
        if (f < 0) continue;
        if (P->bc[f] == ORC_WALL) wall = 1;
        if (P->bc[f] == ORC_VELOCITY && vel < 0) vel = f;
        if (P->bc[f] == ORC_PRESSURE && pres < 0) pres = f;
    }
    r->inward = nid(C, y);
    r->p_fixed = pres >= 0;
    r->p = pres >= 0 ? P->bc_p[pres] : 0.0;
    r->u_fixed = wall || vel >= 0;
    for (int a = 0; a < 3; a++) r->u[a] = wall ? 0.0 : (vel >= 0 ? P->bc_u[vel][a] : 0.0);
}

/* Macroscopic values prescribed directly at the boundaries (Sec. 2.2, last
 * paragraph); non-prescribed values copy the nearest interior node. */
static void apply_bc(const ctx_t *C, double *s)
{
    const int d = C->dim;
    for (long id = 0; id < C->N; id++) {
        int x[3];
        coords(C, id, x);
        if (interior(C, x)) continue;
        bcnode_t r;
        bc_resolve(C, x, &r);
        s[id] = r.p_fixed ? r.p : s[r.inward];
        for (int a = 0; a < d; a++)
            s[(1 + a) * C->N + id] = r.u_fixed ? r.u[a] : s[(1 + a) * C->N + r.inward];
    }
}

/* Transpose of apply_bc acting on a cotangent of the full state: cotangents of copied
 * values move to the interior node they were copied from; boundary cotangents end. */
static void apply_bc_rev(const ctx_t *C, double *sb)
{
    const int d = C->dim;
    for (long id = 0; id < C->N; id++) {
        int x[3];
        coords(C, id, x);
        if (interior(C, x)) continue;
        bcnode_t r;
        bc_resolve(C, x, &r);
        if (!r.p_fixed) sb[r.inward] += sb[id];
        sb[id] = 0;
        for (int a = 0; a < d; a++) {
            if (!r.u_fixed) sb[(1 + a) * C->N + r.inward] += sb[(1 + a) * C->N + id];
            sb[(1 + a) * C->N + id] = 0;
        }
    }
}

/* ----------------------------------------------------- grid separation (Sec. 2.3) */

/* Eq. brinkman_coefficient. */
static double kappa_of(const orc_problem *P, double g)
{
    return P->kappa_max * P->q * g / ((1.0 - g) + P->q);
}

static double dkappa_of(const orc_problem *P, double g)
{
    double den = (1.0 - g) + P->q;
    return P->kappa_max * P->q * (1.0 + P->q) / (den * den);
}

/* Eq. weight_function, read as the cosine kernel (1 + cos(pi r / 2)) / 4, |r| < 2. */
static double wk(double r)
{
    return fabs(r) < 2.0 ? 0.25 * (1.0 + cos(M_PI * r / 2.0)) : 0.0;
}

static double dwk(double r)
{
    return fabs(r) < 2.0 ? -(M_PI / 8.0) * sin(M_PI * r / 2.0) : 0.0;
}

/* Local coordinate of design point m relative to the rotation centre (design-grid
 * spacing 1, centre at the middle of the design grid). */
static void design_xi(const ctx_t *C, long m, double xi[3])
{
    const int *nd = C->P->nd;
    long i = m % nd[0], j = (m / nd[0]) % nd[1], k = m / ((long)nd[0] * nd[1]);
    xi[0] = (double)i - 0.5 * (nd[0] - 1);
    xi[1] = (double)j - 0.5 * (nd[1] - 1);
    xi[2] = C->dim == 3 ? (double)k - 0.5 * (nd[2] - 1) : 0.0;
}

typedef struct {
    double X[3];   /* x^ref: analysis-grid position */
    double US[3];  /* u^S,ref: velocity of the point */
    double r[3];   /* R(theta) xi = x^ref - x^G */
    double axr[3]; /* a x r (unit rotation axis a) */
} pose_t;

/* Eqs. rigid_body_position / rigid_body_velocity, rotation about the axis `axis`
 * through x^G (in 2D the z axis, the only case the paper writes out). */
static void pose_point(const ctx_t *C, const double *B, const double xi[3], pose_t *o)
{
    const double c = cos(B[6]), s = sin(B[6]), om = B[7];
    const int a = C->axis, i = C->pi, j = C->pj;
    o->r[a] = xi[a];
    o->r[i] = c * xi[i] - s * xi[j];
    o->r[j] = s * xi[i] + c * xi[j];
    o->axr[a] = 0.0;
    o->axr[i] = -o->r[j];
    o->axr[j] = o->r[i];
    for (int b = 0; b < 3; b++) {
        o->X[b] = B[b] + o->r[b];
        o->US[b] = B[3 + b] + om * o->axr[b];
    }
}

/* The 4^d taps of a design point: nodes with |x_a - X_a| < 2 on each axis, clipped
 * to interior nodes (the sums over the analysis domain run over interior nodes). */
typedef struct {
    int count;
    long id[64];
    double W[64];
    double dW[64][3]; /* dW/dX_a */
} taps_t;

static void taps_of(const ctx_t *C, const double X[3], taps_t *T)
{
    const int d = C->dim;
    int base[3] = {0, 0, 0};
    for (int a = 0; a < d; a++) base[a] = (int)floor(X[a]) - 1;
    int lim[3] = {4, 4, d == 3 ? 4 : 1};
    T->count = 0;
    for (int tz = 0; tz < lim[2]; tz++)
        for (int ty = 0; ty < lim[1]; ty++)
            for (int tx = 0; tx < lim[0]; tx++) {
                int x[3] = {base[0] + tx, base[1] + ty, d == 3 ? base[2] + tz : 0};
                int ok = 1;
                for (int a = 0; a < 3; a++)
                    if (x[a] < 0 || x[a] >= C->n[a]) ok = 0;
                if (!ok || !interior(C, x)) continue;
                double w1[3], dw1[3];
                for (int a = 0; a < d; a++) {
                    double r = (double)x[a] - X[a];
                    w1[a] = wk(r);
                    dw1[a] = dwk(r);
                }
                double W = 1.0;
                for (int a = 0; a < d; a++) W *= w1[a];
                if (W == 0.0) continue;
                int k = T->count++;
                T->id[k] = nid(C, x);
                T->W[k] = W;
                for (int a = 0; a < 3; a++) {
                    double g = 0.0;
                    if (a < d) {
                        g = -dw1[a]; /* d/dX of w(x - X) */
                        for (int b = 0; b < d; b++)
                            if (b != a) g *= w1[b];
                    }
                    T->dW[k][a] = g;
                }
            }
}

/* kappa(x) = sum_m W kappa_ref_m, u^S(x) = sum_m W u^S,ref_m; Eqs. kappa_mapping,
 * us_mapping (design spacing 1, so dOmega_ref = 1). */
static void spread(const ctx_t *C, const double *kr, const double *B, double *kap, double *uS)
{
    const int d = C->dim;
    memset(kap, 0, sizeof(double) * C->N);
    memset(uS, 0, sizeof(double) * d * C->N);
    for (long m = 0; m < C->ND; m++) {
        double xi[3];
        pose_t ps;
        taps_t T;
        design_xi(C, m, xi);
        pose_point(C, B, xi, &ps);
        taps_of(C, ps.X, &T);
        for (int k = 0; k < T.count; k++) {
            kap[T.id[k]] += T.W[k] * kr[m];
            for (int a = 0; a < d; a++) uS[a * C->N + T.id[k]] += T.W[k] * ps.US[a];
        }
    }
}

/* u^ref_m = sum_x W u(x), Eq. u_mapping. */
static void interp_point(const ctx_t *C, const double *u, const taps_t *T, double UR[3])
{
    UR[0] = UR[1] = UR[2] = 0.0;
    for (int k = 0; k < T->count; k++)
        for (int a = 0; a < C->dim; a++) UR[a] += T->W[k] * u[a * C->N + T->id[k]];
}

/* --------------------------------------------------- body update (Sec. 2.4) */

static int dof_t(const ctx_t *C, int a)
{
    return a < C->dim && (C->P->dof_mask & (1 << a));
}

static int dof_r(const ctx_t *C)
{
    return (C->P->dof_mask & ORC_DOF_ROT) != 0;
}

/* u^G(t) = u^G(t-1) + F/M, x^G(t) = x^G(t-1) + u^G(t); omega, theta likewise. */
static void body_update(const ctx_t *C, const double *Bprev, const double *FT, double *Bout)
{
    const orc_problem *P = C->P;
    for (int b = 0; b < 12; b++) Bout[b] = Bprev[b];
    for (int a = 0; a < 3; a++)
        if (dof_t(C, a)) {
            Bout[3 + a] = Bprev[3 + a] + FT[a] / P->mass;
            Bout[a] = Bprev[a] + Bout[3 + a];
        }
    if (dof_r(C)) {
        Bout[7] = Bprev[7] + FT[3] / P->inertia;
        Bout[6] = Bprev[6] + Bout[7];
    }
}

/* Transpose of body_update: from the cotangent Bb of its output, the cotangent of
 * the force/torque (FTb) and the contribution to the cotangent of Bprev. */
static void body_update_rev(const ctx_t *C, const double *Bb, double *FTb, double *Bprevb)
{
    const orc_problem *P = C->P;
    for (int a = 0; a < 3; a++) {
        if (dof_t(C, a)) {
            double ut = Bb[3 + a] + Bb[a];
            FTb[a] = ut / P->mass;
            Bprevb[a] += Bb[a];
            Bprevb[3 + a] += ut;
        } else {
            FTb[a] = 0.0;
            Bprevb[a] += Bb[a];
            Bprevb[3 + a] += Bb[3 + a];
        }
    }
    if (dof_r(C)) {
        double wt = Bb[7] + Bb[6];
        FTb[3] = wt / P->inertia;
        Bprevb[6] += Bb[6];
        Bprevb[7] += wt;
    } else {
        FTb[3] = 0.0;
        Bprevb[6] += Bb[6];
        Bprevb[7] += Bb[7];
    }
}

/* F = sum_m kappa_ref (u^ref - u^S,ref); T = sum_m e_zab r_a kappa_ref (u^ref - u^S,ref)_b
 * with r = x^ref - x^G, about the rotation axis (Eqs. 5, 7 discretised in Sec. 2.4). */
static void force_point(const ctx_t *C, double kr, const pose_t *ps, const double UR[3], double FT[4])
{
    double D[3] = {0, 0, 0};
    for (int a = 0; a < C->dim; a++) D[a] = UR[a] - ps->US[a];
    for (int a = 0; a < 3; a++) FT[a] += kr * D[a];
    FT[3] += kr * (ps->r[C->pi] * D[C->pj] - ps->r[C->pj] * D[C->pi]);
}

/* ------------------------------------------------- one coupled step (Alg. 1) */

typedef struct {
    double *feq;   /* Q*N */
    double *ustar; /* d*N */
    double *kap;   /* N */
    double *uS;    /* d*N */
    /* per-iteration records for the reverse sweep (K = n_itr) */
    double *Bk;    /* (K+1)*12 */
    double *kapk;  /* K*N */
    double *uSk;   /* K*d*N */
    double *uk;    /* K*d*N */
} work_t;

static int work_alloc(const ctx_t *C, work_t *W, int with_rec)
{
    const int d = C->dim, K = C->has_body ? C->P->n_itr : 0;
    memset(W, 0, sizeof *W);
    W->feq = malloc(sizeof(double) * C->q * C->N);
    W->ustar = malloc(sizeof(double) * d * C->N);
    W->kap = malloc(sizeof(double) * C->N);
    W->uS = malloc(sizeof(double) * d * C->N);
    W->Bk = malloc(sizeof(double) * (K + 1) * 12);
    if (!W->feq || !W->ustar || !W->kap || !W->uS || !W->Bk) return -2;
    if (with_rec && K > 0) {
        W->kapk = malloc(sizeof(double) * K * C->N);
        W->uSk = malloc(sizeof(double) * K * d * C->N);
        W->uk = malloc(sizeof(double) * K * d * C->N);
        if (!W->kapk || !W->uSk || !W->uk) return -2;
    }
    return 0;
}

static void work_free(work_t *W)
{
    free(W->feq);
    free(W->ustar);
    free(W->kap);
    free(W->uS);
    free(W->Bk);
    free(W->kapk);
    free(W->uSk);
    free(W->uk);
}

/* The N_itr fluid <-> body iterations of one step (Alg. 1, inner loop).
 * In: u* (W->ustar) and B(t-1). Out: u(t) into the velocity part of s_out (interior
 * nodes), B(t) into Bout, iterates into W->Bk (and the per-iteration fields when the
 * record arrays exist). */
static void body_loop(const ctx_t *C, const double *kr, double *s_out, const double *Bprev,
                      double *Bout, work_t *W)
{
    const int d = C->dim, K = C->P->n_itr;
    double *u = s_out + C->N; /* velocity components of s_out */
    memcpy(W->Bk, Bprev, sizeof(double) * 12);
    for (int k = 0; k < K; k++) {
        const double *B = W->Bk + 12 * k;
        double *kap = W->kapk ? W->kapk + (long)k * C->N : W->kap;
        double *uS = W->uSk ? W->uSk + (long)k * d * C->N : W->uS;
        /* rigid body -> fluid */
        spread(C, kr, B, kap, uS);
        for (long id = 0; id < C->N; id++) {
            int x[3];
            coords(C, id, x);
            if (!interior(C, x)) continue;
            for (int a = 0; a < d; a++)
                u[a * C->N + id] =
                    (W->ustar[a * C->N + id] + kap[id] * uS[a * C->N + id]) / (1.0 + kap[id]);
        }
        if (W->uk) memcpy(W->uk + (long)k * d * C->N, u, sizeof(double) * d * C->N);
        /* fluid -> rigid body */
        double FT[4] = {0, 0, 0, 0};
        for (long m = 0; m < C->ND; m++) {
            double xi[3], UR[3];
            pose_t ps;
            taps_t T;
            design_xi(C, m, xi);
            pose_point(C, B, xi, &ps);
            taps_of(C, ps.X, &T);
            interp_point(C, u, &T, UR);
            force_point(C, kr[m], &ps, UR, FT);
        }
        body_update(C, Bprev, FT, W->Bk + 12 * (k + 1));
    }
    memcpy(Bout, W->Bk + 12 * K, sizeof(double) * 12);
}

static void step_fwd(const ctx_t *C, const double *kr, const double *s_in, const double *Bin,
                     double *s_out, double *Bout, work_t *W)
{
    const int d = C->dim;
    memcpy(s_out, s_in, sizeof(double) * (d + 1) * C->N);
    lks_gather(C, s_in, s_out, W->feq);
    if (C->has_body) {
        memcpy(W->ustar, s_out + C->N, sizeof(double) * d * C->N);
        body_loop(C, kr, s_out, Bin, Bout, W);
    } else {
        memcpy(Bout, Bin, sizeof(double) * 12);
    }
    apply_bc(C, s_out);
}

/* ------------------------------------------------------- reverse sweep */

/* The LKS gather reversed (the exact transpose; in the fluid interior it is the ALKS of
 * Eqs. ap_tmp..as_tmp). g_i(x) = pb(x)/3 + c_i . ub(x) at interior x is the cotangent of
 * f_i(x - c_i); with the moments pi = sum_i w_i g_i(y + c_i), ups = sum_i w_i c_i g_i,
 * sig = sum_i w_i c_i c_i g_i at node y and the forward velocity u(y) of s_in:
 *   nb_p(y) = 3 pi,  nb_u(y) = 3 ups + 9 sig u - 3 pi u + (transpose of the gradient
 *   stencil applied to 2A sig).
 * ups_out (optional, d*N): the moment ups itself (the paper's u~* of Eq. au_tmp). */
static void alks_gather(const ctx_t *C, const double *s_in, const double *sb, const double *ustb,
                        double *nb, double *ups_out)
{
    const int d = C->dim, Q = C->q;
    const long N = C->N;
    memset(nb, 0, sizeof(double) * (d + 1) * N);
    if (ups_out) memset(ups_out, 0, sizeof(double) * d * N);
    for (long id = 0; id < N; id++) {
        int y[3];
        coords(C, id, y);
        double u[3] = {0, 0, 0};
        for (int b = 0; b < d; b++) u[b] = s_in[(1 + b) * N + id];
        double Sb[3][3] = {{0}};
        for (int i = 0; i < Q; i++) {
            int z[3];
            if (!shifted(C, y, C->c[i], 1, z) || !interior(C, z)) continue;
            long zi = nid(C, z);
            double fb = sb[zi] / 3.0;
            for (int a = 0; a < d; a++) fb += C->c[i][a] * ustb[a * N + zi];
            double cu = 0;
            for (int a = 0; a < d; a++) cu += C->c[i][a] * u[a];
            nb[id] += 3.0 * C->w[i] * fb;
            for (int b = 0; b < d; b++)
                nb[(1 + b) * N + id] +=
                    C->w[i] * fb * (3.0 * C->c[i][b] + 9.0 * cu * C->c[i][b] - 3.0 * u[b]);
            if (ups_out)
                for (int b = 0; b < d; b++) ups_out[b * N + id] += C->w[i] * C->c[i][b] * fb;
            for (int a = 0; a < d; a++)
                for (int b = 0; b < d; b++)
                    Sb[a][b] += 2.0 * C->A * C->w[i] * fb * C->c[i][a] * C->c[i][b];
        }
        /* transpose of the velocity-gradient stencil at y */
        for (int a = 0; a < d; a++) {
            long nodes[3];
            double coef[3];
            int k = deriv_stencil(C, y, a, nodes, coef);
            for (int b = 0; b < d; b++)
                for (int j = 0; j < k; j++) nb[(1 + b) * N + nodes[j]] += coef[j] * Sb[a][b];
        }
    }
}

/* Reverse of one coupled step. s_in, Bin: forward state at t-1. sb (in: cotangent of
 * S(t), out: of S(t-1)), Bb (same for the body), krb accumulates d/dkappa_ref. */
static void step_rev(const ctx_t *C, const double *kr, const double *s_in, const double *Bin,
                     double *sb, double *Bb, double *krb, work_t *W, double *scratch)
{
    const int d = C->dim;
    const long N = C->N;
    /* recompute the forward step with per-iteration records */
    double *s_out = scratch;                 /* (d+1)*N */
    double *ustb = scratch + (d + 1) * N;    /* d*N: cotangent of u* */
    double *ubk = ustb + d * N;              /* d*N: cotangent of u^(k) */
    double *kb = ubk + d * N;                /* N: cotangent of kappa(x) */
    double *uSb = kb + N;                    /* d*N: cotangent of u^S(x) */
    double *nb = uSb + d * N;                /* (d+1)*N: cotangent of S(t-1) */
    memcpy(s_out, s_in, sizeof(double) * (d + 1) * N);
    lks_gather(C, s_in, s_out, W->feq);
    double Btmp[12];
    if (C->has_body) {
        memcpy(W->ustar, s_out + N, sizeof(double) * d * N);
        body_loop(C, kr, s_out, Bin, Btmp, W);
    }

    /* boundary values -> interior values they were copied from */
    apply_bc_rev(C, sb);

    /* body loop, reversed (the N_itr iterations unrolled, last first) */
    if (C->has_body) {
        const int K = C->P->n_itr;
        double Bnext[12], Bprevb[12];
        memcpy(Bnext, Bb, sizeof Bnext);
        memset(Bprevb, 0, sizeof Bprevb);
        memset(ustb, 0, sizeof(double) * d * N);
        for (int k = K - 1; k >= 0; k--) {
            const double *B = W->Bk + 12 * k;
            const double *kap = W->kapk + (long)k * N;
            const double *uS = W->uSk + (long)k * d * N;
            const double *uk = W->uk + (long)k * d * N;
            double FTb[4];
            body_update_rev(C, Bnext, FTb, Bprevb);
            double Bkb[12];
            memset(Bkb, 0, sizeof Bkb);
            if (k == K - 1)
                memcpy(ubk, sb + N, sizeof(double) * d * N);
            else
                memset(ubk, 0, sizeof(double) * d * N);
            /* force/torque and interpolation, reversed; per-point pose cotangents are
             * folded into Bkb directly (the pose is linear in x^G, u^G, omega). */
            double *Xb = malloc(sizeof(double) * 3 * C->ND);
            double *USb = malloc(sizeof(double) * 3 * C->ND);
            double *rb = malloc(sizeof(double) * 3 * C->ND);
            for (long m = 0; m < C->ND; m++) {
                double xi[3], UR[3], D[3] = {0, 0, 0}, Db[3] = {0, 0, 0};
                pose_t ps;
                taps_t T;
                design_xi(C, m, xi);
                pose_point(C, B, xi, &ps);
                taps_of(C, ps.X, &T);
                interp_point(C, uk, &T, UR);
                for (int a = 0; a < d; a++) D[a] = UR[a] - ps.US[a];
                for (int a = 0; a < d; a++) Db[a] = kr[m] * (FTb[a] + FTb[3] * ps.axr[a]);
                double g = 0;
                for (int a = 0; a < d; a++) g += FTb[a] * D[a];
                g += FTb[3] * (ps.r[C->pi] * D[C->pj] - ps.r[C->pj] * D[C->pi]);
                krb[m] += g;
                double *xb = Xb + 3 * m, *usb = USb + 3 * m, *rbm = rb + 3 * m;
                for (int a = 0; a < 3; a++) xb[a] = usb[a] = rbm[a] = 0.0;
                rbm[C->pi] = FTb[3] * kr[m] * D[C->pj];
                rbm[C->pj] = -FTb[3] * kr[m] * D[C->pi];
                for (int a = 0; a < d; a++) usb[a] = -Db[a];
                for (int t = 0; t < T.count; t++) {
                    double dot = 0;
                    for (int a = 0; a < d; a++) {
                        ubk[a * N + T.id[t]] += T.W[t] * Db[a];
                        dot += Db[a] * uk[a * N + T.id[t]];
                    }
                    for (int a = 0; a < d; a++) xb[a] += T.dW[t][a] * dot;
                }
            }
            /* Brinkman correction u = (u* + kappa u^S)/(1 + kappa), reversed */
            for (long id = 0; id < N; id++) {
                int x[3];
                coords(C, id, x);
                kb[id] = 0;
                for (int a = 0; a < d; a++) uSb[a * N + id] = 0;
                if (!interior(C, x)) continue;
                double kp = kap[id], inv = 1.0 / (1.0 + kp), acc = 0;
                for (int a = 0; a < d; a++) {
                    double ub = ubk[a * N + id];
                    ustb[a * N + id] += ub * inv;
                    acc += ub * (uS[a * N + id] - uk[a * N + id]) * inv;
                    uSb[a * N + id] = ub * kp * inv;
                }
                kb[id] = acc;
            }
            /* mapping, reversed */
            for (long m = 0; m < C->ND; m++) {
                double xi[3];
                pose_t ps;
                taps_t T;
                design_xi(C, m, xi);
                pose_point(C, B, xi, &ps);
                taps_of(C, ps.X, &T);
                double *xb = Xb + 3 * m, *usb = USb + 3 * m;
                for (int t = 0; t < T.count; t++) {
                    long id = T.id[t];
                    krb[m] += T.W[t] * kb[id];
                    double dot = kb[id] * kr[m];
                    for (int a = 0; a < d; a++) {
                        usb[a] += T.W[t] * uSb[a * N + id];
                        dot += uSb[a * N + id] * ps.US[a];
                    }
                    for (int a = 0; a < d; a++) xb[a] += T.dW[t][a] * dot;
                }
            }
            /* pose, reversed: x^ref = x^G + R xi, u^S,ref = u^G + omega a x (R xi) */
            const double om = B[7];
            for (long m = 0; m < C->ND; m++) {
                double xi[3];
                pose_t ps;
                design_xi(C, m, xi);
                pose_point(C, B, xi, &ps);
                const double *xb = Xb + 3 * m, *usb = USb + 3 * m, *rbm = rb + 3 * m;
                const int i = C->pi, j = C->pj;
                /* dr/dtheta = a x r; a x (dr/dtheta) = -(r_i, r_j) in the plane */
                double dr_i = -ps.r[j], dr_j = ps.r[i];
                for (int a = 0; a < 3; a++) {
                    Bkb[a] += xb[a];
                    Bkb[3 + a] += usb[a];
                }
                Bkb[7] += usb[i] * ps.axr[i] + usb[j] * ps.axr[j];
                Bkb[6] += (xb[i] + rbm[i]) * dr_i + (xb[j] + rbm[j]) * dr_j +
                          om * (usb[i] * (-ps.r[i]) + usb[j] * (-ps.r[j]));
            }
            free(Xb);
            free(USb);
            free(rb);
            if (k > 0)
                memcpy(Bnext, Bkb, sizeof Bnext);
            else
                for (int b = 0; b < 12; b++) Bprevb[b] += Bkb[b];
        }
        memcpy(Bb, Bprevb, sizeof Bprevb);
    } else {
        memcpy(ustb, sb + N, sizeof(double) * d * N);
    }

    /* LKS gather, reversed (exact transpose; ALKS Eqs. ap_tmp..as in the interior) */
    alks_gather(C, s_in, sb, ustb, nb, NULL);
    memcpy(sb, nb, sizeof(double) * (d + 1) * N);
}

/* ---------------------------------------------------------------- public API */

static double objective_value(const ctx_t *C, const double *B0, const double *B1)
{
    int o = C->P->objective;
    if (o == ORC_OBJ_ANGLE) return B1[6] - B0[6];
    return B1[o] - B0[o];
}

int orc_kappa_ref(const orc_problem *P, const double *gamma, double *kappa_ref)
{
    ctx_t C;
    if (ctx_init(&C, P) || !gamma || !kappa_ref) return -1;
    for (long m = 0; m < C.ND; m++) kappa_ref[m] = kappa_of(P, gamma[m]);
    return 0;
}

int orc_step(const orc_problem *P, const double *gamma, const double *s_in,
             const double *b_in, double *s_out, double *b_out)
{
    ctx_t C;
    if (ctx_init(&C, P) || !s_in || !s_out || !b_in || !b_out) return -1;
    if (C.has_body && !gamma) return -1;
    work_t W;
    double *kr = malloc(sizeof(double) * (C.ND > 0 ? C.ND : 1));
    int rc = work_alloc(&C, &W, 0);
    if (rc == 0 && kr) {
        for (long m = 0; m < C.ND; m++) kr[m] = kappa_of(P, gamma[m]);
        step_fwd(&C, kr, s_in, b_in, s_out, b_out, &W);
    }
    work_free(&W);
    free(kr);
    return rc;
}

int orc_forward(const orc_problem *P, const double *gamma, double *state, double *body,
                double *traj, double *J)
{
    ctx_t C;
    if (ctx_init(&C, P) || !state || !body || P->n_steps < 0) return -1;
    if (C.has_body && !gamma) return -1;
    const long S = (C.dim + 1) * C.N;
    work_t W;
    double *kr = malloc(sizeof(double) * (C.ND > 0 ? C.ND : 1));
    double *tmp = malloc(sizeof(double) * S);
    int rc = work_alloc(&C, &W, 0);
    if (rc == 0 && kr && tmp) {
        double B0[12], B1[12];
        memcpy(B0, body, sizeof B0);
        for (long m = 0; m < C.ND; m++) kr[m] = kappa_of(P, gamma[m]);
        if (traj) memcpy(traj, body, sizeof B0);
        for (int t = 1; t <= P->n_steps; t++) {
            step_fwd(&C, kr, state, body, tmp, B1, &W);
            memcpy(state, tmp, sizeof(double) * S);
            memcpy(body, B1, sizeof B1);
            if (traj) memcpy(traj + 12L * t, body, sizeof B1);
        }
        if (J) *J = objective_value(&C, B0, body);
    } else {
        rc = -2;
    }
    work_free(&W);
    free(kr);
    free(tmp);
    return rc;
}

int orc_gradient(const orc_problem *P, const double *gamma, const double *state0,
                 const double *body0, double seed, const double *dstate_T, const double *dbody_T,
                 double *grad, double *J, double *dstate0, double *dbody0)
{
    ctx_t C;
    if (ctx_init(&C, P) || !state0 || !body0 || !gamma || !grad || P->n_steps < 0) return -1;
    const int d = C.dim;
    const long N = C.N, S = (d + 1) * N;
    const int NT = P->n_steps;
    work_t W;
    double *kr = malloc(sizeof(double) * (C.ND > 0 ? C.ND : 1));
    double *krb = calloc(C.ND > 0 ? C.ND : 1, sizeof(double));
    double *states = malloc(sizeof(double) * S * (NT + 1));
    double *bodies = malloc(sizeof(double) * 12 * (NT + 1));
    double *sb = calloc(S, sizeof(double));
    double *scratch = malloc(sizeof(double) * ((d + 1) * N * 2 + 3 * d * N + N));
    int rc = work_alloc(&C, &W, 1);
    if (rc || !kr || !krb || !states || !bodies || !sb || !scratch) {
        rc = -2;
        goto done;
    }
    for (long m = 0; m < C.ND; m++) kr[m] = kappa_of(P, gamma[m]);
    /* forward, storing every state (plain; the oracle is run on small problems) */
    memcpy(states, state0, sizeof(double) * S);
    memcpy(bodies, body0, sizeof(double) * 12);
    for (int t = 1; t <= NT; t++)
        step_fwd(&C, kr, states + S * (t - 1), bodies + 12 * (t - 1), states + S * t,
                 bodies + 12 * t, &W);
    if (J) *J = objective_value(&C, bodies, bodies + 12 * NT);
    /* reverse, from the terminal adjoint values: seed on the objective's coordinate plus
       the given cotangents of the final state and body (Sec. 3.4) */
    double Bb[12];
    memset(Bb, 0, sizeof Bb);
    Bb[P->objective == ORC_OBJ_ANGLE ? 6 : P->objective] = seed;
    if (dbody_T)
        for (int j = 0; j < 8; j++) Bb[j] += dbody_T[j];
    if (dstate_T) memcpy(sb, dstate_T, sizeof(double) * S);
    for (int t = NT; t >= 1; t--)
        step_rev(&C, kr, states + S * (t - 1), bodies + 12 * (t - 1), sb, Bb, krb, &W, scratch);
    for (long m = 0; m < C.ND; m++) grad[m] = krb[m] * dkappa_of(P, gamma[m]);
    /* J = q(N_t) - q(0): the initial value enters with weight -1 */
    Bb[P->objective == ORC_OBJ_ANGLE ? 6 : P->objective] -= seed;
    if (dstate0) memcpy(dstate0, sb, sizeof(double) * S);
    if (dbody0) memcpy(dbody0, Bb, sizeof Bb);
done:
    work_free(&W);
    free(kr);
    free(krb);
    free(states);
    free(bodies);
    free(sb);
    free(scratch);
    return rc;
}

/* ------------------------------------------------ the paper's adjoint variant (Sec. 2.5)
 * The sensitivity as the paper derives it: the continuous adjoint of the fluid and body
 * equations, discretised like the forward (App. A), instead of the exact reverse of the
 * discrete map. Objective J = sum_t J_I(t) with J_I = omega (Eq. objective2, theta(t1) =
 * integral of omega) or u^G_a (Eq. objective1). Per time level t = N_t .. 1, backwards:
 *  - the ALKS (Eqs. ap_tmp..as_tmp): p~*, u~*, s~* at t gathered from f~eq of level t+1,
 *    f~eq_i = p~ + c_i.(3 u~ + 9 s~ u - 3 p~ u - 2A div s~) with the forward u at t+1
 *    (alks_gather carries (3 p~, 3 u~ + 9 s~ u - 3 p~ u - 2A div s~) and returns the
 *    moments; the boundary values are taken through the transpose of the forward
 *    boundary copies, the same reading as the exact adjoint);
 *  - N_itr iterations at the pose B(t) (Algorithm 1, adjoint loop):
 *      Eq. au:  u~ = (u~* + (u~G kappa + w~ S_k) / 3) / (1 + kappa), with kappa = sum_m W
 *               kappa_m and S_k = sum_m W kappa_m (a x r_m) (p~ = p~*, s~ = s~*);
 *      Eqs. axg, aug, atheta, aomega for x~G, u~G, theta~, w~ at t from their values at
 *               t+1, their right-hand sides at level t taken with the u~G, w~ of the
 *               iteration's start (x~G feeds u~G, theta~ feeds w~ in the same iteration);
 *  - Eq. design_sensitivity: dJ/dkappa_m += 3 sum_x W (u - u^S).u~ - u~G.(u^ref - u^S,ref)_m
 *    - w~ (a x r_m).(u^ref - u^S,ref)_m.
 * Readings (the paper is silent): the level N_t + 1 adjoint is zero (the sources -dJ_I/d.
 * enter at every level, which at t1 gives the paper's stated terminal values); the u~G,
 * w~ iteration starts from the values of level t+1; the sensitivity uses the final
 * values of level t; Eq. au's "u*" is read as u~*; an inactive degree of freedom has zero
 * adjoints. Not the exact derivative of the discrete forward map: O(dt) and Brinkman
 * differences remain (compared with the exact sweep and finite differences in tests).
 * Pinned by its agreement with the exact adjoint (0.1-3 %), which a mistake in Eq. au or
 * in the sensitivity breaks; parity unpinned for the pose-derivative terms of Eqs. axg
 * and atheta, whose effect stays below that difference in every case tried. */
int orc_gradient_paper(const orc_problem *P, const double *gamma, const double *state0,
                       const double *body0, double *grad, double *J)
{
    ctx_t C;
    if (ctx_init(&C, P) || !state0 || !body0 || !gamma || !grad || P->n_steps < 0 || !C.has_body) return -1;
    const int d = C.dim, K = P->n_itr, ax = C.axis, pi = C.pi, pj = C.pj;
    const long N = C.N, S = (d + 1) * N, ND = C.ND;
    const int NT = P->n_steps;
    work_t W;
    double *kr = malloc(sizeof(double) * ND), *krb = calloc(ND, sizeof(double));
    double *states = malloc(sizeof(double) * S * (NT + 1)), *bodies = malloc(sizeof(double) * 12 * (NT + 1));
    double *sb = calloc(S, sizeof(double)), *nb = calloc(S, sizeof(double));
    double *ups = calloc(d * N, sizeof(double)), *upsn = calloc(d * N, sizeof(double));
    double *kap = malloc(sizeof(double) * N), *uS = malloc(sizeof(double) * d * N);
    double *phi = malloc(sizeof(double) * N), *Sv = malloc(sizeof(double) * 3 * N);
    double *Sk = malloc(sizeof(double) * 3 * N), *Rp = malloc(sizeof(double) * 3 * N);
    double *ut = malloc(sizeof(double) * d * N), *h = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * d * N);
    double *Du = malloc(sizeof(double) * 9 * ND), *Dv = malloc(sizeof(double) * 3 * ND);
    int rc = work_alloc(&C, &W, 0);
    if (rc || !kr || !krb || !states || !bodies || !sb || !nb || !ups || !upsn || !kap || !uS || !phi || !Sv ||
        !Sk || !Rp || !ut || !h || !q || !Du || !Dv) {
        rc = -2;
        goto done;
    }
    for (long m = 0; m < ND; m++) kr[m] = kappa_of(P, gamma[m]);
    memcpy(states, state0, sizeof(double) * S);
    memcpy(bodies, body0, sizeof(double) * 12);
    for (int t = 1; t <= NT; t++)
        step_fwd(&C, kr, states + S * (t - 1), bodies + 12 * (t - 1), states + S * t, bodies + 12 * t, &W);
    if (J) *J = objective_value(&C, bodies, bodies + 12 * NT);
    /* dJ_I / d(u^G_a) and dJ_I / d(omega) */
    double dJdU[3] = {0, 0, 0}, dJdOm = 0.0;
    if (P->objective == ORC_OBJ_ANGLE) dJdOm = 1.0;
    else dJdU[P->objective] = 1.0;
    /* body adjoints of level t+1 */
    double Xn[3] = {0, 0, 0}, Un[3] = {0, 0, 0}, Thn = 0.0, Omn = 0.0;
    for (int t = NT; t >= 1; t--) {
        const double *st = states + S * t, *B = bodies + 12 * t;
        const double *u = st + N;
        const double om = B[7];
        apply_bc_rev(&C, sb);
        /* fields at the pose B(t) */
        spread(&C, kr, B, kap, uS);
        memset(phi, 0, sizeof(double) * N);
        memset(Sv, 0, sizeof(double) * 3 * N);
        memset(Sk, 0, sizeof(double) * 3 * N);
        memset(Rp, 0, sizeof(double) * 3 * N);
        double sum_k = 0.0, sum_ks[3] = {0, 0, 0}, sum_ks2 = 0.0;
        for (long m = 0; m < ND; m++) {
            double xi[3], UR[3];
            pose_t ps;
            taps_t T;
            design_xi(&C, m, xi);
            pose_point(&C, B, xi, &ps);
            taps_of(&C, ps.X, &T);
            double rp[3] = {ps.r[0], ps.r[1], ps.r[2]};
            rp[ax] = 0.0; /* part of r across the rotation axis */
            for (int k = 0; k < T.count; k++) {
                long id = T.id[k];
                phi[id] += T.W[k];
                for (int a = 0; a < 3; a++) {
                    Sv[a * N + id] += T.W[k] * ps.axr[a];
                    Sk[a * N + id] += T.W[k] * kr[m] * ps.axr[a];
                    Rp[a * N + id] += T.W[k] * rp[a];
                }
            }
            interp_point(&C, u, &T, UR);
            for (int a = 0; a < 3; a++) Dv[3 * m + a] = a < d ? UR[a] - ps.US[a] : 0.0;
            for (int g = 0; g < 3; g++)
                for (int b = 0; b < 3; b++) {
                    double v = 0.0;
                    if (g < d && b < d)
                        for (int k = 0; k < T.count; k++) v += T.dW[k][g] * u[b * N + T.id[k]];
                    Du[9 * m + 3 * g + b] = v;
                }
            sum_k += kr[m];
            for (int a = 0; a < 3; a++) sum_ks[a] += kr[m] * ps.axr[a];
            sum_ks2 += kr[m] * (ps.axr[0] * ps.axr[0] + ps.axr[1] * ps.axr[1] + ps.axr[2] * ps.axr[2]);
        }
        double Ucur[3] = {Un[0], Un[1], Un[2]}, Omcur = Omn, Xt[3] = {0, 0, 0}, Tht = 0.0;
        for (int it = 0; it < K; it++) {
            /* Eq. au at the nodes, and the node sums of Eqs. aug, atheta, aomega */
            double NU[3] = {0, 0, 0}, NO = 0.0, NTh = 0.0;
            for (long id = 0; id < N; id++) {
                int x[3];
                coords(&C, id, x);
                h[id] = 0.0;
                for (int a = 0; a < d; a++) ut[a * N + id] = q[a * N + id] = 0.0;
                if (!interior(&C, x)) continue;
                const double kp = kap[id];
                for (int a = 0; a < d; a++) {
                    const double v = (ups[a * N + id] + (Ucur[a] * kp + Omcur * Sk[a * N + id]) / 3.0) / (1.0 + kp);
                    ut[a * N + id] = v;
                    h[id] += (u[a * N + id] - uS[a * N + id]) * v;
                    q[a * N + id] = kp * v;
                    NU[a] += 3.0 * kp * v * phi[id];
                    NO += 3.0 * kp * v * Sv[a * N + id];
                    NTh += 3.0 * kp * v * (-om * Rp[a * N + id]);
                }
            }
            /* design sums of Eqs. axg, atheta */
            double AXG[3] = {0, 0, 0}, ATH = NTh;
            for (long m = 0; m < ND; m++) {
                double xi[3];
                pose_t ps;
                taps_t T;
                design_xi(&C, m, xi);
                pose_point(&C, B, xi, &ps);
                taps_of(&C, ps.X, &T);
                double Dh[3] = {0, 0, 0}, Dq[3][3] = {{0}};
                for (int k = 0; k < T.count; k++)
                    for (int g = 0; g < d; g++) {
                        Dh[g] += T.dW[k][g] * h[T.id[k]];
                        for (int b = 0; b < d; b++) Dq[g][b] += T.dW[k][g] * q[b * N + T.id[k]];
                    }
                const double km = kr[m], *s_m = ps.axr, *Dum = Du + 9 * m, *Dvm = Dv + 3 * m;
                double w[3] = {0, 0, 0}; /* w_b = sum_g s_g Du_gb */
                for (int b = 0; b < 3; b++)
                    for (int g = 0; g < 3; g++) w[b] += s_m[g] * Dum[3 * g + b];
                for (int a = 0; a < d; a++) {
                    double v = -3.0 * km * Dh[a];
                    for (int b = 0; b < d; b++)
                        v += 3.0 * ps.US[b] * Dq[a][b] + km * Ucur[b] * Dum[3 * a + b] + Omcur * km * s_m[b] * Dum[3 * a + b];
                    AXG[a] += v;
                }
                double v = 0.0, rpm[3] = {ps.r[0], ps.r[1], ps.r[2]};
                rpm[ax] = 0.0;
                for (int g = 0; g < d; g++) v += -3.0 * km * s_m[g] * Dh[g];
                for (int b = 0; b < d; b++)
                    for (int g = 0; g < d; g++) v += 3.0 * ps.US[b] * Dq[g][b] * s_m[g];
                for (int a = 0; a < d; a++) v += km * Ucur[a] * w[a] + om * km * Ucur[a] * rpm[a];
                v += Omcur * km * (s_m[pi] * Dvm[pj] - s_m[pj] * Dvm[pi]);
                v += Omcur * km * (ps.r[pi] * w[pj] - ps.r[pj] * w[pi]);
                ATH += v;
            }
            /* Eqs. axg, aug (translation) and atheta, aomega (rotation) */
            double Unew[3] = {0, 0, 0}, Omnew = 0.0;
            for (int a = 0; a < d; a++) {
                if (!(P->dof_mask & (1 << a))) {
                    Xt[a] = 0.0;
                    continue;
                }
                Xt[a] = Xn[a] + AXG[a];
                Unew[a] = Un[a] + (Xt[a] + NU[a] - Ucur[a] * sum_k - Omcur * sum_ks[a] - dJdU[a]) / P->mass;
            }
            if (P->dof_mask & ORC_DOF_ROT) {
                Tht = Thn + ATH;
                double us_dot = 0.0;
                for (int a = 0; a < d; a++) us_dot += Ucur[a] * sum_ks[a];
                Omnew = Omn + (Tht + NO - us_dot - Omcur * sum_ks2 - dJdOm) / P->inertia;
            } else {
                Tht = 0.0;
            }
            for (int a = 0; a < 3; a++) Ucur[a] = Unew[a];
            Omcur = Omnew;
        }
        /* Eq. design_sensitivity at level t (h from the last iteration's u~) */
        for (long m = 0; m < ND; m++) {
            double xi[3];
            pose_t ps;
            taps_t T;
            design_xi(&C, m, xi);
            pose_point(&C, B, xi, &ps);
            taps_of(&C, ps.X, &T);
            double H = 0.0;
            for (int k = 0; k < T.count; k++) H += T.W[k] * h[T.id[k]];
            double g = 3.0 * H;
            for (int a = 0; a < d; a++) g -= (Ucur[a] + Omcur * ps.axr[a]) * Dv[3 * m + a];
            krb[m] += g;
        }
        /* the ALKS input of level t: 3 u~ + 9 s~ u - 3 p~ u - 2A div s~ = (the gather's
         * combination, folded) + 3 (u~ - u~*) */
        for (long id = 0; id < N; id++)
            for (int a = 0; a < d; a++) sb[(1 + a) * N + id] += 3.0 * (ut[a * N + id] - ups[a * N + id]);
        for (int a = 0; a < 3; a++) {
            Xn[a] = Xt[a];
            Un[a] = Ucur[a];
        }
        Thn = Tht;
        Omn = Omcur;
        alks_gather(&C, states + S * (t - 1), sb, sb + N, nb, upsn);
        double *tmp = sb;
        sb = nb;
        nb = tmp;
        tmp = ups;
        ups = upsn;
        upsn = tmp;
    }
    for (long m = 0; m < ND; m++) grad[m] = krb[m] * dkappa_of(P, gamma[m]);
done:
    work_free(&W);
    free(kr);
    free(krb);
    free(states);
    free(bodies);
    free(sb);
    free(nb);
    free(ups);
    free(upsn);
    free(kap);
    free(uS);
    free(phi);
    free(Sv);
    free(Sk);
    free(Rp);
    free(ut);
    free(h);
    free(q);
    free(Du);
    free(Dv);
    return rc;
}

int orc_map_design(const orc_problem *P, const double *kappa_ref, const double *body,
                   double *kappa, double *uS)
{
    ctx_t C;
    if (ctx_init(&C, P) || !kappa_ref || !body || !kappa || !uS || !C.has_body) return -1;
    spread(&C, kappa_ref, body, kappa, uS);
    return 0;
}

int orc_interp(const orc_problem *P, const double *u, const double *body, double *uref)
{
    ctx_t C;
    if (ctx_init(&C, P) || !u || !body || !uref || !C.has_body) return -1;
    for (long m = 0; m < C.ND; m++) {
        double xi[3], UR[3];
        pose_t ps;
        taps_t T;
        design_xi(&C, m, xi);
        pose_point(&C, body, xi, &ps);
        taps_of(&C, ps.X, &T);
        interp_point(&C, u, &T, UR);
        for (int a = 0; a < C.dim; a++) uref[a * C.ND + m] = UR[a];
    }
    return 0;
}

int orc_force(const orc_problem *P, const double *kappa_ref, const double *uref,
              const double *body, double *FT)
{
    ctx_t C;
    if (ctx_init(&C, P) || !kappa_ref || !uref || !body || !FT || !C.has_body) return -1;
    FT[0] = FT[1] = FT[2] = FT[3] = 0.0;
    for (long m = 0; m < C.ND; m++) {
        double xi[3], UR[3] = {0, 0, 0};
        pose_t ps;
        design_xi(&C, m, xi);
        pose_point(&C, body, xi, &ps);
        for (int a = 0; a < C.dim; a++) UR[a] = uref[a * C.ND + m];
        force_point(&C, kappa_ref[m], &ps, UR, FT);
    }
    return 0;
}

int orc_body_step(const orc_problem *P, const double *FT, const double *body_prev,
                  double *body_out)
{
    ctx_t C;
    if (ctx_init(&C, P) || !FT || !body_prev || !body_out) return -1;
    body_update(&C, body_prev, FT, body_out);
    return 0;
}

/* F (T) is affine in u^G (omega) for a frozen pose and frozen u*; the slope is read
 * off two evaluations one unit apart. */
int orc_coupling(const orc_problem *P, const double *gamma, const double *state,
                 const double *body, double *K)
{
    ctx_t C;
    if (ctx_init(&C, P) || !gamma || !state || !body || !K || !C.has_body) return -1;
    const int d = C.dim;
    const long N = C.N;
    work_t W;
    double *kr = malloc(sizeof(double) * C.ND);
    double *s1 = malloc(sizeof(double) * (d + 1) * N);
    double *u = malloc(sizeof(double) * d * N);
    int rc = work_alloc(&C, &W, 0);
    if (rc || !kr || !s1 || !u) {
        rc = -2;
        goto done;
    }
    for (long m = 0; m < C.ND; m++) kr[m] = kappa_of(P, gamma[m]);
    memcpy(s1, state, sizeof(double) * (d + 1) * N);
    lks_gather(&C, state, s1, W.feq);
    for (int dof = 0; dof < 4; dof++) {
        double FT2[2][4];
        for (int e = 0; e < 2; e++) {
            double B[12];
            memcpy(B, body, sizeof B);
            if (dof < 3)
                B[3 + dof] += e;
            else
                B[7] += e;
            spread(&C, kr, B, W.kap, W.uS);
            for (long id = 0; id < N; id++)
                for (int a = 0; a < d; a++)
                    u[a * N + id] =
                        (s1[(1 + a) * N + id] + W.kap[id] * W.uS[a * N + id]) / (1.0 + W.kap[id]);
            double FT[4] = {0, 0, 0, 0};
            for (long m = 0; m < C.ND; m++) {
                double xi[3], UR[3];
                pose_t ps;
                taps_t T;
                design_xi(&C, m, xi);
                pose_point(&C, B, xi, &ps);
                taps_of(&C, ps.X, &T);
                interp_point(&C, u, &T, UR);
                force_point(&C, kr[m], &ps, UR, FT);
            }
            memcpy(FT2[e], FT, sizeof FT);
        }
        K[dof] = dof < 3 ? -(FT2[1][dof] - FT2[0][dof]) : -(FT2[1][3] - FT2[0][3]);
        if (dof >= d && dof < 3) K[dof] = 0.0;
    }
done:
    work_free(&W);
    free(kr);
    free(s1);
    free(u);
    return rc;
}

/* ------------------------------------------------------------------ filter (Sec. 3.2) */

/* Weight of Eq. filter between design points i and j (index space, spacing one). */
static double filter_w(double R, const int *a, const int *b) {
    double d2 = 0.0;
    for (int k = 0; k < 3; k++) d2 += (double)(a[k] - b[k]) * (a[k] - b[k]);
    const double d = sqrt(d2);
    return d <= R ? (R - d) / R : 0.0;
}

static int filter_args(int dim, const int nd[3], double R) {
    if ((dim != 2 && dim != 3) || !nd || !(R > 0.0)) return -1;
    if (nd[0] < 1 || nd[1] < 1 || nd[2] < 1 || (dim == 2 && nd[2] != 1)) return -1;
    return 0;
}

/* Visits every design point j with |x_i - x_j| <= R and calls f(j, w_ij). */
#define FOR_NEIGHBOURS(nd, R, xi, j, w, BODY)                                                \
    do {                                                                                     \
        const int r_ = (int)floor(R);                                                        \
        int xj[3];                                                                           \
        for (xj[2] = xi[2] - r_; xj[2] <= xi[2] + r_; xj[2]++)                               \
            for (xj[1] = xi[1] - r_; xj[1] <= xi[1] + r_; xj[1]++)                           \
                for (xj[0] = xi[0] - r_; xj[0] <= xi[0] + r_; xj[0]++) {                     \
                    if (xj[0] < 0 || xj[0] >= nd[0] || xj[1] < 0 || xj[1] >= nd[1] ||        \
                        xj[2] < 0 || xj[2] >= nd[2])                                         \
                        continue;                                                            \
                    const double w = filter_w(R, xi, xj);                                    \
                    if (w <= 0.0) continue;                                                  \
                    const long j = xj[0] + (long)nd[0] * (xj[1] + (long)nd[1] * xj[2]);      \
                    BODY;                                                                    \
                }                                                                            \
    } while (0)

static double proj_den(double beta, double eta) { return tanh(beta * eta) + tanh(beta * (1.0 - eta)); }

int orc_filter(int dim, const int nd[3], double R, double beta, double eta, const double *g, double *gt,
               double *gh) {
    if (filter_args(dim, nd, R) || !g || !gt || !gh || !(beta > 0.0)) return -1;
    const long n = (long)nd[0] * nd[1] * nd[2];
    const double den = proj_den(beta, eta);
    for (long i = 0; i < n; i++) {
        const int xi[3] = {(int)(i % nd[0]), (int)((i / nd[0]) % nd[1]), (int)(i / ((long)nd[0] * nd[1]))};
        double num = 0.0, wsum = 0.0;
        FOR_NEIGHBOURS(nd, R, xi, j, w, {
            num += w * g[j];
            wsum += w;
        });
        gt[i] = num / wsum;
        gh[i] = (tanh(beta * eta) + tanh(beta * (gt[i] - eta))) / den;
    }
    return 0;
}

int orc_filter_adjoint(int dim, const int nd[3], double R, double beta, double eta, const double *gt,
                       const double *gbh, double *gb) {
    if (filter_args(dim, nd, R) || !gt || !gbh || !gb || !(beta > 0.0)) return -1;
    const long n = (long)nd[0] * nd[1] * nd[2];
    const double den = proj_den(beta, eta);
    for (long j = 0; j < n; j++) gb[j] = 0.0;
    /* gb_j = sum_i (dgh_i / dgt_i) gbh_i w_ij / W_i, scattered from every i */
    for (long i = 0; i < n; i++) {
        const int xi[3] = {(int)(i % nd[0]), (int)((i / nd[0]) % nd[1]), (int)(i / ((long)nd[0] * nd[1]))};
        double wsum = 0.0;
        FOR_NEIGHBOURS(nd, R, xi, j, w, {
            (void)j;
            wsum += w;
        });
        const double th = tanh(beta * (gt[i] - eta));
        const double gbt = gbh[i] * beta * (1.0 - th * th) / den;
        FOR_NEIGHBOURS(nd, R, xi, j, w, { gb[j] += w * gbt / wsum; });
    }
    return 0;
}

/* ------------------------------------------------- cyclic periodic design (Sec. 4.2) */

/* The design is defined on one sector and repeated by the rotations by 2 pi k / n_sec
 * about the rotation axis through the design grid's centre. Plane coordinates (u, v)
 * run along the two axes of the rotation plane (pi, pj), w along the rotation axis. On a
 * Cartesian design grid the rotation maps grid points to grid points for n_sec = 1, 2,
 * and, when the plane is square, 4; by a quarter turn (u, v) -> (nv - 1 - v, u).
 * Sector (the design variables), in plane coordinates:
 *   n_sec = 1: the whole plane, index u + nu v;
 *   n_sec = 2: plane indices q = u + nu v with q <= nu nv - 1 - q (the half turn maps q
 *              to nu nv - 1 - q); sector index q;
 *   n_sec = 4: 0 <= u < ceil(n/2), 0 <= v < floor(n/2), index u + ceil(n/2) v, then the
 *              centre (odd n) as the last index.
 * Sector index of a grid point = plane index + (plane sector size) * w. */
typedef struct {
    int pi, pj, ax, nu, nv, nw, n_sec;
    long plane, sector_plane;
} cyc_t;

static int cyc_init(const orc_problem *P, int n_sec, cyc_t *Y) {
    ctx_t C;
    if (ctx_init(&C, P) || !C.has_body) return -1;
    Y->pi = C.pi;
    Y->pj = C.pj;
    Y->ax = C.axis;
    Y->nu = P->nd[C.pi];
    Y->nv = P->nd[C.pj];
    Y->nw = P->nd[C.axis];
    Y->n_sec = n_sec;
    Y->plane = (long)Y->nu * Y->nv;
    if (n_sec == 1) Y->sector_plane = Y->plane;
    else if (n_sec == 2) Y->sector_plane = (Y->plane + 1) / 2;
    else if (n_sec == 4 && Y->nu == Y->nv) Y->sector_plane = (long)((Y->nu + 1) / 2) * (Y->nu / 2) + (Y->nu % 2);
    else return -1;
    return 0;
}

/* sector plane index of (u, v) if the point lies in the sector, else -1 */
static long cyc_in_sector(const cyc_t *Y, int u, int v) {
    const long q = u + (long)Y->nu * v;
    if (Y->n_sec == 1) return q;
    if (Y->n_sec == 2) return q <= Y->plane - 1 - q ? q : -1;
    const int n = Y->nu, cu = (n + 1) / 2, cv = n / 2;
    if (u < cu && v < cv) return u + (long)cu * v;
    if (n % 2 == 1 && u == n / 2 && v == n / 2) return (long)cu * cv;
    return -1;
}

/* one rotation of the group: half turn for n_sec = 2, quarter turn for n_sec = 4 */
static void cyc_rotate(const cyc_t *Y, int *u, int *v) {
    if (Y->n_sec == 2) {
        *u = Y->nu - 1 - *u;
        *v = Y->nv - 1 - *v;
    } else if (Y->n_sec == 4) {
        const int t = *u;
        *u = Y->nv - 1 - *v;
        *v = t;
    }
}

/* sector index of design point m: rotate until the point lies in the sector */
static long cyc_sector_of(const cyc_t *Y, long m, const int nd[3]) {
    int c[3] = {(int)(m % nd[0]), (int)((m / nd[0]) % nd[1]), (int)(m / ((long)nd[0] * nd[1]))};
    int u = c[Y->pi], v = c[Y->pj];
    const int w = c[Y->ax];
    for (int k = 0; k < Y->n_sec; k++) {
        const long s = cyc_in_sector(Y, u, v);
        if (s >= 0) return s + Y->sector_plane * w;
        cyc_rotate(Y, &u, &v);
    }
    return -1; /* not reached for a valid sector */
}

long orc_cyclic_sector_points(const orc_problem *P, int n_sec) {
    cyc_t Y;
    if (cyc_init(P, n_sec, &Y)) return -1;
    return Y.sector_plane * Y.nw;
}

int orc_cyclic_expand(const orc_problem *P, int n_sec, const double *gs, double *g) {
    cyc_t Y;
    if (cyc_init(P, n_sec, &Y) || !gs || !g) return -1;
    const long ND = (long)P->nd[0] * P->nd[1] * P->nd[2];
    for (long m = 0; m < ND; m++) {
        const long s = cyc_sector_of(&Y, m, P->nd);
        if (s < 0) return -2;
        g[m] = gs[s];
    }
    return 0;
}

/* transpose of the expansion: every design point's sensitivity goes to its sector point */
int orc_cyclic_collect(const orc_problem *P, int n_sec, const double *grad, double *gs) {
    cyc_t Y;
    if (cyc_init(P, n_sec, &Y) || !grad || !gs) return -1;
    const long ND = (long)P->nd[0] * P->nd[1] * P->nd[2];
    for (long s = 0; s < Y.sector_plane * Y.nw; s++) gs[s] = 0.0;
    for (long m = 0; m < ND; m++) {
        const long s = cyc_sector_of(&Y, m, P->nd);
        if (s < 0) return -2;
        gs[s] += grad[m];
    }
    return 0;
}
