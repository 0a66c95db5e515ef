/*
 * sanitize_main.c -- TEST INFRASTRUCTURE: a driver that runs every entry point of the
 * FP64 oracle (lks_oracle.c) once on small problems, so that the oracle can be built
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py)
 * and any out-of-bounds access, leak or undefined operation in it is reported.
 *
 * It checks nothing numerically (the pins in tests/ do that); it only exercises the
 * code paths: 2D and 3D, every boundary kind, translation and rotation, terminal
 * cotangents, the coupling constants, the filter pair and the cyclic design pair.
 * Inputs are deterministic smooth fields; exit status 0 means every call returned 0.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lks_oracle.h"

static int fails = 0;

static void check(int rc, const char *what)
{
    if (rc != 0) {
        fprintf(stderr, "%s returned %d\n", what, rc);
        fails++;
    }
}

static double *vec(long n)
{
    double *v = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!v) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return v;
}

/* a smooth field in (0, 1) over n points */
static void fill(double *v, long n, double phase)
{
    for (long i = 0; i < n; i++) v[i] = 0.5 + 0.4 * sin(0.37 * (double)i + phase);
}

static void run_problem(const orc_problem *P, double theta0)
{
    const int d = P->dim;
    const long N = (long)P->n[0] * P->n[1] * P->n[2];
    const long ND = (long)P->nd[0] * P->nd[1] * P->nd[2];
    const long S = (long)(d + 1) * N;
    double *g = vec(ND), *s0 = vec(S), *s = vec(S), *b = vec(12), *b0 = vec(12);
    double *tr = vec(12L * (P->n_steps + 1));
    double *grad = vec(ND), *ds = vec(S), *db = vec(12), *sT = vec(S), *bT = vec(12);
    double *kr = vec(ND), *kap = vec(N), *uS = vec((long)d * N), *uref = vec((long)d * ND);
    double K[4], FT[4], J = 0.0;
    fill(g, ND, 0.3);
    for (long i = 0; i < N; i++) s0[N + i] = 0.04;
    for (int a = 0; a < 3; a++) b0[a] = 0.5 * P->n[a] - 0.3 * a;
    if (d == 2) b0[2] = 0.0;
    b0[6] = theta0;
    fill(sT, S, 1.1);
    fill(bT, 8, 2.2);
    memcpy(s, s0, sizeof(double) * S);
    memcpy(b, b0, sizeof(double) * 12);
    check(orc_forward(P, g, s, b, tr, &J), "orc_forward");
    check(orc_step(P, g, s0, b0, s, b), "orc_step");
    check(orc_gradient(P, g, s0, b0, 1.0, NULL, NULL, grad, &J, ds, db), "orc_gradient");
    check(orc_gradient(P, g, s0, b0, 0.5, sT, bT, grad, &J, ds, db), "orc_gradient (terminal)");
    check(orc_coupling(P, g, s0, b0, K), "orc_coupling");
    check(orc_kappa_ref(P, g, kr), "orc_kappa_ref");
    check(orc_map_design(P, kr, b0, kap, uS), "orc_map_design");
    check(orc_interp(P, s0 + N, b0, uref), "orc_interp");
    check(orc_force(P, kr, uref, b0, FT), "orc_force");
    check(orc_body_step(P, FT, b0, b), "orc_body_step");
    free(g), free(s0), free(s), free(b), free(b0), free(tr), free(grad), free(ds), free(db);
    free(sT), free(bT), free(kr), free(kap), free(uS), free(uref);
}

static void run_design(const orc_problem *P)
{
    const long ND = (long)P->nd[0] * P->nd[1] * P->nd[2];
    double *g = vec(ND), *gt = vec(ND), *gh = vec(ND), *gb = vec(ND);
    fill(g, ND, 0.7);
    for (int r = 0; r < 2; r++) {
        const double R = r ? 2.5 : 1.5;
        check(orc_filter(P->dim, P->nd, R, 8.0, 0.5, g, gt, gh), "orc_filter");
        check(orc_filter_adjoint(P->dim, P->nd, R, 8.0, 0.5, gt, g, gb), "orc_filter_adjoint");
    }
    for (int n = 1; n <= 4; n *= 2) {
        const long ns = orc_cyclic_sector_points(P, n);
        if (ns <= 0) continue;
        double *gs = vec(ns), *gsb = vec(ns);
        fill(gs, ns, 0.1);
        check(orc_cyclic_expand(P, n, gs, g), "orc_cyclic_expand");
        check(orc_cyclic_collect(P, n, g, gsb), "orc_cyclic_collect");
        free(gs), free(gsb);
    }
    free(g), free(gt), free(gh), free(gb);
}

int main(void)
{
    orc_problem P;
    memset(&P, 0, sizeof P);
    /* 2D channel: x- VELOCITY, x+ PRESSURE, WALL in y; free translation and rotation */
    P.dim = 2;
    P.n[0] = 24, P.n[1] = 16, P.n[2] = 1;
    P.bc[0] = ORC_VELOCITY, P.bc[1] = ORC_PRESSURE, P.bc[2] = ORC_WALL, P.bc[3] = ORC_WALL;
    P.bc_u[0][0] = 0.04;
    P.bc_p[1] = 0.001;
    P.nu = 0.1;
    P.nd[0] = 6, P.nd[1] = 5, P.nd[2] = 1;
    P.kappa_max = 0.5, P.q = 0.1, P.mass = 50.0, P.inertia = 500.0;
    P.axis = 2;
    P.dof_mask = ORC_DOF_TX | ORC_DOF_TY | ORC_DOF_ROT;
    P.n_itr = 3, P.n_steps = 4, P.objective = ORC_OBJ_ANGLE;
    run_problem(&P, 0.3);
    run_design(&P);
    P.nd[0] = 6, P.nd[1] = 6;
    run_design(&P);
    /* 2D periodic in y, translation objective */
    P.bc[2] = ORC_PERIODIC, P.bc[3] = ORC_PERIODIC;
    P.dof_mask = ORC_DOF_TX, P.objective = ORC_OBJ_DISP_X;
    run_problem(&P, 0.0);
    /* 3D duct: WALL on y and z, rotation about x plus axial translation */
    memset(&P, 0, sizeof P);
    P.dim = 3;
    P.n[0] = 16, P.n[1] = 12, P.n[2] = 11;
    P.bc[0] = ORC_VELOCITY, P.bc[1] = ORC_PRESSURE;
    P.bc[2] = P.bc[3] = P.bc[4] = P.bc[5] = ORC_WALL;
    P.bc_u[0][0] = 0.04;
    P.nu = 0.08;
    P.nd[0] = 4, P.nd[1] = 4, P.nd[2] = 4;
    P.kappa_max = 0.3, P.q = 0.1, P.mass = 80.0, P.inertia = 900.0;
    P.axis = 0;
    P.dof_mask = ORC_DOF_TX | ORC_DOF_ROT;
    P.n_itr = 2, P.n_steps = 3, P.objective = ORC_OBJ_ANGLE;
    run_problem(&P, 0.2);
    run_design(&P);
    /* 3D periodic in z, rotation about y, translation objective along z */
    P.bc[4] = P.bc[5] = ORC_PERIODIC;
    P.axis = 1;
    P.dof_mask = ORC_DOF_TX | ORC_DOF_TY | ORC_DOF_TZ | ORC_DOF_ROT;
    P.objective = ORC_OBJ_DISP_Z;
    run_problem(&P, 0.1);
    /* body-free */
    P.nd[0] = P.nd[1] = P.nd[2] = 0;
    {
        const long S = 4L * P.n[0] * P.n[1] * P.n[2];
        double *s = vec(S), b[12] = {0}, J = 0.0;
        check(orc_forward(&P, NULL, s, b, NULL, &J), "orc_forward (body-free)");
        free(s);
    }
    if (fails) return 1;
    printf("oracle sanitizer run: all entry points returned 0\n");
    return 0;
}
