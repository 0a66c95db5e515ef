/*
 * lks_oracle.h -- plain serial FP64 CPU oracle for the lattice kinetic scheme (LKS)
 * with a passively moving rigid body and its exact discrete adjoint.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library. The GPU library shares no code with it.
 *
 * Paper: Tanabe, Yaji, Ushijima, "Topology optimization of passively moving rigid
 * bodies in unsteady flows", arXiv 2601.18272.
 *
 * Units are lattice units (grid spacing and time step equal to one, tau = 1).
 *
 * Memory layouts (all host memory, caller-owned):
 *   node index      n = x + nx*(y + ny*z)            (nz = 1 in 2D)
 *   state           [p | u_x | u_y (| u_z)]          (d+1)*N doubles
 *   design          gamma[i + ndx*(j + ndy*k)]       (ndz = 1 in 2D)
 *   body            12 doubles {xG[3], uG[3], theta, omega, unused[4]}
 *
 * Every function returns 0 on success and a negative value on a bad argument.
 */
#ifndef LKS_ORACLE_H
#define LKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_VELOCITY = 1, ORC_PRESSURE = 2, ORC_WALL = 3 };
enum { ORC_OBJ_DISP_X = 0, ORC_OBJ_DISP_Y = 1, ORC_OBJ_DISP_Z = 2, ORC_OBJ_ANGLE = 3 };
enum { ORC_DOF_TX = 1, ORC_DOF_TY = 2, ORC_DOF_TZ = 4, ORC_DOF_ROT = 8 };

typedef struct {
    int dim;              /* 2 (D2Q9) or 3 (D3Q15) */
    int n[3];             /* analysis grid; n[2] = 1 in 2D */
    int bc[6];            /* per face (x-, x+, y-, y+, z-, z+): ORC_* kind */
    double bc_p[6];       /* prescribed pressure of a PRESSURE face */
    double bc_u[6][3];    /* prescribed velocity of a VELOCITY face */
    double nu;            /* kinematic viscosity; A = (1/6 - nu) * 9/2 */
    int nd[3];            /* design grid; nd[2] = 1 in 2D; all zero = no body */
    double kappa_max, q;  /* Brinkman interpolation parameters */
    double mass, inertia; /* M and I about the rotation axis */
    int axis;             /* rotation axis (0, 1, 2); 2 in 2D */
    int dof_mask;         /* ORC_DOF_* bits of the free degrees of freedom */
    int n_itr;            /* fluid <-> body iterations per step */
    int n_steps;          /* time steps */
    int objective;        /* ORC_OBJ_* */
} orc_problem;

/* One coupled time step S(t-1) -> S(t). */
int orc_step(const orc_problem *P, const double *gamma, const double *s_in,
             const double *b_in, double *s_out, double *b_out);

/* n_steps coupled steps, in place on state and body. traj (optional) receives the
 * body state after every step, (n_steps+1)*12 doubles. J receives the objective
 * (displacement or rotation since the start). */
int orc_forward(const orc_problem *P, const double *gamma, double *state, double *body,
                double *traj, double *J);

/* Forward run plus the exact reverse-mode (discrete adjoint) sweep of
 *   L = seed * J + <dstate_T, state(n_steps)> + <dbody_T[0..7], body(n_steps)[0..7]>
 * (dstate_T, dbody_T optional, NULL = zero: the terminal adjoint values, which the
 * periodic problem approximation of Sec. 3.4 takes from the previous optimization
 * iteration). grad receives dL/dgamma (N_D doubles); dstate0 ((d+1)*N) and dbody0 (12)
 * optionally receive dL/d(initial state) and dL/d(initial body state). */
int orc_gradient(const orc_problem *P, const double *gamma, const double *state0,
                 const double *body0, double seed, const double *dstate_T, const double *dbody_T,
                 double *grad, double *J, double *dstate0, double *dbody0);

/* Design -> analysis-grid mapping of kappa_ref and of the rigid-body velocity at the
 * pose `body` (full-grid outputs; non-interior nodes are zero). */
/* The paper's adjoint variant (Sec. 2.5, App. A): the continuous adjoint discretised like
 * the forward, with N_itr fixed-point iterations of the body adjoint per time level and
 * the sensitivity of Eq. design_sensitivity. Not the exact derivative of the discrete
 * forward map (see lks_oracle.c). J: the objective of the forward run. */
int orc_gradient_paper(const orc_problem *P, const double *gamma, const double *state0,
                       const double *body0, double *grad, double *J);

int orc_map_design(const orc_problem *P, const double *kappa_ref, const double *body,
                   double *kappa, double *uS);

/* Analysis -> design interpolation u_ref (d*N_D, component-major) of a velocity field
 * u (d*N, component-major) at the pose `body`. */
int orc_interp(const orc_problem *P, const double *u, const double *body, double *uref);

/* Force F[3] and torque (FT[3]) from kappa_ref, u_ref and the pose `body`. */
int orc_force(const orc_problem *P, const double *kappa_ref, const double *uref,
              const double *body, double *FT);

/* Euler update of the body from the state at t-1 and a force/torque FT[4]. */
int orc_body_step(const orc_problem *P, const double *FT, const double *body_prev,
                  double *body_out);

/* Coupling constants K[4] (x, y, z translation and rotation): minus the slope of the
 * force (torque) with respect to the body velocity (angular velocity) for the first
 * step from `state`/`body`, fluid frozen. */
int orc_coupling(const orc_problem *P, const double *gamma, const double *state,
                 const double *body, double *K);

/* Brinkman interpolation kappa_ref(gamma). */
int orc_kappa_ref(const orc_problem *P, const double *gamma, double *kappa_ref);

/* Density filter with Heaviside projection (Sec. 3.2), on a design grid of dim axes
 * with nd[] points (spacing one):
 *   Eq. filter      gt_i = sum_j w_ij g_j / sum_j w_ij,  w_ij = (R - |x_i - x_j|) / R
 *                   for |x_i - x_j| <= R (else 0), j over the design grid;
 *   Eq. projection  gh_i = (tanh(beta eta) + tanh(beta (gt_i - eta)))
 *                          / (tanh(beta eta) + tanh(beta (1 - eta))).
 * orc_filter returns gt and gh; orc_filter_adjoint maps the cotangent gbh of gh to the
 * cotangent gb of g (the transpose of the projection's and the filter's Jacobians),
 * given gt. */
int orc_filter(int dim, const int nd[3], double R, double beta, double eta, const double *g, double *gt,
               double *gh);
int orc_filter_adjoint(int dim, const int nd[3], double R, double beta, double eta, const double *gt,
                       const double *gbh, double *gb);

/* Cyclic periodic design (Sec. 4.2): the design variables live on one of n_sec sectors
 * (n_sec = 1, 2, or 4 with a square rotation plane) and are repeated by the rotations
 * about the rotation axis through the design grid's centre. Sector size (or -1 if
 * n_sec is not supported for this grid); expansion sector -> design grid; collection
 * (its transpose) design-grid sensitivities -> sector. */
long orc_cyclic_sector_points(const orc_problem *P, int n_sec);
int orc_cyclic_expand(const orc_problem *P, int n_sec, const double *gs, double *g);
int orc_cyclic_collect(const orc_problem *P, int n_sec, const double *grad, double *gs);

#ifdef __cplusplus
}
#endif
#endif
