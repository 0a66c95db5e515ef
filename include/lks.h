/*
 * lks.h -- C ABI of the MI355X (gfx950) library for the lattice kinetic scheme with a
 * passively moving rigid body, and its discrete adjoint.
 *
 * Method: Tanabe, Yaji, Ushijima, "Topology optimization of passively moving rigid
 * bodies in unsteady flows", arXiv 2601.18272. Lattice units (grid spacing = time
 * step = 1, tau = 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors on the
 *    current device), owned by the caller. The library never allocates or frees
 *    device memory; scratch space comes from the caller through `work`.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Every call
 *    is enqueued on it; lks_forward and lks_adjoint additionally synchronise it once
 *    at the end to read the device error flag, unless LKS_FLAG_ASYNC is set.
 *  - Floating-point arrays marked "T" have the precision of lks_problem_t.precision
 *    (float for LKS_FP32, double for LKS_FP64). Body states, force/torque, the
 *    objective and gradients are always double.
 *  - Node index n = x + nx*(y + ny*z) (nz = 1 in 2D). A state is [p | u_x | u_y (| u_z)],
 *    (dim+1)*N elements. Design index m = i + ndx*(j + ndy*k), ndz = 1 in 2D; the design
 *    grid has spacing 1 and is centred on the rotation centre x^G.
 *  - A body state is 12 doubles {x^G[3], u^G[3], theta, omega, reserved[4]}.
 *  - Return codes: LKS_OK, or a negative LKS_E* code; lks_last_error() then holds a
 *    message (thread-local). No exception crosses the ABI.
 *  - Calls that share `work` or `ckpt` buffers must not overlap.
 */
#ifndef LKS_H
#define LKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds per face; macroscopic values are prescribed directly (Sec. 2.2) */
enum { LKS_PERIODIC = 0, LKS_VELOCITY = 1, LKS_PRESSURE = 2, LKS_WALL = 3 };
enum { LKS_FP32 = 0, LKS_FP64 = 1 };
/* objectives, Eqs. objective1 / objective2: displacement of x^G or rotation angle */
enum { LKS_OBJ_DISP_X = 0, LKS_OBJ_DISP_Y = 1, LKS_OBJ_DISP_Z = 2, LKS_OBJ_ANGLE = 3 };
/* free degrees of freedom of the body (Eqs. equation_of_motion_*) */
enum { LKS_DOF_TX = 1, LKS_DOF_TY = 2, LKS_DOF_TZ = 4, LKS_DOF_ROT = 8 };
/* LKS_FLAG_ASYNC: lks_forward / lks_adjoint return without synchronising the stream (the
 *   device error flag is then not read). LKS_FLAG_PROFILE: live kernel timing (below).
 * LKS_FLAG_STABILITY: lks_forward first computes the coupling constants of the fluid <->
 *   body iteration at t = 0 (lks_coupling) and returns LKS_EUNSTABLE, before any time
 *   step, when an active degree of freedom has K/M >= 1 or K_theta/I >= 1 (the
 *   iteration of Sec. 3.1 then does not contract).
 * LKS_FLAG_PAPER_ADJOINT: lks_adjoint computes the paper's own adjoint variant instead of
 *   the exact reverse of the discrete map (below); the flag must also be set in the
 *   lks_workspace_bytes(P, 1) query (the variant needs more scratch).
 * LKS_FLAG_MARCH2D: 2D problems use the column-march LKS and adjoint LKS kernels whatever
 *   the grid size (by default grids of at least 4M nodes march in the forward, of at least
 *   1M nodes in the adjoint, smaller ones use the tile kernels). The results agree to
 *   rounding; a forward and the adjoint that recomputes it should be given the same flag
 *   for the recompute to reproduce the forward bit for bit.
 * LKS_FLAG_PLANE3D: the 3D LKS and adjoint LKS kernels address the fields one plane at a
 *   time, the form they take by themselves for fields of 2^31 bytes and more (smaller
 *   fields are addressed whole). The arithmetic is the same, so are the results; the flag
 *   exists so that the large-field form can be tested on small grids. */
enum {
    LKS_FLAG_ASYNC = 1,
    LKS_FLAG_PROFILE = 2,
    LKS_FLAG_STABILITY = 4,
    LKS_FLAG_PAPER_ADJOINT = 8,
    LKS_FLAG_MARCH2D = 16,
    LKS_FLAG_PLANE3D = 32
};

enum {
    LKS_OK = 0,
    LKS_EINVAL = -1,    /* bad argument: dims, null pointer, n_itr < 1, ... */
    LKS_ENOSPACE = -2,  /* `work` or `ckpt` smaller than the size query returned */
    LKS_EUNSTABLE = -3, /* LKS_FLAG_STABILITY pre-check: the fluid <-> body iteration
                           does not contract (K/M >= 1 or K_theta/I >= 1) */
    LKS_EDIVERGED = -4, /* non-finite body state; a fluid state with a non-finite value
                           or a speed beyond the lattice sound speed 1/sqrt(3) (checked
                           at every checkpoint, every 256 steps without checkpoints, and
                           at the end); or the body moved more than the footprint margin
                           (2 nodes) within one step */
    LKS_EHIP = -5       /* HIP runtime error (text in lks_last_error) */
};

typedef struct lks_problem {
    int dim;              /* 2 (D2Q9) or 3 (D3Q15) */
    int n[3];             /* analysis grid; n[2] = 1 in 2D; >= 3 along every axis used */
    int bc[6];            /* faces x-, x+, y-, y+, z-, z+: LKS_PERIODIC | VELOCITY | PRESSURE | WALL;
                             PERIODIC must be set on both faces of an axis */
    double bc_p[6];       /* pressure prescribed on a PRESSURE face */
    double bc_u[6][3];    /* velocity prescribed on a VELOCITY face (WALL: u = 0) */
    double nu;            /* kinematic viscosity; A = 9/2 (1/6 - nu) (Sec. 2.2) */
    int nd[3];            /* design grid (nd[2] = 1 in 2D); all zero: no body */
    double kappa_max, q;  /* Eq. brinkman_coefficient */
    double mass, inertia; /* M and the moment of inertia about the rotation axis */
    int axis;             /* rotation axis 0/1/2 (ignored in 2D: z) */
    int dof_mask;         /* LKS_DOF_* bits */
    int n_itr;            /* fluid <-> body iterations per step (Sec. 3.1), >= 1 */
    int n_steps;          /* time steps N_t */
    int ckpt_every;       /* checkpoint interval K of the adjoint (>= 1 when ckpt is used) */
    int precision;        /* LKS_FP32 | LKS_FP64: fields, stencils, mapping */
    int objective;        /* LKS_OBJ_* */
    int flags;            /* LKS_FLAG_* */
} lks_problem_t;

/* Elements (not bytes) of one state: (dim+1)*N. */
size_t lks_state_elems(const lks_problem_t *P);

/* Bytes of the checkpoint store that lks_forward fills for lks_adjoint:
 * ceil(n_steps/ckpt_every) states plus their body states and a small header. */
size_t lks_checkpoint_bytes(const lks_problem_t *P);

/* Bytes of scratch space for lks_forward (adjoint = 0) or lks_adjoint (adjoint = 1).
 * The adjoint workspace holds one recomputed segment of ckpt_every states. */
size_t lks_workspace_bytes(const lks_problem_t *P, int adjoint);

/*
 * lks_forward -- n_steps coupled time steps (Algorithm 1, state loop): the LKS update
 * of p, u (Eqs. local_equilibrium_function, p_tmp, u_tmp), then n_itr iterations of
 * rigid body -> fluid (Eqs. rigid_body_position/velocity, kappa_mapping, us_mapping,
 * p, u) and fluid -> rigid body (Eq. u_mapping and the Euler update of Sec. 2.4), then
 * the boundary values.
 *   gamma   [ND] T, design variable in [0, 1] (read only)
 *   state   [(dim+1)*N] T, in: state at t = 0, out: state at t = n_steps
 *   body    [12] double, in: body at t = 0, out: body at t = n_steps
 *   ckpt    optional (NULL = no adjoint later): checkpoint store of ckpt_bytes
 *   work    scratch of lks_workspace_bytes(P, 0) bytes
 *   J       [1] double, out: objective (x^G component or theta at n_steps minus its
 *           initial value)
 * The state arrays passed in and out hold u itself; during the run (and in the
 * checkpoints) the velocity is held as its deviation from the velocity prescribed on
 * the first VELOCITY face (none: no shift), which keeps FP32 fields precise on the small
 * deviations that drive the body.
 * Errors: LKS_EINVAL, LKS_ENOSPACE, LKS_EUNSTABLE (with LKS_FLAG_STABILITY), LKS_EDIVERGED,
 * LKS_EHIP.
 */
int lks_forward(const lks_problem_t *P, const void *gamma, void *state, double *body,
                void *ckpt, size_t ckpt_bytes, void *work, size_t work_bytes, double *J,
                void *stream);

/*
 * lks_forward_noalloc -- lks_forward without checkpoints, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the scratch space lks_forward takes through `work` comes from
 * a static device array of LKS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on (until the process ends). The call allocates nothing: no hipMalloc, hipFree
 * or allocating library routine. The caller still passes the inputs and outputs, with
 * the meaning of lks_forward's (state in/out, body in/out, J out).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or host threads) race and must be serialised by the caller. Each call starts
 * from cleared counters and flags; nothing is carried between calls.
 * Errors: as lks_forward, plus LKS_ENOSPACE when the problem needs more than
 * LKS_NOALLOC_SCRATCH_BYTES of scratch (lks_workspace_bytes(P, 0)), and LKS_EINVAL with
 * LKS_FLAG_PROFILE (profiling creates events).
 */
#define LKS_NOALLOC_SCRATCH_BYTES (32u << 20)
int lks_forward_noalloc(const lks_problem_t *P, const void *gamma, void *state, double *body, double *J,
                        void *stream);

/*
 * lks_adjoint -- reverse-time sweep (Sec. 2.5, Algorithm 1, adjoint loop) giving the
 * design sensitivity (Eq. design_sensitivity) as the exact derivative of the discrete
 * map that lks_forward computes: segments of ckpt_every steps are recomputed from the
 * checkpoints and swept backwards through the LKS, the boundary values, the n_itr
 * body iterations, the mapping and the pose. The sweep differentiates
 *   L = seed * J + <dstate_T, state(n_steps)> + <dbody_T[0..7], body(n_steps)[0..7]>:
 * the terminal adjoint values dstate_T, dbody_T are where the periodic problem
 * approximation (Sec. 3.4) starts the adjoint of optimization iteration k+1 (from
 * dstate0, dbody0 of iteration k); they also chain runs split in time.
 *   gamma    [ND] T, the same design as in the lks_forward call that filled ckpt
 *   ckpt     checkpoint store filled by lks_forward (read only)
 *   work     scratch of lks_workspace_bytes(P, 1) bytes
 *   seed     dL/dJ
 *   dstate_T optional [(dim+1)*N] T (NULL = zero), read only; must not overlap work
 *   dbody_T  optional [12] double (NULL = zero; entries 8..11 are ignored), read only
 *   grad     [ND] double, out: dL/dgamma
 *   dstate0  optional [(dim+1)*N] T, out: dL/d(initial state)
 *   dbody0   optional [12] double, out: dL/d(initial body state)
 * With LKS_FLAG_PAPER_ADJOINT (problems with a design grid; dstate_T, dbody_T, dstate0,
 * dbody0 must be NULL) the sweep is instead the paper's adjoint variant (Sec. 2.5, App. A,
 * Algorithm 1's adjoint loop): the continuous adjoint discretised like the forward. Per
 * time level, backwards: the ALKS of Eqs. ap_tmp..as_tmp with the forward velocity of the
 * same level, then n_itr fixed-point iterations of Eq. au (the Brinkman factor applied to
 * the adjoint moment u~ with the body terms) and Eqs. axg, aug, atheta, aomega for the
 * body adjoints, and the sensitivity of Eq. design_sensitivity. The objective enters as
 * J = sum_t J_I with J_I = omega or u^G_a (Eqs. objective1/2), scaled by seed. It
 * approximates the derivative of the discrete map (the paper's "good agreement"); grad
 * is then that approximation.
 * Errors: LKS_EINVAL, LKS_ENOSPACE, LKS_EHIP.
 */
int lks_adjoint(const lks_problem_t *P, const void *gamma, const void *ckpt, size_t ckpt_bytes,
                void *work, size_t work_bytes, double seed, const void *dstate_T, const double *dbody_T,
                double *grad, void *dstate0, double *dbody0, void *stream);

/*
 * map_design -- grid separation, Eqs. kappa_mapping, us_mapping with the weight of
 * Eq. weight_function: the design-grid Brinkman coefficient and the rigid-body velocity
 * of every design point (Eq. rigid_body_velocity) at pose `body`, mapped onto the
 * interior analysis nodes.
 *   kappa_ref [ND] T (read only)
 *   body      [12] double (read only)
 *   kappa     [N] T, out (zero where no design point reaches)
 *   uS        [dim*N] T, out, component-major
 * Errors: LKS_EINVAL, LKS_EHIP.
 */
int map_design(const lks_problem_t *P, const void *kappa_ref, const double *body, void *kappa,
               void *uS, void *stream);

/*
 * body_step -- explicit Euler update of Sec. 2.4 with the DOF mask:
 *   u^G = u^G_prev + F/M, x^G = x^G_prev + u^G, omega = omega_prev + T/I,
 *   theta = theta_prev + omega; an inactive DOF keeps its previous values.
 *   ft        [4] double {F_x, F_y, F_z, T} (read only)
 *   body_prev [12] double (read only)
 *   body      [12] double, out (may alias nothing)
 * Errors: LKS_EINVAL, LKS_EHIP.
 */
int body_step(const lks_problem_t *P, const double *ft, const double *body_prev, double *body,
              void *stream);

/*
 * lks_coupling -- coupling constants of the fluid <-> body iteration of Sec. 3.1 at the
 * pose `body`: within a time step the iterates satisfy u^G,(k+1) = u^G(t-1) +
 * F(u^G,(k))/M with F affine in the body velocity at a frozen pose and u*, so the
 * iteration contracts when K/M < 1 (and K_theta/I < 1), where
 *   K[a] = -dF_a/du^G_a = sum_m kappa_ref_m - sum_x kappa^2 phi / (1 + kappa)   (a < dim)
 *   K[3] = -dT/domega   = sum_m kappa_ref_m |a x r_m|^2 - sum_x kappa/(1 + kappa) S . S_k
 * with the mapped kappa (Eq. kappa_mapping), phi = sum_m W, S = sum_m W (a x r_m),
 * S_k = sum_m W kappa_ref_m (a x r_m), r_m = x^ref_m - x^G (Eq. rigid_body_position),
 * sums over interior nodes and design points, FP64. Independent of the fluid state.
 *   gamma  [ND] T (read only)
 *   body   [12] double (read only): the pose (x^G, theta)
 *   K      [4] double, out (device); K[a] = 0 for a >= dim
 *   work   scratch of lks_workspace_bytes(P, 0) bytes
 * Synchronises the stream once at the start (to size the footprint box from theta), then
 * enqueues its kernels without synchronising.
 * Errors: LKS_EINVAL (no design grid, null pointer, non-finite body), LKS_ENOSPACE, LKS_EHIP.
 */
int lks_coupling(const lks_problem_t *P, const void *gamma, const double *body, double *K, void *work,
                 size_t work_bytes, void *stream);

/* Density filter and Heaviside projection of the design field (Sec. 3.2). */
typedef struct lks_filter {
    double radius; /* R of Eq. filter in design-grid spacings: R > 0, floor(R) <= 8 in 2D, <= 4 in 3D */
    double beta;   /* steepness of Eq. projection, > 0 */
    double eta;    /* threshold of Eq. projection, in [0, 1] */
} lks_filter_t;

/*
 * lks_design_filter -- Eq. filter, then Eq. projection, on the design grid of P (only
 * P->dim, P->nd and P->precision are used; P must be valid and have a design grid):
 *   gamma_tilde_i = sum_j w_ij gamma_j / sum_j w_ij, w_ij = (R - |x_i - x_j|) / R for
 *                   design points within distance R (the cone is cut at the grid's edge);
 *   gamma_hat_i   = (tanh(beta eta) + tanh(beta (gamma_tilde_i - eta)))
 *                   / (tanh(beta eta) + tanh(beta (1 - eta))).
 * gamma_hat is what lks_forward and lks_adjoint take as their design.
 *   gamma       [ND] T (read only)
 *   gamma_tilde [ND] T, out
 *   gamma_hat   [ND] T, out
 * The three arrays must not overlap. Enqueued on `stream` without synchronising, unless
 * P->flags has LKS_FLAG_PROFILE: then the call synchronises the stream and adds the
 * kernel's duration to LKS_K_FILTER.
 * Errors: LKS_EINVAL, LKS_EHIP.
 */
int lks_design_filter(const lks_problem_t *P, const lks_filter_t *F, const void *gamma, void *gamma_tilde,
                      void *gamma_hat, void *stream);

/* Bytes of scratch space for lks_design_filter_adjoint: ND doubles (0 without a design grid). */
size_t lks_filter_workspace_bytes(const lks_problem_t *P);

/*
 * lks_design_filter_adjoint -- reverse of lks_design_filter, in FP64: a sensitivity with
 * respect to gamma_hat is taken through the derivative of Eq. projection at gamma_tilde
 * and the transpose of Eq. filter:
 *   t_i         = dJ_dgamma_hat_i (d gamma_hat / d gamma_tilde)_i / sum_k w_ik   (into work)
 *   dJ_dgamma_j = sum_i w_ij t_i
 *   gamma_tilde   [ND] T, the filtered field of the forward call (read only)
 *   dJ_dgamma_hat [ND] double (read only), e.g. the grad of lks_adjoint
 *   work          scratch of lks_filter_workspace_bytes(P) bytes
 *   dJ_dgamma     [ND] double, out
 * The four arrays must not overlap. Stream and LKS_FLAG_PROFILE (kernel
 * LKS_K_FILTER_ADJ, both launches) as for lks_design_filter.
 * Errors: LKS_EINVAL, LKS_ENOSPACE, LKS_EHIP.
 */
int lks_design_filter_adjoint(const lks_problem_t *P, const lks_filter_t *F, const void *gamma_tilde,
                              const double *dJ_dgamma_hat, void *work, size_t work_bytes, double *dJ_dgamma,
                              void *stream);

/*
 * Cyclic periodic design (Sec. 4.2): the design variables live on one of n_sectors
 * sectors of the design grid of P and are repeated by the rotations by 2 pi k / n_sectors
 * about P's rotation axis (2D: z) through the design grid's centre. Supported: n_sectors
 * = 1, 2 (half turn), 4 (quarter turn; the rotation plane must be square). In plane
 * coordinates (u, v) along the plane's axes (axis+1, axis+2 mod 3) and w along the axis,
 * the sector is: n = 2: plane indices q = u + nu v with q <= nu nv - 1 - q (index q);
 * n = 4 (side s): u < ceil(s/2), v < floor(s/2) (index u + ceil(s/2) v), then for odd s
 * the centre. Sector index = plane sector index + (points of the plane sector) * w.
 * lks_cyclic_sector_points returns the sector size (0 if unsupported or no design grid).
 */
size_t lks_cyclic_sector_points(const lks_problem_t *P, int n_sectors);

/*
 * lks_design_cyclic_expand -- gamma[m] = gamma_sector[sector index of m's orbit].
 *   gamma_sector [lks_cyclic_sector_points] T (read only)
 *   gamma        [ND] T, out; must not overlap gamma_sector
 * Enqueued on `stream` (LKS_FLAG_PROFILE: synchronises it and records LKS_K_CYC_EXPAND).
 * Errors: LKS_EINVAL, LKS_EHIP.
 */
int lks_design_cyclic_expand(const lks_problem_t *P, int n_sectors, const void *gamma_sector, void *gamma,
                             void *stream);

/*
 * lks_design_cyclic_collect -- transpose of the expansion (FP64): every sector point
 * receives the sum of the sensitivities over its orbit (group order R^0, R^1, ...).
 *   grad        [ND] double (read only), e.g. the grad of lks_adjoint
 *   grad_sector [lks_cyclic_sector_points] double, out; must not overlap grad
 * Enqueued on `stream` (LKS_FLAG_PROFILE: synchronises it and records LKS_K_CYC_COLLECT).
 * Errors: LKS_EINVAL, LKS_EHIP.
 */
int lks_design_cyclic_collect(const lks_problem_t *P, int n_sectors, const double *grad, double *grad_sector,
                              void *stream);

/* ---------------------------------------------------------------- design update (MMA)
 * One step of the method of moving asymptotes for one inequality constraint, the
 * update of Sec. 3.5 / Algorithm 1 (gamma^k, dJ/dgamma, G, dG/dgamma -> gamma^(k+1);
 * the paper cites Svanberg 1987). Minimisation form: the objective's gradient is
 * opt->f0_scale * df0, so df0 = dJ/dgamma with f0_scale = -1 / |J_ref| maximises J scaled
 * to order one.
 * All arrays are device FP64 of n entries; the caller keeps the history:
 *   x     [n] in: x^k, out: x^(k+1)
 *   xold1, xold2 [n] x^(k-1), x^(k-2) (read when iter > 2; may be NULL otherwise)
 *   low, upp [n] in: the previous asymptotes (read when iter > 2), out: this step's
 *   df0, dg1 [n] gradients of the objective and of the constraint at x^k
 *   g1    [1] device: the constraint value at x^k (feasible when <= 0)
 *   lambda [1] device, may be NULL: the multiplier of the constraint
 * iter counts from 1. Asymptotes start at x -+ 0.5 (xmax - xmin), then widen by 1.2 /
 * narrow by 0.7 where the iterates move monotonically / oscillate, within 0.01 .. 10 box
 * widths; move limits are opt->move box widths and 10 % of the way to the asymptotes. The
 * dual is solved by multi-section to double precision; if no multiplier up to 1e20 makes
 * the approximated constraint hold, the step uses 1e20. Deterministic (fixed-order sums).
 * work: at least lks_mma_workspace_bytes(n) bytes of device scratch, caller-owned.
 * Errors: LKS_EINVAL for n < 1, iter < 1, xmin >= xmax, move <= 0, a non-finite f0_scale,
 * null arrays, outputs that overlap inputs, each other or the workspace, a workspace
 * smaller than lks_mma_workspace_bytes(n); LKS_EHIP for a failed launch. Asynchronous on
 * `stream` (no synchronisation). */
typedef struct {
    double xmin, xmax; /* box of the design variables (0, 1 for gamma) */
    double move;       /* move limit, fraction of xmax - xmin */
    double f0_scale;   /* factor on df0 (1 to minimise the given function) */
} lks_mma_t;

/* Device scratch bytes for lks_mma_update / lks_volume_constraint on n variables (0 and
 * LKS_EINVAL for n < 1). */
size_t lks_mma_workspace_bytes(long long n);
int lks_mma_update(const lks_mma_t *opt, long long n, int iter, double *x, const double *xold1,
                   const double *xold2, double *low, double *upp, const double *df0, const double *g1,
                   const double *dg1, double *lambda, void *work, size_t work_bytes, void *stream);

/* Volume constraint of Eq. constraint, read as a lower bound on the solid volume (the
 * paper's text; the printed inequality has the opposite sense):
 * G = 1 - sum(gh) / (vmin n) <= 0 and dG/dgh_j = -1 / (vmin n), from the projected design gh
 * [n] (device FP64). G [1] and dG [n] (may be NULL) are device outputs. work: at least
 * lks_mma_workspace_bytes(n) bytes. Errors: LKS_EINVAL for n < 1, vmin not positive and
 * finite, null arrays, overlaps among the arguments and the workspace, a short workspace;
 * LKS_EHIP for a failed launch. Asynchronous on `stream`. */
int lks_volume_constraint(long long n, const double *gh, double vmin, double *G, double *dG, void *work,
                          size_t work_bytes, void *stream);

/* Message of the last error on this thread ("" if none). */
const char *lks_last_error(void);

/*
 * Live kernel timing. A call made with LKS_FLAG_PROFILE times the kernels of a sample
 * of its time steps (at most 32 sampled steps per call, every kernel of a sampled step)
 * and, after its final synchronisation, adds the durations to process-wide totals. The
 * durations come from HIP events attached to the launch (hipExtLaunchKernelGGL:
 * dispatch to completion, as a profiler counts a launch). In 2D, the LKS and adjoint
 * LKS kernels also stamp their own span on the device wall clock (first blocks' start
 * to last blocks' end, into the workspace) on every other sampled launch, read as
 * LKS_K_GATHER_SPAN and LKS_K_ADJ_GATHER_SPAN. A unit that is two launches (a reduction plus its
 * one-block finish) is timed from the first kernel's begin to the second's end. Not
 * thread-safe.
 *   kernel   LKS_K_* id
 *   total_ms sum of the sampled launch durations (ms); samples: their number
 * Returns LKS_OK or LKS_EINVAL for an unknown id.
 */
enum {
    LKS_K_GATHER = 0,      /* LKS update of p, u on the grid */
    LKS_K_BC = 1,          /* boundary values */
    LKS_K_SPREAD = 2,      /* mapping design -> grid + Brinkman correction */
    LKS_K_INTERP = 3,      /* grid -> design interpolation, force/torque, body update */
    LKS_K_ADJ_GATHER = 4,  /* adjoint LKS update (with the boundary transpose) */
    LKS_K_ADJ_RECOMPUTE = 5,
    LKS_K_ADJ_R1 = 6,
    LKS_K_ADJ_R2 = 7,
    LKS_K_ADJ_R3 = 8,
    LKS_K_ITER = 9,        /* 2D: one fused iteration (partials -> B^(k), tile spread, interp) */
    LKS_K_ITER_FINAL = 10, /* 2D: B^(K) and the step's spread into the state */
    LKS_K_GATHER_SPAN = 11,     /* LKS_K_GATHER, the kernel's own span (no dispatch) */
    LKS_K_ADJ_GATHER_SPAN = 12, /* LKS_K_ADJ_GATHER, the kernel's own span */
    LKS_K_FILTER = 13,          /* lks_design_filter */
    LKS_K_FILTER_ADJ = 14,      /* lks_design_filter_adjoint (its two launches) */
    LKS_K_CYC_EXPAND = 15,      /* lks_design_cyclic_expand */
    LKS_K_CYC_COLLECT = 16,     /* lks_design_cyclic_collect */
    LKS_K_COUNT = 17
};
int lks_profile_read(int kernel, double *total_ms, long long *samples);
void lks_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif
