"""MMA design update -- TEST INFRASTRUCTURE (plain numpy, FP64).

The paper updates the design with the method of moving asymptotes (Sec. 3.5,
Algorithm 1: gamma^k, dJ/dgamma, G, dG/dgamma -> gamma^(k+1)), citing Svanberg (1987).
This is that method for one inequality constraint, restated from the published
method, step by step in the order it is usually presented:

  1. moving asymptotes L_j < x_j < U_j (initial spread, then widened where the
     iterates move monotonically and narrowed where they oscillate);
  2. move limits alpha_j <= x_j <= beta_j inside (L_j, U_j) and the box [xmin, xmax];
  3. the convex separable approximation of f_i (i = 0 objective, 1 constraint):
       f~_i(x) = r_i + sum_j p_ij / (U_j - x_j) + q_ij / (x_j - L_j),
     p_ij, q_ij from the positive and negative parts of df_i/dx_j (with a small
     regularisation), r_i so that f~_i(x^k) = f_i(x^k);
  4. the subproblem min f~_0 s.t. f~_1 <= 0 on [alpha, beta], solved through its
     dual: for lambda >= 0 the minimiser of f~_0 + lambda f~_1 is separable and in
     closed form, and the dual derivative h(lambda) = f~_1(x(lambda)) is
     non-increasing, so lambda* = 0 if h(0) <= 0, else the root of h, found here by
     plain bisection.

Only the tests, __graft_entry__.smoke() and bench.py's cpu_baseline may use it; the GPU
library shares no code with it.

Readings (where the paper states nothing): minimisation form (the paper maximises J,
so f_0 = -J); asymptote parameters 0.5 / 0.7 / 1.2 and bounds 0.01 / 10 times the box
width; move limit as a fraction of the box width; p, q with the factors 1.001 / 0.001
and the regularisation 1e-5 / (xmax - xmin); no artificial variables: if no lambda up to
LAM_MAX makes the approximated constraint feasible, x(LAM_MAX) is returned.
"""
from __future__ import annotations

import numpy as np

ASYINIT, ASYDECR, ASYINCR = 0.5, 0.7, 1.2
ALBEFA = 0.1      # move limit inside the asymptotes: alpha = L + ALBEFA (x - L)
RAA0 = 1e-5       # regularisation of p, q
LAM_MAX = 1e20


def asymptotes(x, xold1, xold2, low, upp, it, xmin, xmax):
    """Step 1 (it counts from 1)."""
    w = xmax - xmin
    if it <= 2:
        return x - ASYINIT * w, x + ASYINIT * w
    s = (x - xold1) * (xold1 - xold2)
    gam = np.where(s < 0, ASYDECR, np.where(s > 0, ASYINCR, 1.0))
    lo = x - gam * (xold1 - low)
    up = x + gam * (upp - xold1)
    lo = np.minimum(np.maximum(lo, x - 10.0 * w), x - 0.01 * w)
    up = np.maximum(np.minimum(up, x + 10.0 * w), x + 0.01 * w)
    return lo, up


def move_limits(x, lo, up, xmin, xmax, move):
    """Step 2."""
    w = xmax - xmin
    alpha = np.maximum(np.maximum(lo + ALBEFA * (x - lo), x - move * w), xmin)
    beta = np.minimum(np.minimum(up - ALBEFA * (up - x), x + move * w), xmax)
    return alpha, beta


def approximation(x, lo, up, df, xmin, xmax):
    """Step 3: p, q of one function from its gradient df."""
    w = xmax - xmin
    dp, dm = np.maximum(df, 0.0), np.maximum(-df, 0.0)
    p = (up - x) ** 2 * (1.001 * dp + 0.001 * dm + RAA0 / w)
    q = (x - lo) ** 2 * (0.001 * dp + 1.001 * dm + RAA0 / w)
    return p, q


def x_of_lambda(lam, p0, q0, p1, q1, lo, up, alpha, beta):
    """Minimiser of f~_0 + lam f~_1 over [alpha, beta], per variable."""
    P, Q = p0 + lam * p1, q0 + lam * q1
    sp, sq = np.sqrt(P), np.sqrt(Q)
    xs = (sp * lo + sq * up) / (sp + sq)
    return np.minimum(np.maximum(xs, alpha), beta)


def mma_step(x, xold1, xold2, low, upp, df0, g1, dg1, it, xmin=0.0, xmax=1.0, move=0.2, iters=400):
    """One MMA update. Returns (x_new, low, upp, lambda)."""
    x, df0, dg1 = (np.asarray(a, dtype=np.float64) for a in (x, df0, dg1))
    lo, up = asymptotes(x, np.asarray(xold1, float), np.asarray(xold2, float), np.asarray(low, float),
                        np.asarray(upp, float), it, xmin, xmax)
    alpha, beta = move_limits(x, lo, up, xmin, xmax, move)
    p0, q0 = approximation(x, lo, up, df0, xmin, xmax)
    p1, q1 = approximation(x, lo, up, dg1, xmin, xmax)
    r1 = float(g1) - np.sum(p1 / (up - x) + q1 / (x - lo))

    def h(lam):
        xl = x_of_lambda(lam, p0, q0, p1, q1, lo, up, alpha, beta)
        return r1 + np.sum(p1 / (up - xl) + q1 / (xl - lo))

    if h(0.0) <= 0.0:
        lam = 0.0
    else:
        hi = 1.0
        while h(hi) > 0.0 and hi < LAM_MAX:
            hi = min(2.0 * hi, LAM_MAX)
        lo_l = 0.0
        if h(hi) > 0.0:
            lam = hi  # LAM_MAX: the approximated constraint cannot be met
        else:
            for _ in range(iters):
                mid = 0.5 * (lo_l + hi)
                if mid <= lo_l or mid >= hi:
                    break
                if h(mid) > 0.0:
                    lo_l = mid
                else:
                    hi = mid
            lam = hi
    xn = x_of_lambda(lam, p0, q0, p1, q1, lo, up, alpha, beta)
    return xn, lo, up, lam


def volume_constraint(gh, vmin):
    """Eq. constraint read as a minimum-volume constraint (the text's intent):
    G = 1 - sum(gh) / (vmin n) <= 0. Returns (G, dG/dgh)."""
    gh = np.asarray(gh, dtype=np.float64)
    n = gh.size
    return 1.0 - gh.sum() / (vmin * n), np.full(n, -1.0 / (vmin * n))
