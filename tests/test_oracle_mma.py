"""Pins of the MMA oracle (oracle/mma.py): closed-form optima, brute force on the
subproblem, the dual condition and the asymptote rules."""
import numpy as np
import pytest

from oracle import mma


def test_converges_to_closed_form_optimum():
    """min sum c_j / x_j s.t. sum x_j <= V: x_j = V sqrt(c_j) / sum sqrt(c_k) when no
    bound is active (Lagrange condition c_j / x_j^2 = lambda)."""
    rng = np.random.default_rng(3)
    n = 40
    c = rng.uniform(0.5, 2.0, n)
    V = 0.3 * n
    xs = V * np.sqrt(c) / np.sqrt(c).sum()
    assert xs.max() < 1.0 and xs.min() > 0.05
    x = np.full(n, 0.25)
    xo1 = xo2 = x.copy()
    lo = up = np.zeros(n)
    for it in range(1, 120):
        df0 = -c / x ** 2
        g1 = x.sum() - V
        xn, lo, up, lam = mma.mma_step(x, xo1, xo2, lo, up, df0, g1, np.ones(n), it, 1e-3, 1.0, 0.2)
        xo2, xo1, x = xo1, x, xn
    assert np.abs(x - xs).max() < 1e-6
    assert abs(lam - (c / xs ** 2).mean()) < 1e-4 * lam


def test_subproblem_minimiser_by_brute_force():
    """x(lambda) minimises P/(U - x) + Q/(x - L) on [alpha, beta] (dense search)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        L, U = -rng.uniform(0.1, 1.0), 1.0 + rng.uniform(0.1, 1.0)
        a, b = sorted(rng.uniform(0.0, 1.0, 2))
        p0, q0, p1, q1 = rng.uniform(0.0, 2.0, 4)
        lam = rng.uniform(0.0, 3.0)
        x = mma.x_of_lambda(lam, np.array([p0]), np.array([q0]), np.array([p1]), np.array([q1]), np.array([L]),
                            np.array([U]), np.array([a]), np.array([b]))[0]
        grid = np.linspace(a, b, 200001)
        f = (p0 + lam * p1) / (U - grid) + (q0 + lam * q1) / (grid - L)
        assert abs(x - grid[np.argmin(f)]) <= 2 * (b - a) / 200000 + 1e-12


@pytest.mark.parametrize("g1", [-0.5, 0.05])
def test_dual_condition(g1):
    """lambda = 0 when the approximated constraint holds at lambda = 0, else the
    approximated constraint is active at the returned point."""
    rng = np.random.default_rng(7)
    n = 200
    x = rng.uniform(0.2, 0.8, n)
    df0 = rng.normal(size=n)
    dg1 = np.full(n, 1.0 / n)
    xn, lo, up, lam = mma.mma_step(x, x, x, np.zeros(n), np.zeros(n), df0, g1, dg1, 1, 0.0, 1.0, 0.2)
    alpha, beta = mma.move_limits(x, lo, up, 0.0, 1.0, 0.2)
    p1, q1 = mma.approximation(x, lo, up, dg1, 0.0, 1.0)
    r1 = g1 - np.sum(p1 / (up - x) + q1 / (x - lo))
    h = r1 + np.sum(p1 / (up - xn) + q1 / (xn - lo))
    assert np.all(xn >= alpha) and np.all(xn <= beta)
    if g1 < 0:
        assert lam == 0.0 and h <= 0.0
    else:
        assert lam > 0.0 and abs(h) < 1e-12


def test_asymptote_rules():
    x = np.array([0.5, 0.5, 0.5])
    xo1 = np.array([0.4, 0.6, 0.5])
    xo2 = np.array([0.3, 0.5, 0.2])  # monotone, oscillating, stalled
    low = np.array([0.1, 0.1, 0.1])
    upp = np.array([0.9, 0.9, 0.9])
    lo, up = mma.asymptotes(x, xo1, xo2, low, upp, 1, 0.0, 1.0)
    assert np.allclose(lo, 0.0) and np.allclose(up, 1.0)
    lo, up = mma.asymptotes(x, xo1, xo2, low, upp, 3, 0.0, 1.0)
    assert np.allclose(lo, [0.5 - 1.2 * 0.3, 0.5 - 0.7 * 0.5, 0.5 - 1.0 * 0.4])
    assert np.allclose(up, [0.5 + 1.2 * 0.5, 0.5 + 0.7 * 0.3, 0.5 + 1.0 * 0.4])


def test_volume_constraint_reading():
    gh = np.full(64, 0.3)
    G, dG = mma.volume_constraint(gh, 0.3)
    assert abs(G) < 1e-15 and np.allclose(dG, -1.0 / (0.3 * 64))
    assert mma.volume_constraint(np.full(64, 0.2), 0.3)[0] > 0  # too little solid: violated


def test_infeasible_step_takes_the_multiplier_cap():
    """No artificial variables: when no multiplier meets the approximated constraint within
    the move limits, the step uses lambda = LAM_MAX itself, and x(LAM_MAX) is the
    constraint's own minimiser on [alpha, beta]; here every variable moves to its upper
    move limit x + 0.2 (the constraint falls as x grows, dg1 = -1)."""
    n = 30
    x = np.full(n, 0.3)
    df0 = np.linspace(-1e-3, 1e-3, n)
    xn, lo, up, lam = mma.mma_step(x, x, x, np.zeros(n), np.zeros(n), df0, float(n), -np.ones(n), 1, 0.0, 1.0, 0.2)
    assert lam == mma.LAM_MAX == 1e20
    assert np.abs(xn - 0.5).max() <= 1e-12
