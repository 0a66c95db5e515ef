"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks. None of them re-types the oracle's formulas:
they use closed forms, invariants, special cases and finite differences, chosen so
that a dropped term, a wrong sign or index, or a transposed operand fails one.
"""
import math

import numpy as np
import pytest

import workloads as W

SQ2 = math.sqrt(2.0)
# Eq. weight_function (cosine reading): w(0) = 1/2, w(+-1) = 1/4, w(+-2) = 0,
# w(+-1/2) = (2 + sqrt 2)/8, w(+-3/2) = (2 - sqrt 2)/8.
W0, W1 = 0.5, 0.25
WH, W3H = (2 + SQ2) / 8, (2 - SQ2) / 8


def periodic(dim, n, **kw):
    n3 = tuple(n) + (1,) * (3 - len(n))
    return W.Problem(dim=dim, n=n3, bc=(W.PERIODIC,) * 6, **kw)


def coords(pb):
    N = pb.N
    i = np.arange(N)
    return i % pb.n[0], (i // pb.n[0]) % pb.n[1], i // (pb.n[0] * pb.n[1])


# ---------------------------------------------------------------- Sec. 2.2 LKS

@pytest.mark.parametrize("case", ["p2", "p3", "ch2", "ch3"])
def test_uniform_flow_is_fixed_point(orc, case):
    """A uniform flow (p = 0, u = U) is steady under Eqs. local_equilibrium_function,
    p_tmp, u_tmp; this fails for the '+3/2 u^2' sign as printed and for any weight
    error (the moment identities of the D2Q9/D3Q15 weights)."""
    U = (0.05, -0.02, 0.03)
    if case == "p2":
        pb = periodic(2, (10, 8), nu=0.12, n_steps=5)
    elif case == "p3":
        pb = periodic(3, (8, 7, 6), nu=0.05, n_steps=5)
    elif case == "ch2":
        pb = W.channel2d(14, 9, U[0], 0.1, n_steps=5)
    else:
        pb = W.Problem(dim=3, n=(10, 6, 5), bc=(W.VELOCITY, W.PRESSURE, 0, 0, 0, 0),
                       bc_u=((U[0], U[1], U[2]),) + ((0, 0, 0),) * 5, nu=0.08, n_steps=5)
    pb = pb.replace(u0=U[: pb.dim] + (0.0,) * (3 - pb.dim)) if case != "ch2" else pb
    s0 = W.initial_state(pb)
    s, _, _ = orc.forward(pb, None, s0, np.zeros(12))
    assert np.abs(s - s0).max() < 1e-16


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", [1, 3, 7])
def test_shear_wave_decay_closed_form(orc, dim, mode):
    """Linear shear wave u_y = a sin(kx): one step multiplies it by
    G(k) = 2/3 + cos(k)/3 + (2A/9) sin^2(k) with nu = (1/6 - 2A/9) (Sec. 2.2), which
    tends to 1 - nu k^2 for small k. Pins the A-term and its factor."""
    nx, nu, a0 = 32, 0.09, 1e-7
    pb = periodic(dim, (nx, 4) if dim == 2 else (nx, 4, 3), nu=nu, n_steps=1)
    N = pb.N
    x, _, _ = coords(pb)
    k = 2 * np.pi * mode / nx
    s0 = np.zeros((dim + 1) * N)
    s0[2 * N:3 * N] = a0 * np.sin(k * x)
    s1, _, _ = orc.forward(pb, None, s0, np.zeros(12))
    A = (1 / 6 - nu) * 9 / 2
    G = 2 / 3 + np.cos(k) / 3 + (2 * A / 9) * np.sin(k) ** 2
    assert np.abs(s1[2 * N:3 * N] - G * s0[2 * N:3 * N]).max() < 1e-14 * a0
    assert np.abs(s1[:N]).max() < 1e-18 and np.abs(s1[N:2 * N]).max() < 1e-18
    # small-k limit of G is the viscous decay 1 - nu k^2
    kk = 1e-3
    Gs = 2 / 3 + np.cos(kk) / 3 + (2 * A / 9) * np.sin(kk) ** 2
    assert abs((1 - Gs) / kk ** 2 - nu) < 1e-6


def test_pressure_sum_conserved_with_body(orc):
    """On a fully periodic grid sum_x p is invariant: p = p* (Eq. p) and the
    equilibrium moments give sum_i f_i = 3p + (2A/3) div u, whose divergence sums
    to zero. Holds with the body, since the Brinkman term only changes u."""
    pb = periodic(2, (30, 28), nu=0.12, nd=(8, 7, 1), kappa_max=0.8, q=0.1, mass=40.0,
                  inertia=3e3, dof_mask=W.DOF_TX | W.DOF_TY | W.DOF_ROT, n_itr=4, n_steps=30,
                  x_g0=(13.2, 14.7, 0), theta0=0.4, seed=3, u0=(0.03, -0.01, 0))
    s0 = W.initial_state(pb)
    s0[:pb.N] = 1e-3 * np.random.default_rng(0).standard_normal(pb.N)
    s, b, _ = orc.forward(pb, W.design(pb), s0, W.initial_body(pb))
    assert abs(s[:pb.N].sum() - s0[:pb.N].sum()) < 1e-15
    assert np.abs(b[:2] - pb.x_g0[:2]).max() > 1e-3  # the body did move


@pytest.mark.parametrize("dim", [2, 3])
def test_momentum_conserved_body_free(orc, dim):
    """Body-free periodic grid: sum_x u is invariant (first moments of the weights)."""
    pb = periodic(dim, (12, 10) if dim == 2 else (9, 8, 7), nu=0.07, n_steps=20)
    rng = np.random.default_rng(1)
    s0 = 1e-2 * rng.standard_normal((dim + 1) * pb.N)
    s, _, _ = orc.forward(pb, None, s0, np.zeros(12))
    for a in range(dim + 1):
        sl = slice(a * pb.N, (a + 1) * pb.N)
        assert abs(s[sl].sum() - s0[sl].sum()) < 1e-14


def poiseuille(dim, nu=0.1, dp=1e-3):
    n = (24, 11, 1) if dim == 2 else (12, 9, 4)
    pb = W.Problem(dim=dim, n=n, bc=(W.PRESSURE, W.PRESSURE, W.WALL, W.WALL, 0, 0),
                   bc_p=(dp, 0, 0, 0, 0, 0), nu=nu, n_steps=1)
    x, y, _ = coords(pb)
    H, G = n[1] - 1, dp / (n[0] - 1)
    s = np.zeros((dim + 1) * pb.N)
    s[:pb.N] = dp - G * x
    s[pb.N:2 * pb.N] = G / (2 * nu) * y * (H - y)
    return pb, s


@pytest.mark.parametrize("dim", [2, 3])
def test_poiseuille_exact_fixed_point(orc, dim):
    """Pressure-driven flow between walls: u_x = (G / 2 nu) y (H - y), p linear, is an
    exact fixed point of the scheme with the boundary treatment (prescribed p on the
    PRESSURE faces, u = 0 on WALL faces, the rest copied from the nearest interior
    node) and one-sided gradients on boundary nodes."""
    pb, s0 = poiseuille(dim)
    s1, _, _ = orc.forward(pb, None, s0, np.zeros(12))
    assert np.abs(s1 - s0).max() < 1e-17


def test_poiseuille_develops_from_rest(orc):
    pb, sref = poiseuille(2)
    s, _, _ = orc.forward(pb.replace(n_steps=6000), None, np.zeros_like(sref), np.zeros(12))
    N = pb.N
    assert np.abs(s[N:2 * N] - sref[N:2 * N]).max() < 1e-10 * sref[N:2 * N].max()


# ------------------------------------------------------------- Sec. 2.3 mapping

def one_point(dim, X, n=(12, 12, 12)):
    n3 = n if dim == 3 else (n[0], n[1], 1)
    pb = periodic(dim, n3[:dim], nd=(1, 1, 1), kappa_max=1.0, q=0.1, mass=1, inertia=1)
    b = np.zeros(12)
    b[:dim] = X
    return pb, b


def test_mapping_node_aligned_weights(orc):
    """A design point on a node spreads with W = w(rx) w(ry): 1/4 on the node, 1/8 on
    the 4 edge neighbours, 1/16 on the 4 diagonal ones, nothing further (Eq.
    weight_function). Fails for the printed '1 - cos' kernel."""
    pb, b = one_point(2, (5.0, 6.0))
    kap, uS = orc.map_design(pb, np.array([1.0]), b)
    k = kap.reshape(12, 12)
    assert k[6, 5] == pytest.approx(W0 * W0, abs=1e-16)
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        assert k[6 + dy, 5 + dx] == pytest.approx(W0 * W1, abs=1e-16)
    for dx, dy in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        assert k[6 + dy, 5 + dx] == pytest.approx(W1 * W1, abs=1e-16)
    assert abs(k.sum() - 1.0) < 1e-15
    assert np.count_nonzero(np.abs(k) > 1e-30) == 9


def test_mapping_half_offset_weights(orc):
    """Point at half offsets in 3D: W is the product of the 1D taps
    ((2-sqrt2)/8, (2+sqrt2)/8, (2+sqrt2)/8, (2-sqrt2)/8) on each axis."""
    pb, b = one_point(3, (5.5, 4.5, 6.5))
    kap, _ = orc.map_design(pb, np.array([2.0]), b)
    k = kap.reshape(12, 12, 12)
    taps = np.array([W3H, WH, WH, W3H])
    expect = 2.0 * np.einsum("i,j,k->ijk", taps, taps, taps)  # (z, y, x)
    got = k[5:9, 3:7, 4:8]
    assert np.abs(got - expect).max() < 1e-15
    assert abs(k.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_partition_of_unity_and_transpose(orc, dim):
    """sum_x W(x - X) = 1 for any X whose taps lie inside, so sum_x kappa = sum_m
    kappa_ref; and the spread (Eqs. kappa_mapping, us_mapping) is the transpose of the
    interpolation (Eq. u_mapping): <S a, b> = <a, I b>."""
    if dim == 2:
        pb = periodic(2, (30, 26), nd=(7, 6, 1), seed=4, kappa_max=1.0, q=0.1, mass=1, inertia=1)
    else:
        pb = periodic(3, (18, 17, 16), nd=(4, 5, 3), seed=4, kappa_max=1.0, q=0.1, mass=1,
                      inertia=1, axis=1)
    rng = np.random.default_rng(7)
    b = np.zeros(12)
    b[:dim] = np.array(pb.n[:dim]) / 2 + rng.random(dim)
    b[6] = 0.7
    a = rng.random(pb.ND)
    kap, _ = orc.map_design(pb, a, b)
    assert abs(kap.sum() - a.sum()) < 1e-12
    f = rng.standard_normal(dim * pb.N)
    uref = orc.interp(pb, f, b)
    lhs = float(kap @ f[:pb.N])
    rhs = float(a @ uref[:pb.ND])
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_rigid_body_kinematics_quarter_turn(orc):
    """Eqs. rigid_body_position / rigid_body_velocity at theta = pi/2: the point at
    xi = (1, 0) sits at x^G + (0, 1) and moves with u^G + omega (-1, 0)
    (counter-clockwise positive). Read back through the mapping at node x^G + (0,1)."""
    pb = periodic(2, (16, 16), nd=(3, 1, 1), kappa_max=1, q=0.1, mass=1, inertia=1)
    b = np.zeros(12)
    b[0:2] = (8.0, 8.0)
    b[3:5] = (0.01, -0.02)
    b[6] = math.pi / 2
    b[7] = 0.3
    kref = np.array([0.7, 1.3, 2.9])  # xi = (-1,0), (0,0), (1,0)
    kap, uS = orc.map_design(pb, kref, b)
    node = 9 * 16 + 8
    assert kap[node] == pytest.approx(W0 * W0 * 2.9 + W0 * W1 * 1.3, abs=1e-14)
    ux = W0 * W0 * (0.01 - 0.3) + W0 * W1 * 0.01
    uy = W0 * W0 * (-0.02) + W0 * W1 * (-0.02)
    assert uS[node] == pytest.approx(ux, abs=1e-14)
    assert uS[256 + node] == pytest.approx(uy, abs=1e-14)
    # the point xi = (-1, 0) is at x^G - (0, 1): node (8, 7) sees it with weight 1/4
    node2 = 7 * 16 + 8
    assert kap[node2] == pytest.approx(W0 * W0 * 0.7 + W0 * W1 * 1.3, abs=1e-14)


# ------------------------------------------------------------ Sec. 2.4 body

def test_body_step_constant_force(orc):
    """Explicit Euler of Sec. 2.4 under a constant force: u^G(t) = u^G(0) + t F/M,
    x^G(t) = x^G(0) + t u^G(0) + (F/M) t(t+1)/2; inactive DOFs keep their values."""
    pb = W.Problem(dim=3, n=(4, 4, 4), bc=(0,) * 6, nd=(1, 1, 1), mass=3.0, inertia=7.0,
                   dof_mask=W.DOF_TX | W.DOF_TZ | W.DOF_ROT, axis=1)
    FT = np.array([0.3, 0.5, -0.2, 0.11])
    b0 = np.array([1.0, 2.0, 3.0, 0.01, 0.02, 0.03, 0.4, 0.05, 0, 0, 0, 0])
    b = b0.copy()
    T = 17
    for _ in range(T):
        b = orc.body_step(pb, FT, b)
    aF = FT[:3] / 3.0
    for a, active in ((0, True), (1, False), (2, True)):
        if active:
            assert b[3 + a] == pytest.approx(b0[3 + a] + T * aF[a], rel=1e-14)
            assert b[a] == pytest.approx(b0[a] + T * b0[3 + a] + aF[a] * T * (T + 1) / 2, rel=1e-14)
        else:
            assert b[a] == b0[a] and b[3 + a] == b0[3 + a]
    al = 0.11 / 7.0
    assert b[7] == pytest.approx(0.05 + T * al, rel=1e-14)
    assert b[6] == pytest.approx(0.4 + T * 0.05 + al * T * (T + 1) / 2, rel=1e-14)


# ----------------------------------------- coupled closed forms (Eqs. u, Alg. 1)

def covering(n_itr, dofs, mass=60.0, kmax=0.5, gam=0.5):
    """Periodic 12x10 grid fully covered by a 22x20 design extending >= 3 nodes beyond
    it: kappa(x) = kappa_ref and the mapped body velocity equal the body's everywhere,
    and sum_m u^ref_m = N u for a uniform u (node-side partition of unity)."""
    pb = periodic(2, (12, 10), nu=0.1, nd=(22, 20, 1), kappa_max=kmax, q=0.1, mass=mass,
                  inertia=1e3, dof_mask=dofs, n_itr=n_itr, n_steps=6,
                  x_g0=(5.5, 4.5, 0.0), u0=(0.04, 0.01, 0.0))
    kr = kmax * 0.1 * gam / (1 - gam + 0.1)
    return pb, np.full(pb.ND, gam), kr


def test_brinkman_relaxation_closed_form(orc):
    """Held body moving with u^G under a uniform flow: with kappa and u^S uniform, Eq. u
    gives u(t) - u^G = (u(t-1) - u^G)/(1 + kappa) and p stays 0."""
    pb, g, kr = covering(2, 0)
    b0 = W.initial_body(pb)
    b0[3:5] = (-0.02, 0.03)
    s, b, _ = orc.forward(pb, g, W.initial_state(pb), b0)
    N = pb.N
    for a, (u0, ug) in enumerate(zip((0.04, 0.01), (-0.02, 0.03))):
        expect = ug + (u0 - ug) / (1 + kr) ** pb.n_steps
        assert np.abs(s[(1 + a) * N:(2 + a) * N] - expect).max() < 1e-16
    assert np.abs(s[:N]).max() < 1e-17
    assert np.array_equal(b, b0)


def test_coupled_iteration_closed_form(orc):
    """Free translation in the covering setting: F = kappa_ref (N u^(k) - N_D u^G,(k)),
    u^(k) = (u* + kappa_ref u^G,(k))/(1 + kappa_ref), each of the N_itr iterations
    restarting the Euler update from t-1 (Sec. 3.1, Alg. 1) and u(t) = u^(N_itr-1)."""
    pb, g, kr = covering(3, W.DOF_TX | W.DOF_TY)
    s, b, _ = orc.forward(pb, g, W.initial_state(pb), W.initial_body(pb))
    N, ND, M = pb.N, pb.ND, pb.mass
    u = np.array([0.04, 0.01])
    uG = np.zeros(2)
    xG = np.array([5.5, 4.5])
    for _ in range(pb.n_steps):
        uGk = uG.copy()
        for _k in range(pb.n_itr):
            uk = (u + kr * uGk) / (1 + kr)
            F = kr * (N * uk - ND * uGk)
            uG_new = uG + F / M
            xG_new = xG + uG_new
            uGk = uG_new
        u, uG, xG = uk, uG_new, xG_new
    assert np.abs(b[3:5] - uG).max() < 1e-15
    assert np.abs(b[0:2] - xG).max() < 1e-13
    for a in range(2):
        assert np.abs(s[(1 + a) * N:(2 + a) * N] - u[a]).max() < 1e-16


def test_force_and_torque_single_point(orc):
    """One porous design point one node above the centre in a uniform flow U along x:
    F_x = kappa U sum_x W/(1 + kappa W) over its 3x3 footprint (weights 1/4, 1/8, 1/16),
    F_y = 0 and the torque about z is T = e_zab r_a F_b = -F_x (lever arm +1 in y).
    One iteration per step so u^G(1) = F/M and omega(1) = T/I exactly."""
    gam = 0.6
    pb = periodic(2, (16, 16), nu=0.1, nd=(1, 3, 1), kappa_max=2.0, q=0.1, mass=5.0,
                  inertia=11.0, dof_mask=W.DOF_TX | W.DOF_TY | W.DOF_ROT, n_itr=1, n_steps=1,
                  x_g0=(8.0, 8.0, 0.0), u0=(0.05, 0.0, 0.0))
    g = np.array([0.0, 0.0, gam])
    k = 2.0 * 0.1 * gam / (1 - gam + 0.1)
    Fx = k * 0.05 * (W0 * W0 / (1 + k * W0 * W0) + 4 * W0 * W1 / (1 + k * W0 * W1)
                     + 4 * W1 * W1 / (1 + k * W1 * W1))
    _, b, _ = orc.forward(pb, g, W.initial_state(pb), W.initial_body(pb))
    assert b[3] == pytest.approx(Fx / 5.0, rel=1e-13)
    assert abs(b[4]) < 1e-18
    assert b[7] == pytest.approx(-Fx / 11.0, rel=1e-13)
    assert b[0] == pytest.approx(8.0 + Fx / 5.0, rel=1e-15)
    assert b[6] == pytest.approx(-Fx / 11.0, rel=1e-13)


def test_quarter_turn_equivariance(orc):
    """Rotating the whole periodic problem by 90 degrees (flow, body position and the
    pose theta0 -> theta0 + pi/2) rotates the solution: D2Q9, the tensor-product
    kernel, Eqs. rigid_body_position/velocity and the torque are all equivariant."""
    L = 20
    base = dict(nu=0.11, nd=(7, 5, 1), kappa_max=0.5, q=0.1, mass=50.0, inertia=2e3,
                dof_mask=W.DOF_TX | W.DOF_TY | W.DOF_ROT, n_itr=3, n_steps=8, seed=8)
    pa = periodic(2, (L, L), x_g0=(10.3, 9.6, 0), theta0=0.1, u0=(0.04, 0.01, 0), **base)
    pr = periodic(2, (L, L), x_g0=(10.4, 10.3, 0), theta0=0.1 + math.pi / 2,
                  u0=(-0.01, 0.04, 0), **base)
    g = W.design(pa)
    sa, ba, _ = orc.forward(pa, g, W.initial_state(pa), W.initial_body(pa))
    sr, br, _ = orc.forward(pr, g, W.initial_state(pr), W.initial_body(pr))
    N = L * L
    x, y, _ = coords(pa)
    rot = (L - y) % L + L * x  # node (x, y) -> (L - y, x)
    assert np.abs(sr[rot] - sa[:N]).max() < 1e-14
    assert np.abs(sr[N + rot] + sa[2 * N:3 * N]).max() < 1e-14
    assert np.abs(sr[2 * N + rot] - sa[N:2 * N]).max() < 1e-14
    assert br[0] == pytest.approx(10.0 - (ba[1] - 10.0), abs=1e-12)
    assert br[1] == pytest.approx(10.0 + (ba[0] - 10.0), abs=1e-12)
    assert br[3] == pytest.approx(-ba[4], abs=1e-15) and br[4] == pytest.approx(ba[3], abs=1e-15)
    assert br[6] - math.pi / 2 == pytest.approx(ba[6], abs=1e-14)
    assert br[7] == pytest.approx(ba[7], abs=1e-15)
    assert abs(ba[7]) > 1e-7  # a torque acted


# ------------------------------------------------- exact adjoint vs finite differences

FD_CASES = {
    "2d-x": lambda: W.small2d(),
    "2d-theta": lambda: W.small2d(objective=W.OBJ_ANGLE, inertia=300.0),
    "2d-y-walls": lambda: W.small2d(objective=W.OBJ_DISP_Y).replace(
        bc=(W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0)),
    "3d-theta": lambda: W.small3d(inertia=150.0),
    "3d-y": lambda: W.small3d(objective=W.OBJ_DISP_Y),
}


@pytest.mark.parametrize("case", sorted(FD_CASES))
def test_gradient_matches_central_differences(orc, case):
    """The oracle's reverse sweep is the exact derivative of its forward map: central
    differences (h = 1e-4, truncation O(h^2)) on random design entries agree."""
    pb = FD_CASES[case]()
    g = W.design(pb)
    s0, b0 = W.initial_state(pb), W.initial_body(pb)
    J, grad = orc.gradient(pb, g, s0, b0)
    assert J == pytest.approx(orc.forward(pb, g, s0, b0)[2], rel=1e-15, abs=1e-300)
    h = 1e-4
    rng = np.random.default_rng(1003)
    idx = rng.choice(pb.ND, 6, replace=False)
    scale = np.abs(grad).max()
    assert scale > 0
    for m in idx:
        gp, gm = g.copy(), g.copy()
        gp[m] += h
        gm[m] -= h
        fd = (orc.forward(pb, gp, s0, b0)[2] - orc.forward(pb, gm, s0, b0)[2]) / (2 * h)
        assert abs(grad[m] - fd) <= 2e-5 * abs(fd) + 2e-6 * scale, (m, grad[m], fd)


@pytest.mark.parametrize("case", ["2d-x", "3d-y"])
def test_initial_state_gradient_matches_central_differences(orc, case):
    """Cotangents of the initial fluid state, at nodes on and next to VELOCITY,
    PRESSURE and WALL faces and in the body's footprint: checks the transposes of the
    boundary treatment and of the one-sided gradients."""
    pb = FD_CASES[case]()
    g = W.design(pb)
    s0, b0 = W.initial_state(pb), W.initial_body(pb)
    J, grad, ds, db = orc.gradient(pb, g, s0, b0, with_initial=True)
    N, nx, ny = pb.N, pb.n[0], pb.n[1]
    z = pb.n[2] // 2
    picks = []
    for (x, y) in ((0, 5), (1, 5), (2, 4), (nx - 1, 6), (nx - 2, 7), (int(pb.x_g0[0]), int(pb.x_g0[1])),
                   (int(pb.x_g0[0]) + 3, 0), (5, 1)):
        node = x + nx * (y + ny * z)
        for comp in range(pb.dim + 1):
            picks.append(comp * N + node)
    h = 1e-6
    scale = np.abs(ds).max()
    for i in picks:
        sp, sm = s0.copy(), s0.copy()
        sp[i] += h
        sm[i] -= h
        fd = (orc.forward(pb, g, sp, b0)[2] - orc.forward(pb, g, sm, b0)[2]) / (2 * h)
        assert abs(ds[i] - fd) <= 1e-5 * abs(fd) + 1e-6 * scale, (i, ds[i], fd)
    # initial body state cotangent (velocity component of the objective's axis)
    for j in (0, 3, 6, 7):
        bp, bm = b0.copy(), b0.copy()
        bp[j] += 1e-6
        bm[j] -= 1e-6
        fd = (orc.forward(pb, g, s0, bp)[2] - orc.forward(pb, g, s0, bm)[2]) / 2e-6
        jac_scale = max(abs(fd), np.abs(db).max())
        assert abs(db[j] - fd) <= 1e-5 * jac_scale + 1e-9, (j, db[j], fd)


def test_invalid_problems_rejected(orc):
    pb = W.small2d()
    with pytest.raises(ValueError):
        orc.forward(pb.replace(dim=4), W.design(pb), W.initial_state(pb), W.initial_body(pb))
    with pytest.raises(ValueError):
        orc.forward(pb.replace(bc=(W.PERIODIC, W.PRESSURE, 0, 0, 0, 0)), W.design(pb),
                    W.initial_state(pb), W.initial_body(pb))
    with pytest.raises(ValueError):
        orc.forward(pb.replace(n_itr=0), W.design(pb), W.initial_state(pb), W.initial_body(pb))


def test_paper_constants_fixture(orc):
    """The printed weights (Sec. 2.2) sum to one and have the second moment 1/3 that the
    shear-wave pin relies on; the viscosity relation at the paper's nu = 0.1 gives A = 0.3,
    and the oracle's shear-wave decay at that A matches the closed form."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")
    c = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            c[k] = float(v)
    assert abs(c["d2q9_w_rest"] + 4 * c["d2q9_w_axis"] + 4 * c["d2q9_w_diag"] - 1) < 1e-15
    assert abs(2 * c["d2q9_w_axis"] + 4 * c["d2q9_w_diag"] - 1 / 3) < 1e-15
    assert abs(c["d3q15_w_rest"] + 6 * c["d3q15_w_axis"] + 8 * c["d3q15_w_corner"] - 1) < 1e-15
    assert abs(2 * c["d3q15_w_axis"] + 8 * c["d3q15_w_corner"] - 1 / 3) < 1e-15
    A = c["A_at_nu_0.1"]
    assert abs((1 / 6 - 2 * A / 9) - 0.1) < 1e-15
    pb = periodic(2, (32, 4), nu=0.1, n_steps=1)
    N = pb.N
    x, _, _ = coords(pb)
    k = 2 * np.pi * 2 / 32
    s0 = np.zeros(3 * N)
    s0[2 * N:] = 1e-7 * np.sin(k * x)
    s1, _, _ = orc.forward(pb, None, s0, np.zeros(12))
    G = 2 / 3 + np.cos(k) / 3 + (2 * A / 9) * np.sin(k) ** 2
    assert np.abs(s1[2 * N:] - G * s0[2 * N:]).max() < 1e-21


# ---------------------------------------------------------------- filter and projection (Sec. 3.2)
FILTER_CASES = [(2, (9, 7, 1), 1.5), (2, (12, 5, 1), 2.6), (3, (6, 5, 4), 1.8), (3, (7, 6, 5), 2.2)]


@pytest.mark.parametrize("dim,nd,R", FILTER_CASES)
def test_filter_preserves_constants(orc, dim, nd, R):
    """Normalised weights sum to one at every point, edges and corners included."""
    n = int(np.prod(nd))
    gt, gh = orc.filter(dim, nd, R, 4.0, 0.5, np.full(n, 0.37))
    assert np.abs(gt - 0.37).max() < 1e-15


@pytest.mark.parametrize("dim,nd,R", FILTER_CASES)
def test_filter_preserves_linear_fields_in_the_interior(orc, dim, nd, R):
    """The cone weights are symmetric about a point whose whole disc lies on the grid, so a
    linear field is reproduced there (and not at the truncated edges)."""
    n = int(np.prod(nd))
    idx = np.arange(n)
    x = np.stack([idx % nd[0], (idx // nd[0]) % nd[1], idx // (nd[0] * nd[1])]).astype(float)
    g = 0.1 + 0.03 * x[0] - 0.02 * x[1] + 0.05 * x[2]
    gt, _ = orc.filter(dim, nd, R, 4.0, 0.5, g)
    r = int(np.floor(R))
    inner = np.all([(x[a] >= r) & (x[a] <= nd[a] - 1 - r) for a in range(dim)], axis=0)
    assert inner.any()
    assert np.abs(gt[inner] - g[inner]).max() < 1e-14
    assert np.abs(gt[~inner] - g[~inner]).max() > 1e-6


@pytest.mark.parametrize("dim,nd,R", FILTER_CASES)
def test_filter_weights_symmetric(orc, dim, nd, R):
    """Responses to unit impulses: gt_i(e_j) / gt_i(e_i) is the raw weight w_ij, which must
    equal w_ji (and 1/gt_i(e_i) is the normaliser W_i)."""
    n = int(np.prod(nd))
    rng = np.random.default_rng(11)
    pts = rng.choice(n, 6, replace=False)
    resp = {}
    for j in pts:
        e = np.zeros(n)
        e[j] = 1.0
        resp[j] = orc.filter(dim, nd, R, 4.0, 0.5, e)[0]
    for i in pts:
        for j in pts:
            wij = resp[j][i] / resp[i][i]
            wji = resp[i][j] / resp[j][j]
            assert abs(wij - wji) < 1e-14


def test_filter_node_weights(orc):
    """Cone weights (R - d)/R: with R = 2 the axis neighbour weighs 1/2 of the centre, the
    diagonal neighbour 1 - sqrt(2)/2, the second axis neighbour nothing."""
    nd = (9, 9, 1)
    e = np.zeros(81)
    c = 4 + 9 * 4
    e[c] = 1.0
    gt, _ = orc.filter(2, nd, 2.0, 1.0, 0.5, e)
    w = gt / gt[c]
    assert abs(w[c + 1] - 0.5) < 1e-15 and abs(w[c + 9] - 0.5) < 1e-15
    assert abs(w[c + 10] - (1 - np.sqrt(2) / 2)) < 1e-15
    assert w[c + 2] == 0.0 and w[c + 18] == 0.0


def test_filter_identity_below_unit_radius(orc):
    g = np.random.default_rng(3).random(60)
    gt, _ = orc.filter(3, (5, 4, 3), 0.9, 2.0, 0.5, g)
    assert np.array_equal(gt, g)


def test_projection_limits_and_symmetry(orc):
    """Projection: 0 -> 0, 1 -> 1, monotone; with eta = 1/2 it is odd about 1/2; beta -> 0
    gives the identity, large beta a step at eta."""
    g = np.linspace(0.0, 1.0, 41)
    nd = (41, 1, 1)
    for beta in (0.5, 4.0, 32.0):
        _, gh = orc.filter(2, nd, 0.5, beta, 0.5, g)
        assert abs(gh[0]) < 1e-15 and abs(gh[-1] - 1.0) < 1e-15
        assert np.all(np.diff(gh) > 0)
        assert np.abs(gh + gh[::-1] - 1.0).max() < 1e-14
    _, gh = orc.filter(2, nd, 0.5, 1e-5, 0.3, g)
    assert np.abs(gh - g).max() < 1e-9
    _, gh = orc.filter(2, nd, 0.5, 2000.0, 0.3, g)
    assert np.all(gh[g < 0.29] < 1e-6) and np.all(gh[g > 0.31] > 1 - 1e-6)


@pytest.mark.parametrize("dim,nd,R", FILTER_CASES)
def test_filter_adjoint_vs_finite_differences(orc, dim, nd, R):
    """<gbh, d gh> = <gb, d g> for a random direction, d gh by central differences."""
    n = int(np.prod(nd))
    rng = np.random.default_rng(7)
    g = rng.random(n)
    beta, eta = 6.0, 0.45
    gt, _ = orc.filter(dim, nd, R, beta, eta, g)
    gbh = rng.standard_normal(n)
    gb = orc.filter_adjoint(dim, nd, R, beta, eta, gt, gbh)
    d = rng.standard_normal(n)
    h = 1e-6
    ghp = orc.filter(dim, nd, R, beta, eta, g + h * d)[1]
    ghm = orc.filter(dim, nd, R, beta, eta, g - h * d)[1]
    lhs = gbh @ ((ghp - ghm) / (2 * h))
    rhs = gb @ d
    assert abs(lhs - rhs) <= 1e-7 * max(abs(rhs), 1.0)


# ------------------------------------------ terminal adjoint values (Sec. 3.4, warm start)

@pytest.mark.parametrize("case", ["2d-theta", "3d-y"])
def test_terminal_cotangents_match_central_differences(orc, case):
    """With terminal adjoint values the sweep differentiates
    L = seed J + <dstate_T, state(N_t)> + <dbody_T, body(N_t)>: central differences of L
    along a random design direction agree."""
    pb = FD_CASES[case]()
    g = W.design(pb)
    s0, b0 = W.initial_state(pb), W.initial_body(pb)
    rng = np.random.default_rng(77)
    sT = rng.standard_normal(s0.size) * 0.1
    bT = np.zeros(12)
    bT[:8] = rng.standard_normal(8)
    seed = 0.6

    def L(gg):
        st, bd, J = orc.forward(pb, gg, s0, b0)
        return seed * J + sT @ st + bT[:8] @ bd[:8]

    J, grad = orc.gradient(pb, g, s0, b0, seed=seed, dstate_T=sT, dbody_T=bT)
    v = rng.standard_normal(g.size)
    h = 1e-4
    fd = (L(g + h * v) - L(g - h * v)) / (2 * h)
    assert grad @ v == pytest.approx(fd, rel=2e-5, abs=1e-9 * np.abs(grad).sum())
    # without the terminal values the sweep is the plain gradient
    J0, grad0 = orc.gradient(pb, g, s0, b0, seed=seed)
    assert np.abs(grad0 - grad).max() > 1e-6 * np.abs(grad).max()


@pytest.mark.parametrize("case", ["2d-x", "2d-theta", "3d-theta"])
def test_gradient_chains_over_split_runs(orc, case):
    """A run of N_t steps split into two runs (the second starts from the first's final
    state and body) gives the same objective and gradient when the second run's initial
    cotangents are the first run's terminal adjoint values: J = J1 + J2 telescopes and the
    two sweeps add up to the sweep of the whole run, initial cotangents included."""
    pb = FD_CASES[case]().replace(n_steps=11)
    n1 = 4
    g = W.design(pb)
    s0, b0 = W.initial_state(pb), W.initial_body(pb)
    seed = 1.3
    J, grad, ds, db = orc.gradient(pb, g, s0, b0, seed=seed, with_initial=True)
    p1, p2 = pb.replace(n_steps=n1), pb.replace(n_steps=pb.n_steps - n1)
    s1, b1, _ = orc.forward(p1, g, s0, b0)
    J2, g2, ds1, db1 = orc.gradient(p2, g, s1, b1, seed=seed, with_initial=True)
    J1, g1, ds0, db0 = orc.gradient(p1, g, s0, b0, seed=seed, with_initial=True, dstate_T=ds1, dbody_T=db1)
    assert J1 + J2 == pytest.approx(J, rel=1e-11, abs=1e-15)
    scale = np.abs(grad).max()
    assert np.abs(g1 + g2 - grad).max() <= 1e-11 * scale
    assert np.abs(ds0 - ds).max() <= 1e-11 * np.abs(ds).max()
    assert np.abs(db0[:8] - db[:8]).max() <= 1e-11 * np.abs(db[:8]).max()


# ------------------------------------------------- cyclic periodic design (Sec. 4.2)

def _design_problem(dim, nd, axis=0):
    pb = W.small2d(nd=nd) if dim == 2 else W.small3d(nd=nd)
    return pb.replace(axis=axis) if dim == 3 else pb


def _plane_view(pb, g):
    """(w, v, u) view of a design array: u, v the rotation plane's axes (pi, pj), w the
    rotation axis, as the library defines them (pi = axis + 1, pj = axis + 2 mod 3)."""
    a = pb.axis if pb.dim == 3 else 2
    pi, pj = (a + 1) % 3, (a + 2) % 3
    arr = np.asarray(g).reshape(pb.nd[2], pb.nd[1], pb.nd[0])  # (z, y, x)
    ax_of = {0: 2, 1: 1, 2: 0}  # grid axis -> array axis
    return np.transpose(arr, (ax_of[a], ax_of[pj], ax_of[pi]))


CYC_CASES = [(2, (6, 6, 1), 0, 4), (2, (5, 5, 1), 0, 4), (2, (7, 4, 1), 0, 2), (2, (5, 3, 1), 0, 2),
             (3, (4, 6, 6), 0, 4), (3, (5, 3, 4), 1, 2), (3, (5, 5, 3), 2, 4), (2, (4, 3, 1), 0, 1)]


@pytest.mark.parametrize("case", range(len(CYC_CASES)))
def test_cyclic_expansion_is_rotation_invariant(orc, case):
    """The expanded design is unchanged by the rotations of the group (checked with
    numpy's rot90 / flips of the plane), every sector variable appears exactly on its
    orbit (orbit sizes n_sec, or 1 at fixed points), and collection is the transpose."""
    dim, nd, axis, n = CYC_CASES[case]
    pb = _design_problem(dim, nd, axis)
    ns = orc.cyclic_sector_points(pb, n)
    assert ns > 0
    rng = np.random.default_rng(case)
    gs = rng.random(ns)
    g = orc.cyclic_expand(pb, n, gs)
    V = _plane_view(pb, g)
    if n == 2:
        assert np.array_equal(V, V[:, ::-1, ::-1])
    if n == 4:
        assert np.array_equal(V, np.rot90(V, 1, axes=(1, 2)))
    # each sector value occupies a whole orbit: counts are orbit sizes, summing to ND
    counts = orc.cyclic_collect(pb, n, np.ones(g.size))
    assert counts.sum() == pytest.approx(g.size)
    assert set(np.unique(counts)) <= {1.0, float(n)}
    assert np.isin(g, gs).all() and np.unique(g).size == ns
    # transpose
    x = rng.standard_normal(g.size)
    assert orc.cyclic_collect(pb, n, x) @ gs == pytest.approx(x @ g, rel=1e-13)


def test_cyclic_expansion_small_tables(orc):
    """Hand-derived layouts: a 3x3 plane with four sectors (corners, edge midpoints,
    centre) and a 3x2 plane with two (q and 5 - q)."""
    pb = _design_problem(2, (3, 3, 1))
    assert orc.cyclic_sector_points(pb, 4) == 3
    a, b, c = 1.0, 2.0, 3.0
    assert np.array_equal(orc.cyclic_expand(pb, 4, [a, b, c]).reshape(3, 3),
                          [[a, b, a], [b, c, b], [a, b, a]])
    pb = _design_problem(2, (3, 2, 1))
    assert orc.cyclic_sector_points(pb, 2) == 3
    assert np.array_equal(orc.cyclic_expand(pb, 2, [a, b, c]), [a, b, c, c, b, a])
    assert orc.cyclic_sector_points(pb, 4) == -1  # quarter turns need a square plane
    assert orc.cyclic_sector_points(pb, 3) == -1


# ----------------------------- coupling constant of the fluid <-> body iteration (Sec. 3.1)

def _covering3d(kmax=0.4, gam=0.5):
    """Periodic 6x5x4 grid covered by a node-aligned 12x11x10 design (design points on
    nodes, >= 2 beyond every face): kappa(x) = kappa_ref and sum_m W r_m = x - x^G."""
    pb = periodic(3, (6, 5, 4), nu=0.1, nd=(12, 11, 10), kappa_max=kmax, q=0.1, mass=60.0,
                  inertia=1e3, axis=0, dof_mask=W.DOF_TX, n_itr=1, n_steps=1,
                  x_g0=(2.5, 2.0, 1.5), u0=(0.04, 0.01, -0.02))
    kr = kmax * 0.1 * gam / (1 - gam + 0.1)
    return pb, np.full(pb.ND, gam), kr


@pytest.mark.parametrize("dim", [2, 3])
def test_coupling_constant_closed_form(orc, dim):
    """The coupling constants K = -dF/du^G and K_theta = -dT/domega at a frozen pose and
    u* (Sec. 3.1's iteration contracts when K/M < 1). With a node-aligned design covering
    the grid, kappa = kappa_ref, sum_m W = 1 at every node and sum_m W r_m = x - x^G
    (the three node weights 1/4, 1/2, 1/4 are symmetric), so
    K = kappa_ref (N_D - N kappa_ref/(1 + kappa_ref)) and
    K_theta = kappa_ref (sum_m |r_m,perp|^2 - kappa_ref/(1 + kappa_ref) sum_x |(x - x^G)_perp|^2),
    perp = the part across the rotation axis. Sums over coordinates only; no weights."""
    if dim == 2:
        pb, g, kr = covering(1, W.DOF_TX)
        plane = (0, 1)
    else:
        pb, g, kr = _covering3d()
        plane = (1, 2)
    N, ND = pb.N, pb.ND
    K = orc.coupling(pb, g, W.initial_state(pb), W.initial_body(pb))
    f = kr / (1 + kr)
    Kt = kr * (ND - N * f)
    # lever arms: design offsets xi_m (theta = 0) and node offsets from x^G
    xi = [np.arange(pb.nd[a]) - 0.5 * (pb.nd[a] - 1) for a in range(3)]
    XI = np.meshgrid(*xi, indexing="ij")
    xs = [np.arange(pb.n[a]) - pb.x_g0[a] for a in range(3)]
    XS = np.meshgrid(*xs, indexing="ij")
    r2 = sum((XI[a] ** 2).sum() for a in plane)
    x2 = sum((XS[a] ** 2).sum() for a in plane)
    Kr = kr * (r2 - f * x2)
    for a in range(dim):
        assert K[a] == pytest.approx(Kt, rel=1e-12)
    for a in range(dim, 3):
        assert K[a] == 0.0
    assert K[3] == pytest.approx(Kr, rel=1e-12)
    assert Kt > 0 and Kr > 0


@pytest.mark.parametrize("mass", [400.0, 60.0, 25.0])
def test_iteration_contracts_at_ratio_K_over_M(orc, mass):
    """Within one step the iterates of Sec. 3.1 satisfy u^G,(k+1) = u^G(t-1) + F(u^G,(k))/M,
    and F is affine in the body velocity with slope -K at a frozen pose: successive
    differences of the iterates shrink by the factor -K/M (the pose moves only by the
    tiny u^G itself). Ties the forward loop to the coupling constant on a generic body
    in a channel, with K/M from 0.007 to 0.11."""
    pb = W.small2d(dof_mask=W.DOF_TX, n_steps=1, mass=mass, theta0=0.0)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    K = orc.coupling(pb, g, s0, b0)
    it = [orc.forward(pb.replace(n_itr=n), g, s0, b0)[1][3] for n in range(1, 6)]
    d = np.diff(it)
    for r in d[1:] / d[:-1]:
        assert r == pytest.approx(-K[0] / mass, rel=1e-4)


def test_rotation_iteration_contracts_at_ratio_K_over_I(orc):
    """The same for a body rotating about a fixed pivot: the angular velocity iterates
    shrink by -K_theta/I (the pose turns with the iterate, so only to 0.5 %)."""
    pb = W.small2d(dof_mask=W.DOF_ROT, n_steps=1, inertia=300.0, theta0=0.0)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    K = orc.coupling(pb, g, s0, b0)
    it = [orc.forward(pb.replace(n_itr=n), g, s0, b0)[1][7] for n in range(1, 6)]
    d = np.diff(it)
    for r in d[1:] / d[:-1]:
        assert r == pytest.approx(-K[3] / pb.inertia, rel=5e-3)


# ------------------------------------------- steady channel: flux and Poiseuille law (Sec. 2.2)

def test_steady_channel_flux_and_poiseuille_law(orc):
    """A body-free channel with a VELOCITY inlet, a PRESSURE outlet and WALLs reaches a
    steady state whose developed part is the plane Poiseuille flow of the scheme's
    viscosity: the flux sum_y u_x is the same in every developed cross-section, the
    pressure is uniform across it, and u_x = (G / 2 nu) y (H - y) with G the measured
    pressure slope (the discrete profile is an exact fixed point, so this holds to
    convergence). Pins the three boundary kinds together with nu = 1/6 - 2A/9."""
    U, nu = 0.05, 0.2
    pb = W.Problem(dim=2, n=(60, 12, 1), bc=(W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0),
                   bc_u=((U, 0, 0),) + ((0, 0, 0),) * 5, nu=nu, u0=(U, 0, 0), n_steps=6000)
    s, _, _ = orc.forward(pb, None, W.initial_state(pb), np.zeros(12))
    N, nx, ny = pb.N, pb.n[0], pb.n[1]
    s2, _, _ = orc.forward(pb.replace(n_steps=50), None, s, np.zeros(12))
    assert np.abs(s2 - s).max() < 1e-14  # steady
    p = s[:N].reshape(ny, nx)
    ux = s[N:2 * N].reshape(ny, nx)
    uy = s[2 * N:].reshape(ny, nx)
    Q = ux.sum(axis=0)
    dev = slice(40, nx - 2)
    assert np.abs(Q[dev] - Q[dev].mean()).max() <= 1e-8 * Q[dev].mean()
    H = ny - 1
    y = np.arange(ny)
    for x in range(45, nx - 2):
        G = -(p[1:-1, x + 1] - p[1:-1, x - 1]).mean() / 2
        assert np.abs(p[:, x] - p[:, x].mean()).max() <= 1e-9 * G
        assert np.abs(ux[:, x] - G / (2 * nu) * y * (H - y)).max() <= 1e-7 * ux[:, x].max()
        assert np.abs(uy[:, x]).max() <= 1e-9 * ux[:, x].max()
    # the inlet's flux sum_y u_x = (ny - 2) U is not the scheme's conserved flux (the
    # macroscopic u differs from the mass flux by the viscous term near the inlet)
    assert Q[0] == pytest.approx((ny - 2) * U, rel=1e-15)


# --------------------------------------- dot-product tests of the reverse sweep (adjointness)

def _rand_state(pb, seed, amp=0.01):
    rng = np.random.default_rng(seed)
    return W.initial_state(pb) + amp * rng.standard_normal(pb.N * (pb.dim + 1))


DOT_CASES = {
    "2d-vel-pres-walls": lambda: W.Problem(dim=2, n=(13, 9, 1),
                                           bc=(W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0),
                                           bc_u=((0.05, 0.01, 0),) + ((0, 0, 0),) * 5,
                                           bc_p=(0, 0.002, 0, 0, 0, 0), nu=0.12, u0=(0.05, 0, 0)),
    "2d-pres-pres-periodic": lambda: W.Problem(dim=2, n=(11, 8, 1),
                                               bc=(W.PRESSURE, W.PRESSURE, 0, 0, 0, 0),
                                               bc_p=(0.01, 0.0, 0, 0, 0, 0), nu=0.15),
    "3d-duct": lambda: W.duct3d(9, 7, 6, 0.04, 0.05),
    "3d-mixed": lambda: W.Problem(dim=3, n=(8, 7, 6),
                                  bc=(W.WALL, W.VELOCITY, W.PRESSURE, W.WALL, 0, 0),
                                  bc_u=((0, 0, 0), (0.02, -0.03, 0.01)) + ((0, 0, 0),) * 4,
                                  bc_p=(0, 0, 0.003, 0, 0, 0), nu=0.07),
}


@pytest.mark.parametrize("case", sorted(DOT_CASES))
def test_one_step_adjoint_dot_product_body_free(orc, case):
    """One LKS step with its boundary values is a quadratic polynomial in the state
    (the equilibrium of Sec. 2.2 is quadratic in u, the gradients linear), so its central
    difference is exact up to rounding: <w, (F(s + h v) - F(s - h v)) / 2h> must equal
    <F'(s)^T w, v>, the reverse sweep's initial-state cotangent for the terminal
    cotangent w, to 1e-11. A transposed stencil, boundary copy or one-sided gradient
    fails it."""
    pb = DOT_CASES[case]().replace(n_steps=1, nd=(0, 0, 0))
    s0 = _rand_state(pb, 5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(s0.size)
    w = rng.standard_normal(s0.size)
    h = 1e-3
    fp = orc.forward(pb, None, s0 + h * v, np.zeros(12))[0]
    fm = orc.forward(pb, None, s0 - h * v, np.zeros(12))[0]
    lhs = w @ ((fp - fm) / (2 * h))
    _, _, ds, _ = orc.gradient(pb, np.zeros(1), s0, np.zeros(12), seed=0.0, with_initial=True,
                               dstate_T=w)
    rhs = ds @ v
    assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-13 * np.abs(ds).sum())


@pytest.mark.parametrize("dim", [2, 3])
def test_one_step_adjoint_dot_product_held_body(orc, dim):
    """With every degree of freedom held, the pose is fixed and a step (LKS, then the
    Brinkman correction with the mapped kappa, u^S of Eqs. kappa_mapping, us_mapping, u)
    stays quadratic in the state: the same exact dot-product test covers the Brinkman
    transpose and the spread over the body's footprint, with a body moving at a given
    velocity (u^S != 0)."""
    pb = (W.small2d() if dim == 2 else W.small3d()).replace(n_steps=1, dof_mask=0, n_itr=2)
    g = W.design(pb)
    s0 = _rand_state(pb, 7)
    b0 = W.initial_body(pb)
    b0[3:6] = (0.01, -0.02, 0.015)[:3]
    b0[7] = 0.003
    rng = np.random.default_rng(8)
    v = rng.standard_normal(s0.size)
    w = rng.standard_normal(s0.size)
    h = 1e-3
    fp = orc.forward(pb, g, s0 + h * v, b0)[0]
    fm = orc.forward(pb, g, s0 - h * v, b0)[0]
    lhs = w @ ((fp - fm) / (2 * h))
    _, _, ds, _ = orc.gradient(pb, g, s0, b0, seed=0.0, with_initial=True, dstate_T=w)
    assert lhs == pytest.approx(ds @ v, rel=1e-11, abs=1e-13 * np.abs(ds).sum())


@pytest.mark.parametrize("dim", [2, 3])
def test_one_step_adjoint_dot_product_free_body(orc, dim):
    """A free body makes the step nonlinear in the state and the body (the pose enters the
    cosine weights): the reverse sweep's cotangents of the initial state and body, for
    random terminal cotangents of both, match a joint central difference (h = 1e-6) along
    random directions, to the truncation error."""
    pb = (W.small2d() if dim == 2 else W.small3d()).replace(n_steps=1, inertia=200.0)
    g = W.design(pb)
    s0 = _rand_state(pb, 9)
    b0 = W.initial_body(pb)
    rng = np.random.default_rng(10)
    v, w = rng.standard_normal(s0.size), rng.standard_normal(s0.size)
    vb, wb = np.zeros(12), np.zeros(12)
    vb[:8] = rng.standard_normal(8)
    wb[:8] = rng.standard_normal(8)
    if dim == 2:  # z components do not exist in 2D
        vb[[2, 5]] = 0.0
        wb[[2, 5]] = 0.0
    h = 1e-6

    def L(s, b):
        st, bd, _ = orc.forward(pb, g, s, b)
        return w @ st + wb[:8] @ bd[:8]

    fd = (L(s0 + h * v, b0 + h * vb) - L(s0 - h * v, b0 - h * vb)) / (2 * h)
    _, _, ds, db = orc.gradient(pb, g, s0, b0, seed=0.0, with_initial=True, dstate_T=w, dbody_T=wb)
    assert ds @ v + db[:8] @ vb[:8] == pytest.approx(fd, rel=1e-7)


def test_unstable_coupling_diverges(orc):
    """The stability reading of Sec. 3.1's iteration: with K/M above one the iterates of
    every step overshoot and the body velocity grows without bound within a few dozen
    steps; at K/M = 0.5 (how the configurations are set) it stays of the order of the
    flow's drag. This is what the library's LKS_FLAG_STABILITY pre-check rejects."""
    base = W.small2d(dof_mask=W.DOF_TX, theta0=0.0, n_steps=1)
    g, s0, b0 = W.design(base), W.initial_state(base), W.initial_body(base)
    K = orc.coupling(base, g, s0, b0)[0]
    speeds = {}
    for ratio in (0.5, 1.6):
        pb = base.replace(mass=K / ratio, n_steps=40)
        _, b, _, tr = orc.forward(pb, g, s0, b0, traj=True)
        speeds[ratio] = np.abs(tr[:, 3])
    assert np.all(np.isfinite(speeds[0.5])) and speeds[0.5].max() < 0.1
    grown = speeds[1.6]
    assert not np.all(np.isfinite(grown)) or grown[-1] > 1e3 * speeds[0.5].max()


# ----------------------------------------- the paper's adjoint variant (Sec. 2.5, App. B)

WALLS2 = (W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0)
PAPER_ADJ = {
    # case: (problem, bound on the relative L2 difference from the exact adjoint)
    "2d-x": (lambda: W.small2d(), 5e-3),
    "2d-theta": (lambda: W.small2d(objective=W.OBJ_ANGLE, inertia=300.0, dof_mask=W.DOF_ROT), 5e-3),
    "3d-x": (lambda: W.small3d(dof_mask=W.DOF_TX, objective=W.OBJ_DISP_X), 5e-3),
    "3d-theta": (lambda: W.small3d(inertia=150.0), 0.1),
    "shear-y": (lambda: W.small2d(dof_mask=W.DOF_TY, objective=W.OBJ_DISP_Y, n_steps=30, x_g0=(14.3, 8.6, 0.0),
                                  mass=20.0, kappa_max=2.0).replace(bc=WALLS2), 3e-2),
    "shear-rot": (lambda: W.small2d(dof_mask=W.DOF_ROT, objective=W.OBJ_ANGLE, n_steps=30, x_g0=(14.3, 8.6, 0.0),
                                    inertia=200.0, kappa_max=2.0).replace(bc=WALLS2), 5e-2),
}


@pytest.mark.parametrize("case", sorted(PAPER_ADJ))
def test_paper_adjoint_agrees_with_the_exact_adjoint(orc, case):
    """The paper's variant (continuous adjoint discretised like the forward: ALKS, Eq. au,
    Eqs. axg..aomega iterated N_itr times, Eq. design_sensitivity) approximates the exact
    derivative of the discrete map, which central differences pin: the paper reports
    "good agreement" with finite differences (App. B). Measured here: 0.1-0.2 % relative
    L2 for the small 2D/3D bodies in a nearly uniform flow, 6 % for a 3D rotation whose
    objective is ~1e-6, 1.5-2.6 % for a strongly coupled body crossing a sheared channel
    flow. Dropping Eq. au's body terms or its Brinkman factor, or the sign of the
    sensitivity's body terms, fails the bounds (checked by planting each mistake). The
    pose-derivative terms of Eqs. axg and atheta are below this discretisation
    difference in every case tried: they are not pinned by it."""
    make, bound = PAPER_ADJ[case]
    pb = make()
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    J, ge = orc.gradient(pb, g, s0, b0)
    Jp, gp = orc.gradient_paper(pb, g, s0, b0)
    assert Jp == J
    rel = np.linalg.norm(gp - ge) / np.linalg.norm(ge)
    assert rel < bound, rel
    # same direction, to the same bound
    cos = gp @ ge / (np.linalg.norm(gp) * np.linalg.norm(ge))
    assert cos > 1.0 - bound
