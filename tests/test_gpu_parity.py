"""Parity of the gfx950 library (through the C ABI) with the FP64 oracle.

Tolerances: FP64 GPU vs FP64 oracle differ only in summation order and contraction,
so states/body agree to ~1e-12 relative after tens of steps; we allow 1e-9 (fields,
body, objective) and 1e-8 relative L2 (gradients). FP32 fields: the objective within
1e-4 relative and the gradient within 1e-3 relative L2 (the accuracy targets of the
FP32 path); fields within 1e-5 of their scale.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2601_18272_amd as lib

    lib._lib.load()
    return lib


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def elem(a, b):
    """Largest entry-wise difference relative to the largest reference entry: a wrong
    small entry (for example on the body's rim) cannot hide under the L2 norm."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def kernel_flags(L, pb, march):
    """Flags selecting the form of the LKS kernels. 2D: the column march (march=True,
    forced) or the size default (the tile kernels at these sizes). 3D: with march=True the
    fields are addressed one plane at a time (the form of fields of 2^31 bytes and more),
    else whole (the form at these sizes)."""
    if march:
        return L._lib.FLAG_MARCH2D if pb.dim == 2 else L._lib.FLAG_PLANE3D
    return 0


def smooth_state(pb, seed, amp=1e-2):
    """Random smooth perturbation of the initial state (boundary values untouched
    matter not: the first step re-imposes them)."""
    rng = np.random.default_rng(seed)
    s = W.initial_state(pb).reshape(pb.dim + 1, -1)
    x = np.arange(pb.N) % pb.n[0]
    y = (np.arange(pb.N) // pb.n[0]) % pb.n[1]
    z = np.arange(pb.N) // (pb.n[0] * pb.n[1])
    for c in range(pb.dim + 1):
        k = rng.integers(1, 3, size=3)
        ph = rng.random(3) * 2 * np.pi
        s[c] += amp * np.sin(2 * np.pi * k[0] * x / pb.n[0] + ph[0]) * np.cos(
            2 * np.pi * k[1] * y / pb.n[1] + ph[1]) * np.cos(2 * np.pi * k[2] * z / max(pb.n[2], 1) + ph[2])
    return s.reshape(-1)


BODYFREE = {
    "2d-periodic": lambda: W.Problem(dim=2, n=(77, 29, 1), bc=(0,) * 6, nu=0.09, n_steps=7),
    "2d-walls": lambda: W.Problem(dim=2, n=(70, 19, 1), bc=(W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0),
                                  bc_u=((0.04, 0.01, 0),) + ((0, 0, 0),) * 5, bc_p=(0, 2e-3, 0, 0, 0, 0),
                                  nu=0.12, n_steps=9),
    "2d-pressure": lambda: W.Problem(dim=2, n=(130, 17, 1), bc=(W.PRESSURE, W.PRESSURE, W.WALL, W.VELOCITY, 0, 0),
                                     bc_u=((0, 0, 0),) * 3 + ((0.02, 0, 0),) + ((0, 0, 0),) * 2,
                                     bc_p=(1e-3, -1e-3, 0, 0, 0, 0), nu=0.05, n_steps=9),
    "3d-periodic": lambda: W.Problem(dim=3, n=(13, 11, 9), bc=(0,) * 6, nu=0.07, n_steps=5),
    # two tiles along x (60 columns each) that wrap across the periodic seam
    "3d-periodic-wide": lambda: W.Problem(dim=3, n=(67, 8, 6), bc=(0,) * 6, nu=0.07, n_steps=4),
    "3d-duct": lambda: W.duct3d(19, 10, 9, 0.04, 0.03, n_steps=6),
    # n - 2 a multiple of the 3D adjoint's output tile (60 x 6): its tiles shift by one
    # node along x and along y
    "3d-duct-shifted-tiles": lambda: W.duct3d(62, 14, 7, 0.04, 0.03, n_steps=4),
    "3d-mixed": lambda: W.Problem(dim=3, n=(12, 9, 10), bc=(W.PRESSURE, W.PRESSURE, 0, 0, W.WALL, W.VELOCITY),
                                  bc_u=((0, 0, 0),) * 5 + ((0.03, -0.01, 0),), bc_p=(2e-3, 0, 0, 0, 0, 0),
                                  nu=0.1, n_steps=5),
}


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
@pytest.mark.parametrize("case", sorted(BODYFREE))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bodyfree_forward(L, orc, case, prec, march):
    pb = BODYFREE[case]()
    fl = kernel_flags(L, pb, march)
    s0 = smooth_state(pb, 3)
    b0 = np.zeros(12)
    ref, _, _ = orc.forward(pb, None, s0, b0)
    st, _, _, _ = L.forward(pb, None, s0, b0, precision=prec, store_ckpt=False, flags=fl)
    got = st.cpu().numpy()
    scale = np.abs(ref).max()
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert np.abs(got - ref).max() <= tol * scale, np.abs(got - ref).max() / scale


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
@pytest.mark.parametrize("case", sorted(BODYFREE))
def test_bodyfree_adjoint_initial_state(L, orc, case, march):
    """The fluid adjoint of the body-free channels, observed through a tiny porous body:
    the gradient and the cotangents of the initial state and body."""
    pb = BODYFREE[case]()
    fl = kernel_flags(L, pb, march)
    pb = pb.replace(ckpt_every=3)
    # attach a small porous body so that the objective depends on the fluid
    d = pb.dim
    nd = (4, 3, 1) if d == 2 else (3, 3, 2)
    xg = tuple(np.array(pb.n[:d]) / 2 + 0.37) + ((0.0,) if d == 2 else ())
    pb = pb.replace(nd=nd, kappa_max=0.4, q=0.1, mass=30.0, inertia=500.0, axis=d == 3 and 1 or 2,
                    dof_mask=W.DOF_TX | W.DOF_TY | W.DOF_ROT, n_itr=2, objective=W.OBJ_DISP_Y,
                    x_g0=xg + (0.0,) * (3 - len(xg)), theta0=0.3, seed=5)
    s0 = smooth_state(pb, 4)
    g = W.design(pb)
    b0 = W.initial_body(pb)
    J, grad, ds, db = orc.gradient(pb, g, s0, b0, with_initial=True)
    _, _, Jg, B = L.forward(pb, g, s0, b0, precision="fp64", flags=fl)
    gg, dsg, dbg = L.adjoint(pb, g, B, precision="fp64", want_initial=True, flags=fl)
    assert abs(Jg.item() - J) <= 1e-9 * abs(J) + 1e-15
    assert rel(gg.cpu().numpy(), grad) < 1e-8
    assert elem(gg.cpu().numpy(), grad) < 1e-8
    assert rel(dsg.cpu().numpy(), ds) < 1e-8
    assert elem(dsg.cpu().numpy(), ds) < 1e-8
    assert np.abs(dbg.cpu().numpy()[:8] - db[:8]).max() <= 1e-8 * np.abs(db[:8]).max()


BODY = {
    "small2d": lambda: W.small2d(ckpt_every=5),
    "small2d-rot": lambda: W.small2d(objective=W.OBJ_ANGLE, inertia=300.0, ckpt_every=4,
                                     dof_mask=W.DOF_ROT),
    "small2d-walls": lambda: W.small2d(ckpt_every=12).replace(bc=(W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0),
                                                              objective=W.OBJ_DISP_Y),
    "small3d": lambda: W.small3d(ckpt_every=4, inertia=150.0),
    "small3d-y": lambda: W.small3d(ckpt_every=6, objective=W.OBJ_DISP_Y, axis=2),
    "small3d-tx": lambda: W.small3d(ckpt_every=2, dof_mask=W.DOF_TX, objective=W.OBJ_DISP_X,
                                    theta0=0.0, axis=1),
}


@pytest.mark.parametrize("case", sorted(BODY))
def test_coupled_forward_fp64(L, orc, case):
    pb = BODY[case]()
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    sref, bref, Jref = orc.forward(pb, g, s0, b0)
    st, bd, J, _ = L.forward(pb, g, s0, b0, precision="fp64", store_ckpt=False)
    assert np.abs(st.cpu().numpy() - sref).max() <= 1e-11 * np.abs(sref).max()
    assert np.abs(bd.cpu().numpy()[:8] - bref[:8]).max() <= 1e-11 * max(1.0, np.abs(bref[:8]).max())
    assert abs(J.item() - Jref) <= 1e-9 * abs(Jref) + 1e-16


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
@pytest.mark.parametrize("case", sorted(BODY))
def test_coupled_gradient_fp64(L, orc, case, march):
    pb = BODY[case]()
    fl = kernel_flags(L, pb, march)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    Jref, gref = orc.gradient(pb, g, s0, b0, seed=1.7)
    _, _, J, B = L.forward(pb, g, s0, b0, precision="fp64", flags=fl)
    gg = L.adjoint(pb, g, B, seed=1.7, precision="fp64", flags=fl).cpu().numpy()
    assert abs(J.item() - Jref) <= 1e-9 * abs(Jref) + 1e-16
    assert rel(gg, gref) < 1e-8
    assert elem(gg, gref) < 1e-8


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
@pytest.mark.parametrize("case", sorted(BODY))
def test_coupled_fp32_targets(L, orc, case, march):
    """FP32 fields with FP64 body state and reductions: objective within 1e-4 relative,
    gradient within 1e-3 relative L2 of the FP64 oracle."""
    pb = BODY[case]()
    fl = kernel_flags(L, pb, march)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    Jref, gref = orc.gradient(pb, g, s0, b0)
    _, _, J, B = L.forward(pb, g, s0, b0, precision="fp32", flags=fl)
    gg = L.adjoint(pb, g, B, precision="fp32", flags=fl).cpu().numpy()
    assert abs(J.item() - Jref) <= 1e-4 * abs(Jref)
    assert rel(gg, gref) < 1e-3
    assert elem(gg, gref) < 1e-3


def test_map_design_matches_oracle(L, orc):
    for pb, th in ((W.small2d(), 0.7), (W.small3d(), -1.1), (W.small3d(axis=1), 2.5)):
        kr = orc.kappa_ref(pb, W.design(pb))
        b = W.initial_body(pb)
        b[6] = th
        b[3:6] = (0.01, -0.02, 0.03)
        b[7] = 0.004
        kref, uref = orc.map_design(pb, kr, b)
        for prec, tol in (("fp64", 1e-13), ("fp32", 2e-6)):
            k, u = L.map_design(pb, kr, b, precision=prec)
            assert np.abs(k.cpu().numpy() - kref).max() <= tol * np.abs(kref).max()
            assert np.abs(u.cpu().numpy() - uref).max() <= tol * np.abs(uref).max()


def test_body_step_matches_oracle(L, orc):
    pb = W.small3d(dof_mask=W.DOF_TX | W.DOF_TZ | W.DOF_ROT)
    rng = np.random.default_rng(2)
    for _ in range(3):
        b = rng.standard_normal(12)
        ft = rng.standard_normal(4)
        ref = orc.body_step(pb, ft, b)
        got = L.body_step(pb, ft, b).cpu().numpy()
        assert np.abs(got[:8] - ref[:8]).max() <= 1e-15 * np.abs(ref[:8]).max()
        assert np.array_equal(got[8:], b[8:])


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
def test_deterministic_and_checkpoint_consistent(L, march):
    """Two runs are bitwise identical (gather-form mapping, fixed-order reductions),
    and the gradient does not depend on the checkpoint interval beyond rounding."""
    pb = W.small2d(ckpt_every=5)
    fl = kernel_flags(L, pb, march)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    outs = []
    for _ in range(2):
        st, bd, J, B = L.forward(pb, g, s0, b0, precision="fp32", flags=fl)
        gr = L.adjoint(pb, g, B, precision="fp32", flags=fl)
        outs.append((st.cpu().numpy(), bd.cpu().numpy(), J.item(), gr.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2] and np.array_equal(outs[0][3], outs[1][3])
    # the recomputed segment reproduces the forward bit for bit: any K gives the same
    pb2 = pb.replace(ckpt_every=3)
    _, _, J2, B2 = L.forward(pb2, g, s0, b0, precision="fp32", flags=fl)
    gr2 = L.adjoint(pb2, g, B2, precision="fp32", flags=fl).cpu().numpy()
    assert J2.item() == outs[0][2]
    assert np.array_equal(gr2, outs[0][3])


def test_autograd_function(L, orc):
    import torch

    pb = W.small2d(ckpt_every=6)
    g = torch.tensor(W.design(pb), dtype=torch.float64, device="cuda", requires_grad=True)
    J = L.LKSFunction.apply(g, pb, "fp64", W.initial_state(pb), W.initial_body(pb))
    (2.5 * J).backward()
    Jref, gref = orc.gradient(pb, W.design(pb), W.initial_state(pb), W.initial_body(pb), seed=2.5)
    assert abs(J.item() - Jref) <= 1e-9 * abs(Jref)
    assert rel(g.grad.cpu().numpy(), gref) < 1e-8
    assert elem(g.grad.cpu().numpy(), gref) < 1e-8


def test_empty_run_and_no_body(L, orc):
    pb = W.small2d(n_steps=0, ckpt_every=1)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    st, bd, J, _ = L.forward(pb, g, s0, b0, precision="fp64", store_ckpt=False)
    assert np.array_equal(st.cpu().numpy(), s0) and J.item() == 0.0
    pb = BODYFREE["2d-walls"]().replace(ckpt_every=4)
    s0 = smooth_state(pb, 1)
    st, bd, J, B = L.forward(pb, None, s0, np.zeros(12), precision="fp64")
    assert J.item() == 0.0


def test_divergence_is_reported(L):
    """A body pushed far beyond the footprint margin within one step -> LKS_EDIVERGED."""
    pb = W.small2d(mass=0.1, n_steps=3)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    with pytest.raises(L.LksError) as e:
        L.forward(pb, g, s0, b0, precision="fp64", store_ckpt=False)
    assert e.value.code == -4


# ------------------------------------------ terminal adjoint values (Sec. 3.4, warm start)

TERMINAL = ["small2d", "small2d-walls", "small3d"]


@pytest.mark.parametrize("march", [False, True], ids=["default", "alt"])
@pytest.mark.parametrize("case", TERMINAL)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_with_terminal_values(L, orc, case, prec, march):
    """lks_adjoint started from given cotangents of the final state and body matches the
    oracle's sweep of seed J + <dstate_T, state> + <dbody_T, body> (gradient and initial
    cotangents)."""
    pb = BODY[case]()
    fl = kernel_flags(L, pb, march)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    rng = np.random.default_rng(91)
    sT = rng.standard_normal(s0.size) * 0.05
    bT = np.zeros(12)
    bT[:8] = rng.standard_normal(8)
    seed = 0.8
    if prec == "fp32":
        sT = sT.astype(np.float32).astype(np.float64)
    J, gref, dsref, dbref = orc.gradient(pb, g, s0, b0, seed=seed, with_initial=True, dstate_T=sT, dbody_T=bT)
    _, _, Jg, B = L.forward(pb, g, s0, b0, precision=prec, flags=fl)
    gg, ds, db = L.adjoint(pb, g, B, seed=seed, precision=prec, want_initial=True, dstate_T=sT, dbody_T=bT,
                           flags=fl)
    tol = 1e-8 if prec == "fp64" else 1e-3
    assert rel(gg.cpu().numpy(), gref) < tol
    assert elem(gg.cpu().numpy(), gref) < tol
    assert rel(ds.cpu().numpy(), dsref) < tol
    assert elem(ds.cpu().numpy(), dsref) < tol
    assert np.abs(db.cpu().numpy()[:8] - dbref[:8]).max() <= tol * np.abs(dbref[:8]).max()


@pytest.mark.parametrize("case", ["small2d-rot", "small3d"])
def test_gradient_chains_over_split_runs(L, case):
    """Two lks_forward calls (the second from the first's final state and body) and two
    lks_adjoint calls (the first run's sweep starting from the second's initial
    cotangents) give the gradient of one run over all steps."""
    pb = BODY[case]().replace(n_steps=11, ckpt_every=3)
    n1 = 5
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    _, _, J, B = L.forward(pb, g, s0, b0, precision="fp64")
    grad, ds, db = L.adjoint(pb, g, B, seed=1.1, precision="fp64", want_initial=True)
    p1, p2 = pb.replace(n_steps=n1), pb.replace(n_steps=pb.n_steps - n1)
    s1, b1, J1, B1 = L.forward(p1, g, s0, b0, precision="fp64")
    _, _, J2, B2 = L.forward(p2, g, s1, b1, precision="fp64")
    g2, ds1, db1 = L.adjoint(p2, g, B2, seed=1.1, precision="fp64", want_initial=True)
    g1, ds0, db0 = L.adjoint(p1, g, B1, seed=1.1, precision="fp64", want_initial=True, dstate_T=ds1, dbody_T=db1)
    assert J1.item() + J2.item() == pytest.approx(J.item(), rel=1e-11, abs=1e-15)
    gr = grad.cpu().numpy()
    assert np.abs((g1 + g2).cpu().numpy() - gr).max() <= 1e-10 * np.abs(gr).max()
    assert np.abs(ds0.cpu().numpy() - ds.cpu().numpy()).max() <= 1e-10 * np.abs(ds.cpu().numpy()).max()
    dbr = db.cpu().numpy()[:8]
    assert np.abs(db0.cpu().numpy()[:8] - dbr).max() <= 1e-10 * np.abs(dbr).max()
