"""The paper's adjoint variant on the GPU (lks_adjoint with LKS_FLAG_PAPER_ADJOINT) against
the oracle's implementation of the same variant (orc_gradient_paper): the same
equations (ALKS, Eq. au, Eqs. axg..aomega iterated N_itr times, Eq. design_sensitivity),
so the FP64 path agrees to summation order (1e-8 relative L2 and entry-wise) and the FP32
path to the gradient target 1e-3. Cases with several checkpoint segments, 2D and 3D,
translation and rotation, a channel with walls."""
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
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def elem(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


WALLS2 = (W.VELOCITY, W.PRESSURE, W.WALL, W.WALL, 0, 0)
CASES = {
    "small2d": lambda: W.small2d(ckpt_every=5),
    "small2d-rot": lambda: W.small2d(objective=W.OBJ_ANGLE, inertia=300.0, ckpt_every=4, dof_mask=W.DOF_ROT),
    "shear-y": lambda: W.small2d(dof_mask=W.DOF_TY, objective=W.OBJ_DISP_Y, n_steps=20, ckpt_every=7,
                                 x_g0=(14.3, 8.6, 0.0), mass=20.0, kappa_max=2.0).replace(bc=WALLS2),
    "small3d": lambda: W.small3d(ckpt_every=4, inertia=150.0),
    "small3d-x": lambda: W.small3d(ckpt_every=3, dof_mask=W.DOF_TX, objective=W.OBJ_DISP_X, theta0=0.0),
    "small3d-y-axis2": lambda: W.small3d(ckpt_every=6, objective=W.OBJ_DISP_Y, axis=2),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_adjoint_matches_oracle(L, orc, case, prec):
    pb = CASES[case]()
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    Jref, gref = orc.gradient_paper(pb, g, s0, b0)
    B = L.Buffers(pb, prec, adjoint=True, paper=True)
    _, _, J, B = L.forward(pb, g, s0, b0, precision=prec, buffers=B)
    gg = L.adjoint_paper(pb, g, B, seed=1.3, precision=prec).cpu().numpy() / 1.3
    tol = 1e-8 if prec == "fp64" else 1e-3
    print(f"paper adjoint {case} {prec}: rel {rel(gg, gref):.2e} elem {elem(gg, gref):.2e}", flush=True)
    assert abs(J.item() - Jref) <= (1e-9 if prec == "fp64" else 1e-4) * abs(Jref)
    assert rel(gg, gref) < tol
    assert elem(gg, gref) < tol


def test_paper_adjoint_close_to_exact_on_gpu(L):
    """The two adjoints of the library on one problem: the paper's variant within its
    discretisation difference of the exact one (as the oracle shows)."""
    pb = W.small2d(ckpt_every=4)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    B = L.Buffers(pb, "fp64", adjoint=True, paper=True)
    _, _, _, B = L.forward(pb, g, s0, b0, precision="fp64", buffers=B)
    ge = L.adjoint(pb, g, B, precision="fp64").cpu().numpy()
    gp = L.adjoint_paper(pb, g, B, precision="fp64").cpu().numpy()
    assert rel(gp, ge) < 5e-3


def test_paper_adjoint_argument_checks(L):
    pb = W.small2d(ckpt_every=4, n_steps=4)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    B = L.Buffers(pb, "fp32", adjoint=True, paper=True)
    _, _, _, B = L.forward(pb, g, s0, b0, precision="fp32", buffers=B)
    with pytest.raises(L.LksError) as e:
        L.adjoint(pb, g, B, precision="fp32", flags=L._lib.FLAG_PAPER_ADJOINT, want_initial=True)
    assert e.value.code == L._lib.EINVAL
    # a workspace sized without the flag is too small for the variant
    B0 = L.Buffers(pb, "fp32", adjoint=True)
    _, _, _, B0 = L.forward(pb, g, s0, b0, precision="fp32", buffers=B0)
    with pytest.raises(L.LksError) as e:
        L.adjoint_paper(pb, g, B0, precision="fp32")
    assert e.value.code == L._lib.ENOSPACE
