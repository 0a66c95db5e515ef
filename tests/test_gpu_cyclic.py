"""Parity of the cyclic periodic design (Sec. 4.2) through the C ABI with the oracle.

The expansion copies values: bit-exact in FP32 and FP64. The collection sums at most
four FP64 sensitivities per sector point; the library adds them in the group's order,
the oracle in design-index order, so they agree to 4 ulp of the summed magnitudes."""
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


def problem(dim, nd, axis=0):
    return W.small2d(nd=nd) if dim == 2 else W.small3d(nd=nd).replace(axis=axis)


CASES = [(2, (10, 8, 1), 0, 2), (2, (9, 9, 1), 0, 4), (2, (12, 12, 1), 0, 4), (2, (7, 5, 1), 0, 1),
         (2, (1, 1, 1), 0, 4), (3, (6, 5, 5), 0, 4), (3, (5, 7, 6), 1, 2), (3, (7, 7, 4), 2, 4),
         (3, (4, 9, 9), 0, 2),
         # full design grids of the 2D channel (128^2, 256^2) and the 3D duct (96^3, rotation about x)
         (2, (128, 128, 1), 0, 4), (2, (256, 256, 1), 0, 2), (3, (96, 96, 96), 0, 4)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_cyclic_expand_and_collect(L, orc, case):
    dim, nd, axis, n = CASES[case]
    pb = problem(dim, nd, axis)
    ns = orc.cyclic_sector_points(pb, n)
    assert L.cyclic_sector_points(pb, n) == ns
    rng = np.random.default_rng(300 + case)
    gs = rng.random(ns)
    grad = rng.standard_normal(int(np.prod(nd)))
    print(f"cyclic case {case} dim={dim} nd={nd} axis={axis} n={n}", flush=True)
    ref = orc.cyclic_expand(pb, n, gs)
    for prec in ("fp64", "fp32"):
        src = gs if prec == "fp64" else gs.astype(np.float32)
        got = L.design_cyclic_expand(pb, n, src, precision=prec).cpu().numpy()
        exp = ref if prec == "fp64" else ref.astype(np.float32)
        assert np.array_equal(got, exp)
    refc = orc.cyclic_collect(pb, n, grad)
    gotc = L.design_cyclic_collect(pb, n, grad).cpu().numpy()
    mag = orc.cyclic_collect(pb, n, np.abs(grad))
    assert np.all(np.abs(gotc - refc) <= 4 * np.finfo(np.float64).eps * mag)


@pytest.mark.parametrize("dim", [2, 3])
def test_cyclic_design_gradient_chain(L, orc, dim):
    """sector -> expand -> lks_forward / lks_adjoint -> collect, against the oracle's
    chain (FP64): the objective and the sector gradient."""
    pb = W.small2d(ckpt_every=4) if dim == 2 else W.small3d(ckpt_every=3)
    n = 2 if dim == 2 else 4
    rng = np.random.default_rng(17)
    gs = 0.2 + 0.6 * rng.random(orc.cyclic_sector_points(pb, n))
    s0, b0 = W.initial_state(pb), W.initial_body(pb)
    g_ref = orc.cyclic_expand(pb, n, gs)
    J_ref, grad_ref = orc.gradient(pb, g_ref, s0, b0)
    gsec_ref = orc.cyclic_collect(pb, n, grad_ref)
    g = L.design_cyclic_expand(pb, n, gs, precision="fp64")
    _, _, J, B = L.forward(pb, g, s0, b0, precision="fp64")
    gsec = L.design_cyclic_collect(pb, n, L.adjoint(pb, g, B, precision="fp64")).cpu().numpy()
    assert abs(J.item() - J_ref) <= 1e-9 * abs(J_ref) + 1e-15
    assert np.linalg.norm(gsec - gsec_ref) <= 1e-8 * np.linalg.norm(gsec_ref)
