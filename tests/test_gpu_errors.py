"""The error contract of the C ABI on the GPU, and the coupling constants against the oracle.

- lks_coupling (the constants K = -dF/du^G, K_theta = -dT/domega of the fluid <-> body
  iteration, Sec. 3.1) equals the oracle's finite-difference constants (FP64; the map
  is affine in the body velocity, so the oracle's unit step is exact up to rounding).
- LKS_FLAG_STABILITY makes lks_forward return LKS_EUNSTABLE (-3) before any step when
  an active degree of freedom has K/M >= 1 (the oracle pin
  test_unstable_coupling_diverges shows the iteration then blows up), and run normally
  below that.
- A fluid state that is not finite or faster than the lattice sound speed, and a
  design with a NaN, are reported as LKS_EDIVERGED (-4).
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


COUPLING = {
    "small2d": lambda: W.small2d(),
    "small2d-theta0": lambda: W.small2d(theta0=0.0),
    "small3d": lambda: W.small3d(),
    "small3d-axis1": lambda: W.small3d(axis=1, theta0=-0.7),
    "config2": lambda: W.config("config2"),
    "config5d": lambda: W.config("config5d"),
}


@pytest.mark.parametrize("case", sorted(COUPLING))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coupling_matches_oracle(L, orc, case, prec):
    pb = COUPLING[case]()
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    if prec == "fp32":  # the library forms kappa_ref from the design it is given
        g = g.astype(np.float32).astype(np.float64)
    Kref = orc.coupling(pb, g, s0, b0)
    K = L.coupling(pb, g, b0, precision=prec).cpu().numpy()
    print(f"{case} {prec}: K {K} oracle {Kref}", flush=True)
    for a in range(pb.dim):
        assert K[a] == pytest.approx(Kref[a], rel=1e-9)
    for a in range(pb.dim, 3):
        assert K[a] == 0.0 and Kref[a] == 0.0
    assert K[3] == pytest.approx(Kref[3], rel=1e-9)


@pytest.mark.parametrize("name", ["config2", "config5d", "config4"])
def test_configurations_sit_at_half_the_stability_limit(L, name):
    """Every configuration's kappa_max was chosen so that K = M/2 (the smallest margin
    over its active degrees of freedom) at t = 0; the GPU constants reproduce that."""
    pb = W.config(name)
    K = L.coupling(pb, W.design(pb), W.initial_body(pb), precision="fp32").cpu().numpy()
    ratios = [K[a] / pb.mass for a in range(pb.dim) if pb.dof_mask & (1 << a)]
    if pb.dof_mask & W.DOF_ROT:
        ratios.append(K[3] / pb.inertia)
    assert max(ratios) == pytest.approx(0.5, rel=1e-4)


def test_stability_precheck(L):
    """K/M >= 1 (translation) or K_theta/I >= 1 (rotation) with LKS_FLAG_STABILITY ->
    LKS_EUNSTABLE before any step; below the limit the run proceeds."""
    base = W.small2d(n_steps=4, theta0=0.0)
    g, s0, b0 = W.design(base), W.initial_state(base), W.initial_body(base)
    K = L.coupling(base, g, b0, precision="fp64").cpu().numpy()
    flag = L._lib.FLAG_STABILITY
    bad = [base.replace(mass=0.9 * K[0], dof_mask=W.DOF_TX),
           base.replace(mass=0.99 * K[1], dof_mask=W.DOF_TY),
           base.replace(inertia=0.8 * K[3], dof_mask=W.DOF_ROT)]
    for pb in bad:
        with pytest.raises(L.LksError) as e:
            L.forward(pb, g, s0, b0, precision="fp32", store_ckpt=False, flags=flag)
        assert e.value.code == L._lib.EUNSTABLE
    good = base.replace(mass=2.0 * K[0], inertia=2.0 * K[3])
    _, bd, J, _ = L.forward(good, g, s0, b0, precision="fp32", store_ckpt=False, flags=flag)
    assert np.isfinite(J.item())
    # an inactive degree of freedom is not checked
    _, _, J, _ = L.forward(base.replace(mass=0.5 * K[0], dof_mask=W.DOF_ROT, inertia=2.0 * K[3]), g, s0, b0,
                           precision="fp32", store_ckpt=False, flags=flag)
    assert np.isfinite(J.item())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fluid_divergence_is_reported(L, prec):
    """A fluid state faster than the lattice sound speed 1/sqrt(3), or with a non-finite
    value, is reported as LKS_EDIVERGED; a state just below that speed is not."""
    pb = W.Problem(dim=2, n=(20, 12, 1), bc=(0,) * 6, nu=0.1, n_steps=3)
    for u0, ok in ((0.6, False), (0.5, True)):
        p = pb.replace(u0=(u0, 0.1, 0.0))
        s0 = W.initial_state(p)  # uniform: a fixed point of the scheme at any speed
        assert (math.hypot(u0, 0.1) <= 1 / math.sqrt(3)) == ok
        if ok:
            L.forward(p, None, s0, np.zeros(12), precision=prec, store_ckpt=False)
        else:
            with pytest.raises(L.LksError) as e:
                L.forward(p, None, s0, np.zeros(12), precision=prec, store_ckpt=False)
            assert e.value.code == L._lib.EDIVERGED
    s0 = W.initial_state(pb.replace(u0=(0.05, 0.0, 0.0)))
    s0[pb.N + 7 * pb.n[0] + 9] = np.nan
    with pytest.raises(L.LksError) as e:
        L.forward(pb, None, s0, np.zeros(12), precision=prec, store_ckpt=False)
    assert e.value.code == L._lib.EDIVERGED
    # a 3D duct with checkpoints: the state is checked at every checkpoint
    p3 = W.duct3d(14, 9, 8, 0.04, 0.05, n_steps=7, ckpt_every=3)
    s3 = W.initial_state(p3)
    s3[3 * p3.N + 4 + p3.n[0] * (4 + p3.n[1] * 4)] = np.inf
    with pytest.raises(L.LksError) as e:
        L.forward(p3, None, s3, np.zeros(12), precision=prec)
    assert e.value.code == L._lib.EDIVERGED


def test_nan_design_is_reported(L):
    pb = W.small3d(n_steps=2)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    g[5] = np.nan
    with pytest.raises(L.LksError) as e:
        L.forward(pb, g, s0, b0, precision="fp32", store_ckpt=False)
    assert e.value.code == L._lib.EDIVERGED
