"""Choose kappa_max (and config 3's mass) from the oracle's coupling constants.

TEST INFRASTRUCTURE: calls only the oracle. Prints the values stored in
``workloads.KAPPA`` / ``workloads.MASS3``.

Within a step, each fluid <-> body iteration restarts from the body state at t-1,
so an error e in the body velocity maps to -(K/M) e, where K is minus the slope of
the force with respect to the body velocity (orc_coupling). The iteration contracts
only if K/M < 1. For each configuration kappa_max is chosen so that
max over the free degrees of freedom of K/M (K/I for rotation) equals 1/2 at t = 0.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
import workloads as W  # noqa: E402


def ratio(pb):
    K = oracle.coupling(pb, W.design(pb), W.initial_state(pb), W.initial_body(pb))
    r = []
    for a in range(3):
        if pb.dof_mask & (1 << a):
            r.append(K[a] / pb.mass)
    if pb.dof_mask & W.DOF_ROT:
        r.append(K[3] / pb.inertia)
    return max(r), K


def solve(pb, target=0.5):
    k0 = 1e-3
    r0, _ = ratio(pb.replace(kappa_max=k0))
    k1 = k0 * target / r0
    for _ in range(6):
        r1, _ = ratio(pb.replace(kappa_max=k1))
        if abs(r1 - target) < 1e-4 * target:
            break
        k0, r0, k1 = k1, r1, k1 + (target - r1) * (k1 - k0) / (r1 - r0)
    return k1


if __name__ == "__main__":
    names = sys.argv[1:] or ["config1", "config2", "config4", "config5d", "config5", "config3"]
    for name in names:
        pb = W.config(name)
        if name == "config3":
            r, K = ratio(pb)
            print(f"{name}: kappa_max=300 K={K} -> mass = 2K = {2 * K[0]:.6g}")
            continue
        k = solve(pb)
        r, K = ratio(pb.replace(kappa_max=k))
        print(f"{name}: kappa_max = {k:.6g}  (K/M = {r:.4f}, K = {K})", flush=True)
