"""TEST INFRASTRUCTURE. The two adjoints against central differences along a line of
design entries, the comparison the paper makes in App. B (its figures, with the
geometry, are not part of its text): a translating body (objective: displacement,
Eq. objective1) and a rotating one (objective: angle, Eq. objective2) in a channel.

For each design entry on the middle row of the design grid: FD (central, FP64,
h = 1e-5 on gamma), ADJ(exact) (orc_gradient, the exact reverse of the discrete map)
and ADJ(paper) (orc_gradient_paper, the paper's continuous adjoint discretised), all
from the oracle. Prints markdown tables.

Run: python oracle/compare_adjoints.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CASES = {
    "translation (x, objective x^G displacement, 40 steps)": W.small2d(dof_mask=W.DOF_TX, theta0=0.0, n_steps=40),
    "rotation (fixed pivot, objective theta, 40 steps)": W.small2d(dof_mask=W.DOF_ROT, objective=W.OBJ_ANGLE,
                                                                   inertia=300.0, theta0=0.0, n_steps=40),
}


def main():
    oracle.lib()
    h = 1e-5
    for name, pb in CASES.items():
        g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
        J, ge = oracle.gradient(pb, g, s0, b0)
        _, gp = oracle.gradient_paper(pb, g, s0, b0)
        j = pb.nd[1] // 2
        print(f"\n{name}: J = {J:.6e}; whole design: |paper - exact| / |exact| = "
              f"{np.linalg.norm(gp - ge) / np.linalg.norm(ge):.2e} (relative L2)\n")
        print("| i | FD | ADJ (exact) | ADJ (paper) | exact vs FD | paper vs FD |")
        print("|---|---|---|---|---|---|")
        for i in range(pb.nd[0]):
            m = i + pb.nd[0] * j
            gpl, gm = g.copy(), g.copy()
            gpl[m] += h
            gm[m] -= h
            fd = (oracle.forward(pb, gpl, s0, b0)[2] - oracle.forward(pb, gm, s0, b0)[2]) / (2 * h)
            print(f"| {i} | {fd:.6e} | {ge[m]:.6e} | {gp[m]:.6e} | {abs(ge[m] - fd) / abs(fd):.1e} | "
                  f"{abs(gp[m] - fd) / abs(fd):.1e} |")


if __name__ == "__main__":
    main()
