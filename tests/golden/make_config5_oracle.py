"""Writes config5_oracle_3steps.json: the FP64 oracle's objective and sampled gradient
entries for the 256x128x128 duct of config 5 (96^3 design, rotation about x plus axial
translation) truncated to 3 time steps with checkpoints every 2.

The oracle needs several minutes for this run, longer than a GPU test may take, so the
values are computed once on the CPU by this script (which calls only oracle/ and the
seeded generators of workloads.py) and the GPU test compares its own run with them:
the objective, the final body state, the gradient's L2 norm, and 64 gradient entries
(the 16 largest in magnitude and 48 drawn with default_rng(1003)).

Run: python tests/golden/make_config5_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "config5_oracle_3steps.json")


def main():
    pb = W.config("config5").replace(n_steps=3, ckpt_every=2)
    g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
    t = time.time()
    J, grad = oracle.gradient(pb, g, s0, b0)
    _, body, J2 = oracle.forward(pb, g, s0, b0)
    assert J2 == J
    top = np.argsort(-np.abs(grad))[:16]
    rng = np.random.default_rng(1003)
    rest = rng.choice(pb.ND, 48, replace=False)
    idx = [int(i) for i in np.concatenate([top, rest])]
    rec = {
        "workload": "config5 truncated: n_steps 3, ckpt_every 2 (FP64 oracle)",
        "n_steps": 3,
        "ckpt_every": 2,
        "J": J,
        "body": [float(v) for v in body[:8]],
        "grad_l2": float(np.linalg.norm(grad)),
        "grad_max": float(np.abs(grad).max()),
        "idx": idx,
        "grad": [float(grad[i]) for i in idx],
        "oracle_seconds": round(time.time() - t, 1),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT, "J =", J, "in", rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
