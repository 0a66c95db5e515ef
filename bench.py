#!/usr/bin/env python3
"""Benchmark of the gfx950 library: forward + adjoint (design gradient) throughput.

One bench step = one full gradient of the workload: lks_forward over all N_t time
steps (with checkpoints) + lks_adjoint (segment recompute + reverse sweep). The
metric is MLUPS = analysis nodes x N_t / (forward + adjoint time) / 1e6, inputs
resident in HBM before the timed region. Also reported: FP32-vs-FP64 relative errors
of the objective and the gradient (FP64 run of the same workload, untimed), the FP64
speed, the LKS kernel against the HBM roofline (durations from kernel-stamped HIP
events on sampled time steps of the forward passes inside the timed region, where no
other work shares the GPU), and the FP64 CPU oracle on a bounded sample of the same
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config2]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "fwd+adjoint MLUPS, % HBM roofline; FP32 vs FP64 at stated rel. error"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_TFLOPS = 157.3
FP64_VECTOR_TFLOPS = 78.6

DESCRIPTIONS = {
    "config1": "2D D2Q9 128x64 channel, Re 20, body free in x (M 50), design 32x32, 1000 steps",
    "config2": "2D D2Q9 512x256 channel, Re 100, body rotating about a fixed pivot (I 1e4), "
               "design 128x128, 10000 steps, objective rotation angle",
    "config3": "2D D2Q9 1024x512 channel, Re 200, translating body, design 256x256, 20000 steps, "
               "checkpoints every 250",
    "config4": "3D D3Q15 128x64x64 duct, Re 100, 3-DOF translating body (M 500), design 48^3, "
               "5000 steps, checkpoints every 200",
    "config5": "3D D3Q15 256x128x128 duct, Re 300, body rotating about the duct axis + axial "
               "translation, design 96^3, 10000 steps, checkpoints every 500",
    "config5d": "3D D3Q15 64x32x32 duct (downscaled config5), design 24^3, 10000 steps",
}


# Kernels of the fluid <-> body iterations: per launch the method must read kappa_ref once
# per design point (4 B); the footprint fields they build and read stay in LDS / L2.
BODY_KERNELS = ("iter", "iter_final", "spread", "interp", "adj_recompute", "adj_r1", "adj_r2", "adj_r3")


def alg_bytes_per_launch(kernel, pb, elt):
    """Bytes the method must move per launch (each field read and written once)."""
    d, N = pb.dim, pb.N
    if kernel == "gather":        # read p, u; write p*, u*
        return 2 * (d + 1) * N * elt
    if kernel == "adj_gather":    # read pbar, ubar and forward u(t-1); write pbar, ubar
        return (3 * d + 2) * N * elt
    if kernel in BODY_KERNELS:    # kappa_ref, one read per design point
        return 4 * pb.ND
    return None


def gradient_bytes_per_node_step(dim, elt=4):
    """Algorithmic bytes of one gradient per node and time step: forward (read and write
    p, u), checkpoint recompute (the forward plus storing the state), adjoint (read pbar,
    ubar and forward u; write pbar, ubar): 92 B in 2D, 124 B in 3D (FP32)."""
    fwd = 2 * (dim + 1) * elt
    rec = fwd + (dim + 1) * elt
    adj = (3 * dim + 2) * elt
    return fwd + rec + adj


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def kernel_source_hash():
    """sha256 of the HIP sources: traffic counters taken on other sources are stale."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2601_18272_amd", "csrc")
    for name in sorted(os.listdir(src)):
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from profiles/traffic_<workload>.md (FETCH_SIZE and
    WRITE_SIZE runs, scaled by a copy kernel of known size), or None if absent or taken
    on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if blob.get("source_sha256") != kernel_source_hash():
        return None
    k = blob.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def launches_per_gradient(pb):
    NT, K = pb.n_steps, pb.n_itr
    # 2D: the forward pass forms the boundary values inside its LKS kernel and runs the
    # boundary launch only at checkpoints and at the end; the recompute after every step
    nbc = NT + NT // max(pb.ckpt_every, 1) + 1 if pb.dim == 2 else 2 * NT
    return {"gather": 2 * NT, "bc": nbc, "spread": 2 * K * NT, "interp": 2 * K * NT,
            "adj_gather": NT, "adj_recompute": NT, "adj_r1": K * NT, "adj_r2": K * NT,
            "adj_r3": K * NT, "iter": 2 * K * NT, "iter_final": 2 * NT}


def run_cpu_baseline(pb, sample_steps):
    import oracle
    import workloads as W

    # checkpoint interval no longer than the sample (the oracle stores every state; the
    # GPU's segment buffers are then sized for the sample, not for the full workload)
    spb = pb.replace(n_steps=sample_steps, ckpt_every=max(1, min(pb.ckpt_every, sample_steps)))
    g, s0, b0 = W.design(spb), W.initial_state(spb), W.initial_body(spb)
    t0 = time.perf_counter()
    J, grad = oracle.gradient(spb, g, s0, b0)
    dt = time.perf_counter() - t0
    return spb, J, grad, dt


def copy_bandwidth(mib=1024, reps=5):
    """GB/s of a plain elementwise device copy (read + write) of `mib` MiB."""
    import torch

    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * n * 4 / sec / 1e9


SWEEP = {
    2: [(512, 256), (1024, 512), (2048, 1024), (4096, 2048), (8192, 4096), (8192, 8192)],
    3: [(128, 64, 64), (256, 128, 128), (512, 256, 128), (512, 256, 256)],
}


def roofline_sweep(args):
    """Body-free gradients (forward with checkpoints + adjoint) of growing channels and
    ducts: the LKS and adjoint LKS kernels against the HBM roofline once the fields no
    longer fit the caches (8192 x 8192 2D and 512 x 256 x 256 3D move > 1 GB per
    launch)."""
    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    only = [tuple(int(v) for v in g.split("x")) for g in args.grids.split(",")] if args.grids else None
    for dim in (2, 3):
        for n in SWEEP[dim]:
            if only is None or tuple(n) in only:
                print(json.dumps(sweep_point(dim, n, args.steps)), flush=True)
    print(json.dumps({"sweep": "copy", "elementwise_copy_1GiB_GBs": round(copy_bandwidth(), 1)}), flush=True)


def sweep_point(dim, n, steps):
    """One body-free gradient size of the roofline sweep: the LKS and adjoint LKS kernels'
    live launch durations against their algorithmic bytes."""
    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    # one checkpoint segment: the adjoint's recompute then runs alone, not beside the
    # reverse sweep, so every sampled kernel has the GPU to itself
    if dim == 2:
        pb = W.channel2d(n[0], n[1], 0.05, 0.128, n_steps=16, ckpt_every=16, name=f"channel {n[0]}x{n[1]}")
    else:
        pb = W.duct3d(*n, 0.04, 0.01707, n_steps=8, ckpt_every=8, name="duct " + "x".join(map(str, n)))
    s0 = torch.tensor(W.initial_state(pb), dtype=torch.float32, device="cuda")
    b0 = torch.zeros(12, dtype=torch.float64, device="cuda")
    bufs = lks.Buffers(pb, "fp32", adjoint=True)

    def grad_step():
        _, _, _, B = lks.forward(pb, None, s0, b0, "fp32", buffers=bufs, flags=_lib.FLAG_PROFILE)
        lks.adjoint(pb, None, B, precision="fp32", flags=_lib.FLAG_PROFILE)

    grad_step()
    torch.cuda.synchronize()
    _lib.profile_reset()
    t0 = time.perf_counter()
    for _ in range(max(steps, 1)):
        grad_step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / max(steps, 1)
    prof = _lib.profile_read()
    _lib.profile_reset()
    line = {"sweep": "body-free roofline", "workload": pb.name, "dim": dim, "nodes": pb.N,
            "dtype": "f32", "gradient_MLUPS": round(pb.N * pb.n_steps / wall / 1e6, 1)}
    for k in ("gather", "adj_gather"):
        ms, cnt = prof[k]
        us = ms / cnt * 1e3
        by = alg_bytes_per_launch(k, pb, 4)
        line[k] = {"avg_launch_us": round(us, 2), "bytes_per_launch": by,
                   "achieved_GBs": round(by / us / 1e3, 1), "frac": round(by / us / 1e3 / HBM_PEAK_GBS, 4),
                   "samples": cnt}
        sms, scnt = prof.get(k + "_span", (0.0, 0))
        if scnt:
            sus = sms / scnt * 1e3
            line[k].update({"kernel_span_us": round(sus, 2), "achieved_GBs_span": round(by / sus / 1e3, 1)})
    del bufs, s0
    torch.cuda.empty_cache()
    return line


def config5_measure():
    """Config 5 in full: one 10000-step FP32 gradient (forward with checkpoints every 500 +
    adjoint), timed, with live kernel durations on sampled steps; then the FP64 gradient of
    the same workload (checkpoints every 250, untimed) for the FP32 errors per result."""
    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    pb = W.config("config5")
    g = torch.tensor(W.design(pb), dtype=torch.float32, device="cuda")
    s0 = torch.tensor(W.initial_state(pb), dtype=torch.float32, device="cuda")
    b0 = torch.tensor(W.initial_body(pb), dtype=torch.float64, device="cuda")
    bufs = lks.Buffers(pb, "fp32", adjoint=True)
    _lib.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st32, bd32, J32, B = lks.forward(pb, g, s0, b0, "fp32", buffers=bufs, flags=_lib.FLAG_PROFILE)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    prof_f = _lib.profile_read()
    _lib.profile_reset()
    grad32 = lks.adjoint(pb, g, B, precision="fp32", flags=_lib.FLAG_PROFILE)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof_a = _lib.profile_read()
    _lib.profile_reset()
    g32, bd32 = grad32.cpu().numpy(), bd32.cpu().numpy()
    del bufs, B, st32, grad32
    torch.cuda.empty_cache()
    print("# config5 fp32 gradient done", file=sys.stderr, flush=True)
    out = {"workload": "config5: " + DESCRIPTIONS["config5"], "nodes": pb.N, "n_steps": pb.n_steps,
           "gradient_s": round(wall, 3), "gradient_MLUPS": round(pb.N * pb.n_steps / wall / 1e6, 1),
           "forward_s": round(tf, 3), "forward_MLUPS": round(pb.N * pb.n_steps / tf / 1e6, 1)}
    avg = {}
    for src in (prof_a, prof_f):  # forward kernels at their forward-pass durations
        for k, (ms, n) in src.items():
            if n > 0:
                avg[k] = (ms, n)
    lp = launches_per_gradient(pb)
    est = {k: ms / n * lp[k] for k, (ms, n) in avg.items() if k in lp}
    dom = max(est, key=est.get)
    out["kernel_avg_us"] = {k: round(ms / n * 1e3, 3) for k, (ms, n) in avg.items()}
    out["share_of_gradient_est"] = {k: round(v / sum(est.values()), 3) for k, v in est.items()}
    for name in dict.fromkeys([dom, "gather", "adj_gather"]):
        by = alg_bytes_per_launch(name, pb, 4)
        ms, n = avg[name]
        us = ms / n * 1e3
        out[f"roofline_{name}"] = {"bound": "hbm", "bytes_per_launch": by, "avg_launch_us": round(us, 2),
                                   "achieved": round(by / us / 1e3, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(by / us / 1e3 / HBM_PEAK_GBS, 4),
                                   "traffic": measured_traffic("config5", name), "samples": n}
    out["dominant_kernel"] = dom
    gb = gradient_bytes_per_node_step(3) * pb.N * pb.n_steps
    out["gradient_pass"] = {"algorithmic_bytes": gb, "GBs": round(gb / wall / 1e9, 1),
                            "frac": round(gb / wall / 1e9 / HBM_PEAK_GBS, 4)}
    pb64 = pb.replace(ckpt_every=250)
    bufs64 = lks.Buffers(pb64, "fp64", adjoint=True)
    _, bd64, J64, B64 = lks.forward(pb64, g.double(), s0.double(), b0, "fp64", buffers=bufs64)
    g64 = lks.adjoint(pb64, g.double(), B64, precision="fp64").cpu().numpy()
    bd64 = bd64.cpu().numpy()
    del bufs64, B64
    torch.cuda.empty_cache()
    print("# config5 fp64 reference done", file=sys.stderr, flush=True)
    j32, j64 = J32.item(), J64.item()
    x0 = float(W.initial_body(pb)[0])
    out["fp32_vs_fp64"] = {
        "theta_J_fp32": j32, "theta_J_fp64": j64, "J_rel_err": abs(j32 - j64) / max(abs(j64), 1e-300),
        "x_displacement_fp32": float(bd32[0] - x0), "x_displacement_fp64": float(bd64[0] - x0),
        "x_displacement_rel_err": abs(bd32[0] - bd64[0]) / max(abs(bd64[0] - x0), 1e-300),
        "grad_rel_l2": float(np.linalg.norm(g32 - g64) / max(np.linalg.norm(g64), 1e-300)),
        "grad_max_rel": float(np.abs(g32 - g64).max() / max(np.abs(g64).max(), 1e-300))}
    return out


def paper_adjoint_measure(pb, g, s0, b0, grad_exact):
    """The paper's adjoint variant (LKS_FLAG_PAPER_ADJOINT) on the workload: one FP32
    gradient (forward with checkpoints + the variant's sweep), timed, and its relative L2
    difference from the exact adjoint's gradient of the timed run."""
    import torch

    import paper_2601_18272_amd as lks

    bufs = lks.Buffers(pb, "fp32", adjoint=True, paper=True)
    lks.forward(pb, g, s0, b0, "fp32", buffers=bufs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, B = lks.forward(pb, g, s0, b0, "fp32", buffers=bufs)
    gp = lks.adjoint_paper(pb, g, B, precision="fp32")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gp = gp.cpu().numpy()
    del bufs
    torch.cuda.empty_cache()
    return {"gradient_s": round(wall, 3), "gradient_MLUPS": round(pb.N * pb.n_steps / wall / 1e6, 1),
            "rel_l2_vs_exact_adjoint": float(np.linalg.norm(gp - grad_exact) / np.linalg.norm(grad_exact))}


def ball_taps(dim, R):
    """Design points within distance R of a point (the taps of the density filter)."""
    r = int(np.floor(R))
    ax = np.arange(-r, r + 1)
    if dim == 2:
        d2 = ax[:, None] ** 2 + ax[None, :] ** 2
    else:
        d2 = ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
    return int((np.sqrt(d2) <= R).sum())


def filter_measure(pb, reps=20):
    """Density filter + projection and its reverse on the workload's design grid (FP32
    forward, FP64 reverse), live kernel durations from HIP events (LKS_FLAG_PROFILE)."""
    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    R, beta, eta = W.FILTER_R, 8.0, W.FILTER_ETA
    nd = pb.nd
    ND = int(np.prod(nd))
    g = torch.tensor(W.raw_design(nd, pb.seed), dtype=torch.float32, device="cuda")
    gbh = torch.tensor(W.cotangent(ND, pb.seed + 1), dtype=torch.float64, device="cuda")
    work = torch.empty(lks.filter_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        gt, gh = lks.design_filter(pb, g, R, beta, eta, "fp32")
        lks.design_filter_adjoint(pb, gt, gbh, R, beta, eta, "fp32", work=work)
    torch.cuda.synchronize()
    _lib.profile_reset()
    for _ in range(reps):
        lks.design_filter(pb, g, R, beta, eta, "fp32", flags=_lib.FLAG_PROFILE)
        lks.design_filter_adjoint(pb, gt, gbh, R, beta, eta, "fp32", flags=_lib.FLAG_PROFILE, work=work)
    p = _lib.profile_read()
    _lib.profile_reset()
    taps = ball_taps(pb.dim, R)
    fwd_s = p["filter"][0] / p["filter"][1] / 1e3
    adj_s = p["filter_adj"][0] / p["filter_adj"][1] / 1e3
    flops = 2.0 * taps * ND  # one multiply-add per tap and point
    return {
        "design": list(nd[:pb.dim]), "radius": R, "beta": beta, "eta": eta, "taps": taps,
        "forward": {"kernel": "k_filter_tile (FP32)", "avg_launch_us": round(fwd_s * 1e6, 3),
                    "samples": p["filter"][1], "bound": "alu",
                    "achieved_TFLOPs": round(flops / fwd_s / 1e12, 3), "peak_TFLOPs": FP32_VECTOR_TFLOPS,
                    "frac": round(flops / fwd_s / 1e12 / FP32_VECTOR_TFLOPS, 4),
                    "hbm_GBs": round(3 * 4 * ND / fwd_s / 1e9, 1)},
        "reverse": {"kernels": "k_filter_scale + k_filter_tile (FP64), first begin to last end",
                    "avg_us": round(adj_s * 1e6, 3), "samples": p["filter_adj"][1], "bound": "alu",
                    "achieved_TFLOPs": round(flops / adj_s / 1e12, 3), "peak_TFLOPs": FP64_VECTOR_TFLOPS,
                    "frac": round(flops / adj_s / 1e12 / FP64_VECTOR_TFLOPS, 4),
                    "hbm_GBs": round((4 + 8 + 8) * ND / adj_s / 1e9, 1)},
    }


def mma_measure(pb, reps=20):
    """One MMA design update (FP64, iteration 3: asymptote history read) and the volume
    constraint on the workload's design grid, timed with HIP events on the stream the
    library's kernels run on (torch's current stream). Algorithmic bytes of the update per
    design variable: the prep pass reads x, x^(k-1), x^(k-2), L, U, df0, dg1 and writes L,
    U and 8 coefficients (17 x 8 B); each of the MMA_PASSES = 16 dual passes reads the 8
    coefficients (128 x 8 B); the final pass reads them and writes x (9 x 8 B)."""
    import torch

    import paper_2601_18272_amd as lks

    n = int(np.prod(pb.nd))
    rng = np.random.default_rng(pb.seed + 5)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    x = rng.uniform(0.05, 0.95, n)
    x1, x2 = np.clip(x + rng.normal(0, 0.05, n), 0, 1), np.clip(x + rng.normal(0, 0.05, n), 0, 1)
    args = dict(xold1=t(x1), xold2=t(x2), low=t(x - rng.uniform(0.1, 0.6, n)), upp=t(x + rng.uniform(0.1, 0.6, n)))
    xd, df0, dg1 = t(x), t(rng.normal(size=n) * 1e-3), t(np.full(n, -1.0 / (0.3 * n)))
    work = torch.empty(lks.mma_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    G, _ = lks.volume_constraint(xd, 0.3, work=work)
    for _ in range(3):
        lks.mma_update(xd, df0, G, dg1, 3, work=work, **args)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        lks.mma_update(xd, df0, G, dg1, 3, work=work, **args)
    ev[1].record()
    for _ in range(reps):
        lks.volume_constraint(xd, 0.3, work=work)
    ev[2].record()
    torch.cuda.synchronize()
    upd_us = ev[0].elapsed_time(ev[1]) / reps * 1e3
    vol_us = ev[1].elapsed_time(ev[2]) / reps * 1e3
    by = (17 + 16 * 8 + 9) * 8 * n
    vby = 2 * 8 * n
    return {"design_points": n,
            "update": {"kernels": "k_mma_prep, k_mma_r1, 16 x (k_mma_dual, k_mma_pick), k_mma_x",
                       "avg_us": round(upd_us, 2), "bytes": by, "GBs": round(by / upd_us / 1e3, 1),
                       "frac_hbm": round(by / upd_us / 1e3 / HBM_PEAK_GBS, 4)},
            "volume_constraint": {"avg_us": round(vol_us, 2), "bytes": vby, "GBs": round(vby / vol_us / 1e3, 1)}}


def cyclic_measure(pb, reps=20):
    """Cyclic periodic design on the workload's design grid (quarter turns when the
    rotation plane is square, else half turns): expansion (FP32) and collection (FP64),
    live kernel durations from HIP events (LKS_FLAG_PROFILE)."""
    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    a = pb.axis if pb.dim == 3 else 2
    n = 4 if pb.nd[(a + 1) % 3] == pb.nd[(a + 2) % 3] else 2
    ns = lks.cyclic_sector_points(pb, n)
    ND = int(np.prod(pb.nd))
    gs = torch.rand(ns, dtype=torch.float32, device="cuda")
    grad = torch.tensor(W.cotangent(ND, pb.seed + 2), dtype=torch.float64, device="cuda")
    for _ in range(3):
        lks.design_cyclic_expand(pb, n, gs, "fp32")
        lks.design_cyclic_collect(pb, n, grad)
    torch.cuda.synchronize()
    _lib.profile_reset()
    for _ in range(reps):
        lks.design_cyclic_expand(pb, n, gs, "fp32", flags=_lib.FLAG_PROFILE)
        lks.design_cyclic_collect(pb, n, grad, flags=_lib.FLAG_PROFILE)
    p = _lib.profile_read()
    _lib.profile_reset()
    out = {"sectors": n, "sector_points": ns, "design_points": ND}
    for name, key, by in (("expand", "cyc_expand", 4 * (ns + ND)), ("collect", "cyc_collect", 8 * (ND + ns))):
        us = p[key][0] / p[key][1] * 1e3
        out[name] = {"avg_launch_us": round(us, 3), "samples": p[key][1], "bound": "hbm", "bytes": by,
                     "GBs": round(by / us / 1e3, 1), "frac": round(by / us / 1e3 / HBM_PEAK_GBS, 4)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--n-steps", type=int, default=None, help="override the workload's time steps")
    ap.add_argument("--cpu-steps", type=int, default=40, help="time steps of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="body-free roofline sweep of the LKS and adjoint LKS kernels over grid sizes "
                         "up to > 1 GB per step (one JSON line per size instead of the headline)")
    ap.add_argument("--grids", default=None,
                    help="with --sweep: only these grids of the sweep, comma-separated (e.g. 8192x8192,512x256x256)")
    ap.add_argument("--only-gradient", action="store_true",
                    help="time the gradient steps only (no extra measurements, no FP64 or CPU runs): "
                         "for profiler runs")
    ap.add_argument("--no-config5", action="store_true", help="skip the full config 5 gradient in extra")
    ap.add_argument("--no-sweep-points", action="store_true", help="skip the largest sweep points in extra")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.only_gradient:
        args.no_cpu = args.no_fp64 = args.no_config5 = args.no_sweep_points = True
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the grid would be "
              "cut into x-slabs, one per GPU, with a two-layer halo exchange per step and a "
              "force/torque allreduce per fluid-body iteration)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2601_18272_amd as lks
    import workloads as W
    from paper_2601_18272_amd import _lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.sweep:
        roofline_sweep(args)
        return
    pb = W.config(args.workload)
    if args.n_steps:
        pb = pb.replace(n_steps=args.n_steps)
    if pb.ckpt_every < 1:
        pb = pb.replace(ckpt_every=250)
    elt = 4
    g = torch.tensor(W.design(pb), dtype=torch.float32, device="cuda")
    s0 = torch.tensor(W.initial_state(pb), dtype=torch.float32, device="cuda")
    b0 = torch.tensor(W.initial_body(pb), dtype=torch.float64, device="cuda")
    bufs = lks.Buffers(pb, "fp32", adjoint=True)
    flags = _lib.FLAG_PROFILE

    # Live kernel timing, kept apart for the two passes: in the forward pass nothing runs
    # beside the sampled kernels; in the adjoint pass the recompute of the next segment
    # (second stream) shares the GPU with the reverse sweep.
    prof_f, prof_a = {}, {}

    def collect(dst):
        for k, (ms, n) in _lib.profile_read().items():
            a = dst.get(k, (0.0, 0))
            dst[k] = (a[0] + ms, a[1] + n)
        _lib.profile_reset()

    def gradient_step(record=True):
        _, _, J, B = lks.forward(pb, g, s0, b0, "fp32", buffers=bufs, flags=flags)
        if record:
            collect(prof_f)
        grad = lks.adjoint(pb, g, B, precision="fp32", flags=flags)
        if record:
            collect(prof_a)
        return J, grad

    print(f"# workload {pb.name}: {DESCRIPTIONS.get(pb.name, '')}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        gradient_step(record=False)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    _lib.profile_reset()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        J32, grad32 = gradient_step()
        print(f"# step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / args.steps
    node_steps = pb.N * pb.n_steps
    value = node_steps * args.steps / wall / 1e6
    avg_f = {k: ms / n for k, (ms, n) in prof_f.items() if n > 0}
    avg_a = {k: ms / n for k, (ms, n) in prof_a.items() if n > 0}
    # forward kernels at their forward-pass durations (the recompute overlaps the sweep)
    prof = {k: v for k, v in prof_a.items() if v[1] > 0}
    prof.update({k: v for k, v in prof_f.items() if v[1] > 0})

    # dominant kernel: largest estimated share of the gradient (sampled avg x launches)
    lp = launches_per_gradient(pb)
    est = {k: (ms / n) * lp[k] for k, (ms, n) in prof.items() if n > 0 and k in lp}
    dom = max(est, key=est.get)

    def roofline_of(name):
        by = alg_bytes_per_launch(name, pb, elt)
        ms, n = prof[name]
        avg_s = ms / n / 1e3
        ach = by / avg_s / 1e9
        r = {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 6),
             "traffic": measured_traffic(pb.name, name),
             "bytes_per_launch": by, "avg_launch_us": round(avg_s * 1e6, 3), "samples": n}
        span = prof.get(name + "_span")
        if span and span[1] > 0:
            span_s = span[0] / span[1] / 1e3
            r["kernel_span_us"] = round(span_s * 1e6, 3)
            r["achieved_kernel_span"] = round(by / span_s / 1e9, 1)
        return r

    # the dominant kernel (largest estimated share of the gradient) against the HBM
    # roofline with its algorithmic bytes; the LKS kernel beside it
    roof = roofline_of(dom)
    roof["dominant_kernel"] = dom
    roof["share_of_gradient_est"] = {k: round(v / sum(est.values()), 3) for k, v in est.items()}
    gb = gradient_bytes_per_node_step(pb.dim) * pb.N * pb.n_steps
    roof["gradient_pass"] = {"algorithmic_bytes_per_node_step": gradient_bytes_per_node_step(pb.dim),
                             "GBs": round(gb / (wall / args.steps) / 1e9, 1),
                             "frac": round(gb / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4)}
    roof_lks = roofline_of("gather") if "gather" in prof else None

    if args.calibrate_copy:
        n = 64 * 1024 * 1024
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.mul(src, 1.0, out=dst)  # one elementwise pass: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        del src, dst
        print("# calibration copy done (2 x 256 MiB)", file=sys.stderr, flush=True)

    extra = {"ms_per_step_gpu_events": round(gpu_ms / args.steps, 3), "roofline_lks_kernel": roof_lks,
             "kernel_avg_us": {"forward_pass": {k: round(v * 1e3, 3) for k, v in avg_f.items()},
                               "adjoint_pass": {k: round(v * 1e3, 3) for k, v in avg_a.items()}}}

    if args.only_gradient:
        print(json.dumps({"metric": METRIC, "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
                          "workload": pb.name, "roofline": roof, "extra": extra}), flush=True)
        return

    # forward pass alone (with its checkpoints), outside the timed region
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lks.forward(pb, g, s0, b0, "fp32", buffers=bufs)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t1
    extra["forward_only"] = {"ms": round(tf * 1e3, 2), "MLUPS": round(pb.N * pb.n_steps / tf / 1e6, 2)}
    extra["copy_GBs_elementwise_1GiB"] = round(copy_bandwidth(), 1)
    extra["design_filter"] = filter_measure(pb)
    extra["cyclic_design"] = cyclic_measure(pb)
    extra["mma_update"] = mma_measure(pb)
    print("# design filter, cyclic design and MMA update done", file=sys.stderr, flush=True)
    extra["paper_adjoint"] = paper_adjoint_measure(pb, g, s0, b0, grad32.cpu().numpy())
    print("# paper's adjoint variant done", file=sys.stderr, flush=True)

    if not args.no_fp64:
        bufs64 = lks.Buffers(pb, "fp64", adjoint=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, J64, B64 = lks.forward(pb, g.double(), s0.double(), b0, "fp64", buffers=bufs64)
        grad64 = lks.adjoint(pb, g.double(), B64, precision="fp64")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        j32, j64 = J32.item(), J64.item()
        g32, g64 = grad32.cpu().numpy(), grad64.cpu().numpy()
        extra["fp32_vs_fp64"] = {
            "J_fp32": j32, "J_fp64": j64, "J_rel_err": abs(j32 - j64) / max(abs(j64), 1e-300),
            "grad_rel_l2": float(np.linalg.norm(g32 - g64) / max(np.linalg.norm(g64), 1e-300)),
            "fp64_ms_per_step": round(t64 * 1e3, 1),
            "speedup_fp32_over_fp64": round(t64 / (wall / args.steps), 3)}
        del bufs64
        print("# fp64 reference done", file=sys.stderr, flush=True)

    del bufs
    torch.cuda.empty_cache()
    if not args.no_config5:
        extra["config5"] = config5_measure()
    if not args.no_sweep_points:
        extra["sweep_largest"] = [sweep_point(2, SWEEP[2][-1], 2), sweep_point(3, SWEEP[3][-1], 2)]
        print("# largest sweep points done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        spb, Jo, go, dt = run_cpu_baseline(pb, args.cpu_steps)
        model, ncpu = cpu_info()
        cpu = {"value": round(spb.N * spb.n_steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
               "kind": "oracle",
               "sample": f"{pb.name} truncated to its first {spb.n_steps} time steps "
                         f"(forward + exact adjoint, serial FP64, {dt:.1f} s, one core of {ncpu} x {model})",
               "cpu_model": model, "nproc": ncpu}
        # parity of the GPU FP32 path on the same full-grid sample
        sb = lks.Buffers(spb, "fp32", adjoint=True)
        _, _, Js, Bs = lks.forward(spb, g, s0, b0, "fp32", buffers=sb)
        gs = lks.adjoint(spb, g, Bs, precision="fp32").cpu().numpy()
        extra["oracle_parity_sample"] = {
            "n_steps": spb.n_steps, "J_rel_err_fp32": abs(Js.item() - Jo) / max(abs(Jo), 1e-300),
            "grad_rel_l2_fp32": float(np.linalg.norm(gs - go) / max(np.linalg.norm(go), 1e-300))}
        print("# cpu baseline done", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{pb.name}: {DESCRIPTIONS.get(pb.name, '')}", "grid": list(pb.n[:pb.dim]),
                   "design": list(pb.nd[:pb.dim]), "n_steps": pb.n_steps, "n_itr": pb.n_itr,
                   "ckpt_every": pb.ckpt_every, "pass": "forward + adjoint (gradient)"},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
