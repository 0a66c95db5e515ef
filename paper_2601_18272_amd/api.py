"""Python binding of the gfx950 library: argument marshalling only.

Every step of the computation runs in the HIP kernels of liblks_hip.so; torch supplies
device memory and the current stream. Problems are described by any object with the
fields of ``workloads.Problem`` (dim, n, bc, bc_p, bc_u, nu, nd, kappa_max, q, mass,
inertia, axis, dof_mask, n_itr, n_steps, ckpt_every, objective).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import LksError, LksFilter, LksProblem  # noqa: F401

DTYPES = {"fp32": torch.float32, "fp64": torch.float64}


def problem_struct(pb, precision: str = "fp32", flags: int = 0) -> LksProblem:
    s = LksProblem()
    s.dim = int(pb.dim)
    for a in range(3):
        s.n[a] = int(pb.n[a])
        s.nd[a] = int(pb.nd[a])
    for f in range(6):
        s.bc[f] = int(pb.bc[f])
        s.bc_p[f] = float(pb.bc_p[f])
        for a in range(3):
            s.bc_u[f][a] = float(pb.bc_u[f][a])
    s.nu = float(pb.nu)
    s.kappa_max = float(pb.kappa_max)
    s.q = float(pb.q)
    s.mass = float(pb.mass)
    s.inertia = float(pb.inertia)
    s.axis = int(pb.axis)
    s.dof_mask = int(pb.dof_mask)
    s.n_itr = int(pb.n_itr)
    s.n_steps = int(pb.n_steps)
    s.ckpt_every = int(pb.ckpt_every)
    s.precision = _lib.FP32 if precision == "fp32" else _lib.FP64
    s.objective = int(pb.objective)
    s.flags = int(flags)
    return s


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype):
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(x, dtype=dtype, device="cuda").contiguous()


def state_elems(pb) -> int:
    return int(_lib.load().lks_state_elems(C.byref(problem_struct(pb))))


def checkpoint_bytes(pb, precision="fp32") -> int:
    return int(_lib.load().lks_checkpoint_bytes(C.byref(problem_struct(pb, precision))))


def workspace_bytes(pb, adjoint: bool, precision="fp32") -> int:
    return int(_lib.load().lks_workspace_bytes(C.byref(problem_struct(pb, precision)), int(adjoint)))


class Buffers:
    """Device buffers for repeated calls on one problem (no allocation per call)."""

    def __init__(self, pb, precision="fp32", adjoint=True, paper=False):
        L = _lib.load()
        self.pb = pb
        self.precision = precision
        self.dtype = DTYPES[precision]
        # paper: size the adjoint workspace for the paper's adjoint variant as well
        self.s = problem_struct(pb, precision, _lib.FLAG_PAPER_ADJOINT if paper else 0)
        nbytes = int(L.lks_workspace_bytes(C.byref(self.s), int(adjoint)))
        if nbytes == 0:
            raise LksError(_lib.EINVAL, L.lks_last_error().decode())
        self.work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ckpt = None
        if adjoint:
            cb = int(L.lks_checkpoint_bytes(C.byref(self.s)))
            self.ckpt = torch.empty(cb, dtype=torch.uint8, device="cuda")
        self.J = torch.zeros(1, dtype=torch.float64, device="cuda")


def forward(pb, gamma, state0, body0, precision="fp32", buffers: Buffers | None = None,
            store_ckpt: bool = True, flags: int = 0):
    """Run pb.n_steps coupled steps. Returns (state, body, J, buffers)."""
    L = _lib.load()
    dt = DTYPES[precision]
    B = buffers or Buffers(pb, precision, adjoint=store_ckpt)
    s = problem_struct(pb, precision, flags)
    g = _dev(gamma, dt) if gamma is not None else None
    st = _dev(state0, dt).clone()
    bd = _dev(body0, torch.float64).clone()
    ck = B.ckpt if store_ckpt else None
    _lib.check(L.lks_forward(C.byref(s), _p(g), _p(st), _p(bd), _p(ck),
                             ck.numel() if ck is not None else 0, _p(B.work), B.work.numel(),
                             _p(B.J), _stream()))
    return st, bd, B.J.clone(), B


def adjoint(pb, gamma, buffers: Buffers, seed: float = 1.0, precision="fp32",
            want_initial: bool = False, flags: int = 0, dstate_T=None, dbody_T=None):
    """Reverse sweep after forward(..., store_ckpt=True) of seed * J plus, optionally,
    <dstate_T, final state> + <dbody_T, final body> (terminal adjoint values). Returns
    grad (float64) and, with want_initial, the cotangents of the initial state and body."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision, flags)
    g = _dev(gamma, dt) if gamma is not None else None
    sT = _dev(dstate_T, dt) if dstate_T is not None else None
    bT = _dev(dbody_T, torch.float64) if dbody_T is not None else None
    if sT is not None and sT.numel() != state_elems(pb):
        raise ValueError("dstate_T must have the size of a state")
    if bT is not None and bT.numel() < 8:
        raise ValueError("dbody_T needs at least 8 entries")
    grad = torch.empty(max(int(pb.nd[0] * pb.nd[1] * pb.nd[2]), 1), dtype=torch.float64, device="cuda")
    ds = torch.empty(state_elems(pb), dtype=dt, device="cuda") if want_initial else None
    db = torch.empty(12, dtype=torch.float64, device="cuda") if want_initial else None
    _lib.check(L.lks_adjoint(C.byref(s), _p(g), _p(buffers.ckpt), buffers.ckpt.numel(),
                             _p(buffers.work), buffers.work.numel(), float(seed), _p(sT), _p(bT), _p(grad),
                             _p(ds), _p(db), _stream()))
    return (grad, ds, db) if want_initial else grad


def coupling(pb, gamma, body, precision="fp32"):
    """Coupling constants K[0..2] = -dF/du^G and K[3] = -dT/domega of the fluid <-> body
    iteration at the pose `body` (float64 tensor of 4)."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision)
    nbytes = int(L.lks_workspace_bytes(C.byref(s), 0))
    if nbytes == 0:
        raise LksError(_lib.EINVAL, L.lks_last_error().decode())
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    g = _dev(gamma, dt)
    bd = _dev(body, torch.float64)
    K = torch.empty(4, dtype=torch.float64, device="cuda")
    _lib.check(L.lks_coupling(C.byref(s), _p(g), _p(bd), _p(K), _p(work), work.numel(), _stream()))
    return K


def adjoint_paper(pb, gamma, buffers: Buffers, seed: float = 1.0, precision="fp32", flags: int = 0):
    """The paper's adjoint variant (Sec. 2.5) after forward(..., store_ckpt=True) with
    Buffers(..., paper=True): an approximation of dJ/dgamma (float64)."""
    return adjoint(pb, gamma, buffers, seed=seed, precision=precision, flags=flags | _lib.FLAG_PAPER_ADJOINT)


def map_design(pb, kappa_ref, body, precision="fp32"):
    """Mapped Brinkman coefficient and body velocity on the analysis grid."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision)
    kr = _dev(kappa_ref, dt)
    bd = _dev(body, torch.float64)
    N = int(pb.n[0] * pb.n[1] * pb.n[2])
    kap = torch.empty(N, dtype=dt, device="cuda")
    uS = torch.empty(pb.dim * N, dtype=dt, device="cuda")
    _lib.check(L.map_design(C.byref(s), _p(kr), _p(bd), _p(kap), _p(uS), _stream()))
    return kap, uS


def body_step(pb, ft, body_prev):
    """Euler update of the body from a force/torque [F_x, F_y, F_z, T]."""
    L = _lib.load()
    s = problem_struct(pb)
    f = _dev(ft, torch.float64)
    bp = _dev(body_prev, torch.float64)
    out = torch.empty(12, dtype=torch.float64, device="cuda")
    _lib.check(L.body_step(C.byref(s), _p(f), _p(bp), _p(out), _stream()))
    return out


def filter_struct(radius: float, beta: float, eta: float = 0.5) -> LksFilter:
    f = LksFilter()
    f.radius, f.beta, f.eta = float(radius), float(beta), float(eta)
    return f


def design_filter(pb, gamma, radius, beta, eta=0.5, precision="fp32", flags: int = 0):
    """Filtered and projected design (gamma_tilde, gamma_hat) on pb's design grid."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision, flags)
    g = _dev(gamma, dt).reshape(-1)
    gt = torch.empty_like(g)
    gh = torch.empty_like(g)
    f = filter_struct(radius, beta, eta)
    _lib.check(L.lks_design_filter(C.byref(s), C.byref(f), _p(g), _p(gt), _p(gh), _stream()))
    return gt, gh


def filter_workspace_bytes(pb) -> int:
    return int(_lib.load().lks_filter_workspace_bytes(C.byref(problem_struct(pb))))


def design_filter_adjoint(pb, gamma_tilde, dJ_dgamma_hat, radius, beta, eta=0.5, precision="fp32",
                          flags: int = 0, work=None):
    """dJ/dgamma (FP64) from dJ/dgamma_hat through the projection and the filter. `work`
    (optional) is a uint8 device tensor of filter_workspace_bytes(pb) bytes."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision, flags)
    gt = _dev(gamma_tilde, dt).reshape(-1)
    gbh = _dev(dJ_dgamma_hat, torch.float64).reshape(-1)
    gb = torch.empty_like(gbh)
    if work is None:
        nbytes = int(L.lks_filter_workspace_bytes(C.byref(s)))
        if nbytes == 0:
            raise LksError(_lib.EINVAL, L.lks_last_error().decode())
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    f = filter_struct(radius, beta, eta)
    _lib.check(L.lks_design_filter_adjoint(C.byref(s), C.byref(f), _p(gt), _p(gbh), _p(work), work.numel(),
                                           _p(gb), _stream()))
    return gb


def cyclic_sector_points(pb, n_sectors: int) -> int:
    return int(_lib.load().lks_cyclic_sector_points(C.byref(problem_struct(pb)), int(n_sectors)))


def design_cyclic_expand(pb, n_sectors: int, gamma_sector, precision="fp32", flags: int = 0):
    """Sector design -> design grid (cyclic periodic design)."""
    L = _lib.load()
    dt = DTYPES[precision]
    s = problem_struct(pb, precision, flags)
    gs = _dev(gamma_sector, dt).reshape(-1)
    g = torch.empty(int(pb.nd[0] * pb.nd[1] * pb.nd[2]), dtype=dt, device="cuda")
    _lib.check(L.lks_design_cyclic_expand(C.byref(s), int(n_sectors), _p(gs), _p(g), _stream()))
    return g


def design_cyclic_collect(pb, n_sectors: int, grad, flags: int = 0):
    """Design-grid sensitivities (FP64) -> sector (transpose of the expansion)."""
    L = _lib.load()
    s = problem_struct(pb, "fp32", flags)
    gr = _dev(grad, torch.float64).reshape(-1)
    n = int(L.lks_cyclic_sector_points(C.byref(s), int(n_sectors)))
    if n == 0:
        raise LksError(_lib.EINVAL, L.lks_last_error().decode())
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    _lib.check(L.lks_design_cyclic_collect(C.byref(s), int(n_sectors), _p(gr), _p(out), _stream()))
    return out


def mma_workspace_bytes(n: int) -> int:
    return int(_lib.load().lks_mma_workspace_bytes(int(n)))


def mma_update(x, df0, g1, dg1, it: int, xold1=None, xold2=None, low=None, upp=None, xmin: float = 0.0,
               xmax: float = 1.0, move: float = 0.2, work=None, f0_scale: float = 1.0):
    """One MMA step (FP64, on the device) minimising the function whose gradient is
    f0_scale * df0: returns (x_new, low, upp, lambda). x, df0, dg1 are design arrays, g1 the
    constraint value (a 1-element device tensor or a float); pass the previous asymptotes
    low, upp and x^(k-1), x^(k-2) from iteration 3 on."""
    L = _lib.load()
    xd = _dev(x, torch.float64).reshape(-1).clone()
    n = xd.numel()
    f0 = _dev(df0, torch.float64).reshape(-1)
    f1 = _dev(dg1, torch.float64).reshape(-1)
    if not torch.is_tensor(g1):
        g1 = torch.tensor([float(g1)], dtype=torch.float64)
    g = _dev(g1, torch.float64).reshape(-1)
    lo = _dev(low, torch.float64).reshape(-1).clone() if low is not None else torch.zeros(n, dtype=torch.float64,
                                                                                           device="cuda")
    up = _dev(upp, torch.float64).reshape(-1).clone() if upp is not None else torch.zeros(n, dtype=torch.float64,
                                                                                           device="cuda")
    x1 = _dev(xold1, torch.float64).reshape(-1) if xold1 is not None else None
    x2 = _dev(xold2, torch.float64).reshape(-1) if xold2 is not None else None
    lam = torch.zeros(1, dtype=torch.float64, device="cuda")
    nbytes = mma_workspace_bytes(n)
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    opt = _lib.LksMma(float(xmin), float(xmax), float(move), float(f0_scale))
    _lib.check(L.lks_mma_update(C.byref(opt), n, int(it), _p(xd), _p(x1), _p(x2), _p(lo), _p(up), _p(f0), _p(g),
                                _p(f1), _p(lam), _p(work), work.numel(), _stream()))
    return xd, lo, up, lam


def volume_constraint(gh, vmin: float, work=None):
    """G = 1 - sum(gh) / (vmin n) and dG/dgh on the device (FP64)."""
    L = _lib.load()
    g = _dev(gh, torch.float64).reshape(-1)
    n = g.numel()
    G = torch.zeros(1, dtype=torch.float64, device="cuda")
    dG = torch.empty(n, dtype=torch.float64, device="cuda")
    if work is None:
        work = torch.empty(mma_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    _lib.check(L.lks_volume_constraint(n, _p(g), float(vmin), _p(G), _p(dG), _p(work), work.numel(), _stream()))
    return G, dG


def optimize(pb, gamma0, state0, body0, vmin: float, radius: float, betas, qs=None, n_opt: int = 40,
             eta: float = 0.5, move: float = 0.2, precision: str = "fp32", periodic: bool = False,
             tol: float = 1e-6, callback=None):
    """The optimisation procedure of Sec. 3.5 / Algorithm 1 with the continuation scheme of
    Sec. 3.3: for each continuation step l (beta = betas[l], q = qs[l]) up to n_opt design
    iterations of filter + projection -> forward -> J, G -> adjoint -> reverse of the filter
    -> MMA update, ending a step early when |J^k - J^(k-1)| <= tol |J^(k-1)| with G <= 0
    (Eq. stopping_criterion). J is maximised subject to the minimum-volume constraint
    G = 1 - sum(gamma_hat) / (vmin n) <= 0. With periodic=True the terminal state and body
    start the next iteration and the initial adjoint values end its reverse sweep (Sec. 3.4).

    The host only sequences the library's calls; every array stays on the device. The
    objective is scaled by 1 / |J| of the first iteration; the asymptote history restarts
    with each continuation step (the subproblem changes with beta and q). pb.ckpt_every
    sets the checkpoint interval of the reverse sweeps. Returns (gamma, history), history
    a list of dicts with l, k, J, G, lambda."""
    dt = DTYPES[precision]
    qs = list(qs) if qs is not None else [pb.q] * len(betas)
    if len(qs) != len(betas):
        raise ValueError("qs and betas need the same length")
    g = _dev(gamma0, torch.float64).reshape(-1).clone()
    n = g.numel()
    s0 = _dev(state0, dt).clone()
    b0 = _dev(body0, torch.float64).clone()
    mwork = torch.empty(mma_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    fwork = torch.empty(filter_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    scale, hist = None, []
    adj_s = adj_b = None
    for l, (beta, q) in enumerate(zip(betas, qs)):
        pbl = pb.replace(q=float(q))
        B = Buffers(pbl, precision, adjoint=True)
        lo = up = x1 = x2 = None
        J_prev = None
        for k in range(1, n_opt + 1):
            gt, gh = design_filter(pbl, g, radius, beta, eta, precision)
            st, bd, J, _ = forward(pbl, gh, s0, b0, precision, buffers=B, store_ckpt=True)
            G, dGh = volume_constraint(gh, vmin, work=mwork)
            Jv, Gv = float(J.item()), float(G.item())
            if J_prev is not None and Gv <= 0.0 and abs(Jv - J_prev) <= tol * abs(J_prev):
                hist.append(dict(l=l, k=k, J=Jv, G=Gv, lam=None))
                break
            if periodic:
                grad_h, ds, db = adjoint(pbl, gh, B, 1.0, precision, want_initial=True, dstate_T=adj_s, dbody_T=adj_b)
                adj_s, adj_b = ds, db
                s0, b0 = st, bd
            else:
                grad_h = adjoint(pbl, gh, B, 1.0, precision)
            dJ = design_filter_adjoint(pbl, gt, grad_h, radius, beta, eta, precision, work=fwork)
            dG = design_filter_adjoint(pbl, gt, dGh, radius, beta, eta, precision, work=fwork)
            if scale is None:
                scale = -1.0 / abs(Jv) if Jv != 0.0 else -1.0
            g_old = g.clone()
            g, lo, up, lam = mma_update(g, dJ, G, dG, k, x1, x2, lo, up, 0.0, 1.0, move, mwork, scale)
            x2, x1 = x1, g_old
            hist.append(dict(l=l, k=k, J=Jv, G=Gv, lam=float(lam.item())))
            if callback is not None:
                callback(hist[-1], g)
            J_prev = Jv
    return g, hist


class LKSFunction(torch.autograd.Function):
    """J = LKSFunction.apply(gamma, problem, precision, state0, body0).

    forward runs lks_forward with checkpoints every problem.ckpt_every steps; backward
    runs lks_adjoint with seed dL/dJ and returns dL/dgamma."""

    @staticmethod
    def forward(ctx, gamma, pb, precision, state0, body0):
        _, _, J, B = forward(pb, gamma.detach(), state0, body0, precision, store_ckpt=True)
        ctx.pb, ctx.precision, ctx.buffers = pb, precision, B
        ctx.save_for_backward(gamma)
        return J.reshape(()).to(gamma.dtype)

    @staticmethod
    def backward(ctx, gJ):
        (gamma,) = ctx.saved_tensors
        grad = adjoint(ctx.pb, gamma.detach(), ctx.buffers, seed=float(gJ), precision=ctx.precision)
        return grad.to(gamma.dtype).reshape(gamma.shape), None, None, None, None
