"""Plain serial FP64 CPU oracle -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library never loads it, and it shares
no code with the GPU library (see ``lks_oracle.c`` for what it computes and which
passages of the paper each routine follows).

``build()`` compiles ``lks_oracle.c`` with gcc into ``liblks_oracle.so`` next to
this file; the wrappers below marshal numpy arrays into the C entry points.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lks_oracle.c")
_LIB = os.path.join(_HERE, "liblks_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, -O2, no fast-math, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_int * 3),
        ("bc", C.c_int * 6),
        ("bc_p", C.c_double * 6),
        ("bc_u", (C.c_double * 3) * 6),
        ("nu", C.c_double),
        ("nd", C.c_int * 3),
        ("kappa_max", C.c_double),
        ("q", C.c_double),
        ("mass", C.c_double),
        ("inertia", C.c_double),
        ("axis", C.c_int),
        ("dof_mask", C.c_int),
        ("n_itr", C.c_int),
        ("n_steps", C.c_int),
        ("objective", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(OrcProblem)
        L.orc_step.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_forward.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_gradient.argtypes = [pp, dp, dp, dp, C.c_double, dp, dp, dp, dp, dp, dp]
        L.orc_gradient_paper.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_cyclic_sector_points.argtypes = [pp, C.c_int]
        L.orc_cyclic_sector_points.restype = C.c_long
        L.orc_cyclic_expand.argtypes = [pp, C.c_int, dp, dp]
        L.orc_cyclic_collect.argtypes = [pp, C.c_int, dp, dp]
        L.orc_map_design.argtypes = [pp, dp, dp, dp, dp]
        L.orc_interp.argtypes = [pp, dp, dp, dp]
        L.orc_force.argtypes = [pp, dp, dp, dp, dp]
        L.orc_body_step.argtypes = [pp, dp, dp, dp]
        L.orc_coupling.argtypes = [pp, dp, dp, dp, dp]
        L.orc_kappa_ref.argtypes = [pp, dp, dp]
        ip = C.POINTER(C.c_int)
        L.orc_filter.argtypes = [C.c_int, ip, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_filter_adjoint.argtypes = [C.c_int, ip, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        _lib = L
    return _lib


def problem_struct(pb) -> OrcProblem:
    """Marshal a ``workloads.Problem`` into the oracle's own struct."""
    s = OrcProblem()
    s.dim = pb.dim
    for a in range(3):
        s.n[a] = pb.n[a]
        s.nd[a] = pb.nd[a]
    for f in range(6):
        s.bc[f] = pb.bc[f]
        s.bc_p[f] = pb.bc_p[f]
        for a in range(3):
            s.bc_u[f][a] = pb.bc_u[f][a]
    s.nu = pb.nu
    s.kappa_max = pb.kappa_max
    s.q = pb.q
    s.mass = pb.mass
    s.inertia = pb.inertia
    s.axis = pb.axis
    s.dof_mask = pb.dof_mask
    s.n_itr = pb.n_itr
    s.n_steps = pb.n_steps
    s.objective = pb.objective
    return s


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def step(pb, gamma, state, body):
    s = problem_struct(pb)
    so = np.empty_like(_f64(state))
    bo = np.empty(12)
    _check(lib().orc_step(C.byref(s), _p(_f64(gamma)) if gamma is not None else None,
                          _p(_f64(state)), _p(_f64(body)), _p(so), _p(bo)), "orc_step")
    return so, bo


def forward(pb, gamma, state, body, traj=False):
    """Run pb.n_steps steps. Returns (state, body, J[, trajectory])."""
    s = problem_struct(pb)
    st = _f64(state).copy()
    bd = _f64(body).copy()
    tr = np.empty((pb.n_steps + 1, 12)) if traj else None
    J = C.c_double(0.0)
    g = _f64(gamma) if gamma is not None else None
    _check(lib().orc_forward(C.byref(s), _p(g), _p(st), _p(bd), _p(tr), C.byref(J)),
           "orc_forward")
    return (st, bd, J.value, tr) if traj else (st, bd, J.value)


def gradient(pb, gamma, state0, body0, seed=1.0, with_initial=False, dstate_T=None, dbody_T=None):
    """Exact discrete adjoint of seed * J + <dstate_T, state(N_t)> + <dbody_T, body(N_t)>
    (the terminal cotangents are optional). Returns (J, grad[, dstate0, dbody0])."""
    s = problem_struct(pb)
    g = _f64(gamma)
    grad = np.zeros_like(g)
    J = C.c_double(0.0)
    ds = np.zeros_like(_f64(state0)) if with_initial else None
    db = np.zeros(12) if with_initial else None
    sT = _f64(dstate_T) if dstate_T is not None else None
    bT = _f64(dbody_T) if dbody_T is not None else None
    if bT is not None and bT.size < 8:
        raise ValueError("dbody_T needs at least 8 entries")
    if sT is not None and sT.size != _f64(state0).size:
        raise ValueError("dstate_T must have the size of a state")
    _check(lib().orc_gradient(C.byref(s), _p(g), _p(_f64(state0)), _p(_f64(body0)),
                              float(seed), _p(sT), _p(bT), _p(grad), C.byref(J), _p(ds), _p(db)),
           "orc_gradient")
    return (J.value, grad, ds, db) if with_initial else (J.value, grad)


def gradient_paper(pb, gamma, state0, body0):
    """The paper's adjoint variant (continuous adjoint discretised, Sec. 2.5): returns
    (J, grad). Not the exact derivative of the discrete forward map."""
    s = problem_struct(pb)
    g = _f64(gamma)
    grad = np.zeros_like(g)
    J = C.c_double(0.0)
    _check(lib().orc_gradient_paper(C.byref(s), _p(g), _p(_f64(state0)), _p(_f64(body0)), _p(grad), C.byref(J)),
           "orc_gradient_paper")
    return J.value, grad


def kappa_ref(pb, gamma):
    s = problem_struct(pb)
    g = _f64(gamma)
    out = np.empty_like(g)
    _check(lib().orc_kappa_ref(C.byref(s), _p(g), _p(out)), "orc_kappa_ref")
    return out


def map_design(pb, kref, body):
    s = problem_struct(pb)
    N = int(np.prod(pb.n))
    kap = np.empty(N)
    uS = np.empty(pb.dim * N)
    _check(lib().orc_map_design(C.byref(s), _p(_f64(kref)), _p(_f64(body)), _p(kap), _p(uS)),
           "orc_map_design")
    return kap, uS


def interp(pb, u, body):
    s = problem_struct(pb)
    ND = int(np.prod(pb.nd))
    uref = np.empty(pb.dim * ND)
    _check(lib().orc_interp(C.byref(s), _p(_f64(u)), _p(_f64(body)), _p(uref)), "orc_interp")
    return uref


def force(pb, kref, uref, body):
    s = problem_struct(pb)
    FT = np.zeros(4)
    _check(lib().orc_force(C.byref(s), _p(_f64(kref)), _p(_f64(uref)), _p(_f64(body)), _p(FT)),
           "orc_force")
    return FT


def body_step(pb, FT, body_prev):
    s = problem_struct(pb)
    out = np.empty(12)
    _check(lib().orc_body_step(C.byref(s), _p(_f64(FT)), _p(_f64(body_prev)), _p(out)),
           "orc_body_step")
    return out


def coupling(pb, gamma, state, body):
    s = problem_struct(pb)
    K = np.zeros(4)
    _check(lib().orc_coupling(C.byref(s), _p(_f64(gamma)), _p(_f64(state)), _p(_f64(body)),
                              _p(K)), "orc_coupling")
    return K


def filter(dim, nd, R, beta, eta, g):
    """Density filter + Heaviside projection (Sec. 3.2): returns (gt, gh)."""
    nd3 = (C.c_int * 3)(*[int(v) for v in nd])
    g = _f64(g)
    gt, gh = np.empty_like(g), np.empty_like(g)
    _check(lib().orc_filter(int(dim), nd3, float(R), float(beta), float(eta), _p(g), _p(gt), _p(gh)),
           "orc_filter")
    return gt, gh


def filter_adjoint(dim, nd, R, beta, eta, gt, gbh):
    """Cotangent of gamma from the cotangent of the projected field."""
    nd3 = (C.c_int * 3)(*[int(v) for v in nd])
    gt, gbh = _f64(gt), _f64(gbh)
    gb = np.empty_like(gt)
    _check(lib().orc_filter_adjoint(int(dim), nd3, float(R), float(beta), float(eta), _p(gt), _p(gbh), _p(gb)),
           "orc_filter_adjoint")
    return gb


def cyclic_sector_points(pb, n_sec):
    """Design variables of one sector of the cyclic periodic design (Sec. 4.2), or -1."""
    return int(lib().orc_cyclic_sector_points(C.byref(problem_struct(pb)), int(n_sec)))


def cyclic_expand(pb, n_sec, gs):
    """Sector design -> design grid (repeated by the rotations about the rotation axis)."""
    s = problem_struct(pb)
    gs = _f64(gs)
    if gs.size != cyclic_sector_points(pb, n_sec):
        raise ValueError("sector array has the wrong size")
    g = np.empty(int(np.prod(pb.nd)))
    _check(lib().orc_cyclic_expand(C.byref(s), int(n_sec), _p(gs), _p(g)), "orc_cyclic_expand")
    return g


def cyclic_collect(pb, n_sec, grad):
    """Design-grid sensitivities -> sector (transpose of cyclic_expand)."""
    s = problem_struct(pb)
    grad = _f64(grad)
    gs = np.empty(cyclic_sector_points(pb, n_sec))
    _check(lib().orc_cyclic_collect(C.byref(s), int(n_sec), _p(grad), _p(gs)), "orc_cyclic_collect")
    return gs
