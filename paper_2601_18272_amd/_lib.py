"""ctypes view of the C ABI declared in include/lks.h (liblks_hip.so, built in-tree).

Loading fails loudly if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblks_hip.so")

PERIODIC, VELOCITY, PRESSURE, WALL = 0, 1, 2, 3
FP32, FP64 = 0, 1
FLAG_ASYNC = 1
FLAG_PROFILE = 2
FLAG_STABILITY = 4
FLAG_PAPER_ADJOINT = 8
FLAG_MARCH2D = 16
FLAG_PLANE3D = 32
KERNELS = ("gather", "bc", "spread", "interp", "adj_gather", "adj_recompute", "adj_r1", "adj_r2",
           "adj_r3", "iter", "iter_final", "gather_span", "adj_gather_span", "filter", "filter_adj",
           "cyc_expand", "cyc_collect")

OK, EINVAL, ENOSPACE, EUNSTABLE, EDIVERGED, EHIP = 0, -1, -2, -3, -4, -5

EXPORTS = ("lks_state_elems", "lks_checkpoint_bytes", "lks_workspace_bytes", "lks_forward",
           "lks_adjoint", "map_design", "body_step", "lks_last_error", "lks_profile_read",
           "lks_profile_reset", "lks_design_filter", "lks_design_filter_adjoint",
           "lks_filter_workspace_bytes", "lks_cyclic_sector_points", "lks_design_cyclic_expand",
           "lks_design_cyclic_collect", "lks_mma_workspace_bytes", "lks_mma_update", "lks_volume_constraint",
           "lks_coupling", "lks_forward_noalloc")
NOALLOC_SCRATCH_BYTES = 32 << 20


class LksProblem(C.Structure):
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
        ("ckpt_every", C.c_int),
        ("precision", C.c_int),
        ("objective", C.c_int),
        ("flags", C.c_int),
    ]


class LksFilter(C.Structure):
    _fields_ = [("radius", C.c_double), ("beta", C.c_double), ("eta", C.c_double)]


class LksMma(C.Structure):
    _fields_ = [("xmin", C.c_double), ("xmax", C.c_double), ("move", C.c_double), ("f0_scale", C.c_double)]


class LksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lks error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load liblks_hip.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2601_18272_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    pp = C.POINTER(LksProblem)
    vp = C.c_void_p
    dp = C.c_void_p
    L.lks_state_elems.argtypes = [pp]
    L.lks_state_elems.restype = C.c_size_t
    L.lks_checkpoint_bytes.argtypes = [pp]
    L.lks_checkpoint_bytes.restype = C.c_size_t
    L.lks_workspace_bytes.argtypes = [pp, C.c_int]
    L.lks_workspace_bytes.restype = C.c_size_t
    L.lks_forward.argtypes = [pp, vp, vp, dp, vp, C.c_size_t, vp, C.c_size_t, dp, vp]
    L.lks_forward.restype = C.c_int
    L.lks_adjoint.argtypes = [pp, vp, vp, C.c_size_t, vp, C.c_size_t, C.c_double, vp, dp, dp, vp, dp, vp]
    L.lks_adjoint.restype = C.c_int
    L.map_design.argtypes = [pp, vp, dp, vp, vp, vp]
    L.map_design.restype = C.c_int
    L.body_step.argtypes = [pp, dp, dp, dp, vp]
    L.lks_coupling.argtypes = [pp, vp, dp, dp, vp, C.c_size_t, vp]
    L.lks_coupling.restype = C.c_int
    L.lks_forward_noalloc.argtypes = [pp, vp, vp, dp, dp, vp]
    L.lks_forward_noalloc.restype = C.c_int
    L.body_step.restype = C.c_int
    fp = C.POINTER(LksFilter)
    L.lks_design_filter.argtypes = [pp, fp, vp, vp, vp, vp]
    L.lks_design_filter.restype = C.c_int
    L.lks_design_filter_adjoint.argtypes = [pp, fp, vp, dp, vp, C.c_size_t, dp, vp]
    L.lks_design_filter_adjoint.restype = C.c_int
    L.lks_filter_workspace_bytes.argtypes = [pp]
    L.lks_filter_workspace_bytes.restype = C.c_size_t
    L.lks_cyclic_sector_points.argtypes = [pp, C.c_int]
    L.lks_cyclic_sector_points.restype = C.c_size_t
    L.lks_design_cyclic_expand.argtypes = [pp, C.c_int, vp, vp, vp]
    L.lks_design_cyclic_expand.restype = C.c_int
    L.lks_design_cyclic_collect.argtypes = [pp, C.c_int, dp, dp, vp]
    L.lks_design_cyclic_collect.restype = C.c_int
    L.lks_mma_workspace_bytes.argtypes = [C.c_longlong]
    L.lks_mma_workspace_bytes.restype = C.c_size_t
    L.lks_mma_update.argtypes = [C.POINTER(LksMma), C.c_longlong, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                 vp, C.c_size_t, vp]
    L.lks_mma_update.restype = C.c_int
    L.lks_volume_constraint.argtypes = [C.c_longlong, dp, C.c_double, dp, dp, vp, C.c_size_t, vp]
    L.lks_volume_constraint.restype = C.c_int
    L.lks_last_error.argtypes = []
    L.lks_last_error.restype = C.c_char_p
    L.lks_profile_read.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
    L.lks_profile_read.restype = C.c_int
    L.lks_profile_reset.argtypes = []
    L.lks_profile_reset.restype = None
    _lib = L
    return L


def check(rc: int):
    if rc != OK:
        raise LksError(rc, load().lks_last_error().decode())


def profile_read() -> dict:
    """{kernel name: (sampled total ms, samples)} from calls made with FLAG_PROFILE."""
    L = load()
    out = {}
    for i, name in enumerate(KERNELS):
        ms = C.c_double(0.0)
        n = C.c_longlong(0)
        check(L.lks_profile_read(i, C.byref(ms), C.byref(n)))
        out[name] = (ms.value, n.value)
    return out


def profile_reset() -> None:
    load().lks_profile_reset()
