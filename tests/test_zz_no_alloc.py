"""lks_forward_noalloc (the entry point for callers that cannot allocate) against
lks_forward, through the C ABI: two calls in a row on one GPU, the second with a smaller
problem, each bitwise equal to lks_forward on the same inputs (the same kernels run on
the same workspace layout), the second also against the FP64 oracle; a problem beyond
the static scratch and the profiling flag are rejected."""
import ctypes as C

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


def _noalloc(L, pb, g, s0, b0, prec, flags=0):
    import torch

    lib = L._lib.load()
    dt = L.api.DTYPES[prec]
    s = L.problem_struct(pb, prec, flags)
    gd = torch.as_tensor(g, dtype=dt, device="cuda") if g is not None else None
    st = torch.as_tensor(s0, dtype=dt, device="cuda").clone()
    bd = torch.as_tensor(b0, dtype=torch.float64, device="cuda").clone()
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    rc = lib.lks_forward_noalloc(C.byref(s), p(gd), p(st), p(bd), p(J), stream)
    return rc, st, bd, J


def test_noalloc_forward_matches_forward(L, orc):
    cases = [(W.config("config2").replace(n_steps=60), "fp32"),
             (W.small2d(), "fp64")]  # the second call is the smaller problem
    for pb, prec in cases:
        g, s0, b0 = W.design(pb), W.initial_state(pb), W.initial_body(pb)
        need = L.workspace_bytes(pb, False, prec)
        print(f"noalloc {pb.name} {prec}: scratch {need} of {L._lib.NOALLOC_SCRATCH_BYTES} bytes", flush=True)
        assert need <= L._lib.NOALLOC_SCRATCH_BYTES
        rc, st, bd, J = _noalloc(L, pb, g, s0, b0, prec)
        assert rc == 0, L._lib.load().lks_last_error()
        st_r, bd_r, J_r, _ = L.forward(pb, g, s0, b0, precision=prec, store_ckpt=False)
        assert np.array_equal(st.cpu().numpy(), st_r.cpu().numpy())
        assert np.array_equal(bd.cpu().numpy(), bd_r.cpu().numpy())
        assert J.item() == J_r.item()
    # the smaller problem also against the oracle (FP64 bar)
    pb = cases[1][0]
    sref, bref, Jref = orc.forward(pb, W.design(pb), W.initial_state(pb), W.initial_body(pb))
    assert np.abs(st.cpu().numpy() - sref).max() <= 1e-11 * np.abs(sref).max()
    assert abs(J.item() - Jref) <= 1e-9 * abs(Jref)


def test_noalloc_rejects_what_it_cannot_serve(L):
    lib = L._lib
    pb = W.config("config5").replace(n_steps=1)
    assert L.workspace_bytes(pb, False) > lib.NOALLOC_SCRATCH_BYTES
    s0 = np.zeros(4)  # never read: rejected before any device access
    rc, _, _, _ = _noalloc(L, pb, np.zeros(4), s0, np.zeros(12), "fp32")
    assert rc == lib.ENOSPACE and b"scratch" in lib.load().lks_last_error()
    pb = W.small2d(n_steps=2)
    rc, _, _, _ = _noalloc(L, pb, W.design(pb), W.initial_state(pb), W.initial_body(pb), "fp32",
                           flags=lib.FLAG_PROFILE)
    assert rc == lib.EINVAL
