"""gld_create_static (the entry point for callers that cannot allocate device
memory) against gld_create with a caller workspace: the same system stepped
through the C ABI gives the same state, bit for bit (same kernels, same
reduction order), on two creations in a row, the second with a smaller
system; and the static workspace refuses a system larger than it holds and a
second live system on the same device."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1808_00270_amd import workloads as wl

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_00270_amd as p
    p.lib()
    return p


def dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def read(lib, B, h, n, m_max):
    out = {k: np.zeros((n, 3)) for k in ("r", "v", "f_c", "f_d", "f_r")}
    hist = np.zeros((m_max - 1, n, 3))
    st = B.gld_state(r=dp(out["r"]), v=dp(out["v"]), f_c=dp(out["f_c"]), f_d=dp(out["f_d"]), f_r=dp(out["f_r"]),
                     history=dp(hist))
    assert lib.gld_read_state(h, C.byref(st)) == B.GLD_OK
    out["history"] = hist
    out["step"] = st.step
    return out


def run_static(pkg, w, fp64, steps, hist, stream):
    """Create through gld_create_static, install a state with history, step."""
    lib, B = pkg.lib(), pkg._binding
    ref = pkg.System.from_workload(w, fp64=fp64)  # its params (and the reference run below)
    R, V = w.initial_state()
    h = C.c_void_p()
    Rc, Vc = np.ascontiguousarray(R), np.ascontiguousarray(V)
    st = lib.gld_create_static(C.byref(ref.params), dp(Rc), dp(Vc), C.c_void_p(stream.cuda_stream), C.byref(h))
    assert st == B.GLD_OK, lib.gld_last_error()
    hc = np.ascontiguousarray(hist)
    state = B.gld_state(r=dp(Rc), v=dp(Vc), history=dp(hc), step=11)
    assert lib.gld_write_state(h, C.byref(state)) == B.GLD_OK
    assert lib.gld_step(h, steps) == B.GLD_OK
    got = read(lib, B, h, w.n, w.m_max)
    assert lib.gld_destroy(h) == B.GLD_OK
    # the caller-workspace entry point on the same inputs
    ref.write_state(R, V, step=11, history=hist)
    ref.step(steps)
    want = ref.read_state(history=True)
    ref.close()
    return got, want


@pytest.mark.parametrize("fp64", [True, False])
def test_static_workspace_matches_caller_workspace(pkg, fp64):
    import torch
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(5)
    # two calls in a row, the second with a smaller system
    for w in (wl.config(1, n=300, rho=0.05, m_max=200), wl.config(1, n=64, m_max=120)):
        hist = wl.random_history(rng, w.m_max, w.n, scale=0.01)
        log(f"  static vs caller workspace: n={w.n} m_max={w.m_max} fp64={fp64}")
        got, want = run_static(pkg, w, fp64, 25, hist, stream)
        assert got["step"] == want["step"] == 36
        for k in ("r", "v", "f_c", "f_d", "f_r", "history"):
            assert np.array_equal(got[k], want[k]), k


def test_static_workspace_limits(pkg):
    import torch
    lib, B = pkg.lib(), pkg._binding
    stream = torch.cuda.Stream()
    big = wl.config(2)  # N = 1e4, m_max = 500: far beyond the static workspace
    ref_big = pkg.System.from_workload(wl.config(1), fp64=True)
    p = ref_big.params
    wbig = big
    k_self, g, wt, r0, dr = wbig.tables()
    Rb, Vb = wbig.initial_state()
    pb = B.gld_params.from_buffer_copy(p)
    pb.n = wbig.n
    pb.box = (C.c_double * 3)(wbig.box, wbig.box, wbig.box)
    pb.m_max = wbig.m_max
    pb.k_self, pb.k_pair_g = dp(k_self), dp(g)
    h = C.c_void_p()
    st = lib.gld_create_static(C.byref(pb), dp(Rb), dp(Vb), C.c_void_p(stream.cuda_stream), C.byref(h))
    assert st == B.GLD_ERR_OOM and b"static workspace" in lib.gld_last_error()
    ref_big.close()
    # one live static system per device
    w = wl.config(1)
    ref = pkg.System.from_workload(w)
    R, V = w.initial_state()
    h1, h2 = C.c_void_p(), C.c_void_p()
    assert lib.gld_create_static(C.byref(ref.params), dp(R), dp(V), C.c_void_p(stream.cuda_stream),
                                 C.byref(h1)) == B.GLD_OK
    assert lib.gld_create_static(C.byref(ref.params), dp(R), dp(V), C.c_void_p(stream.cuda_stream),
                                 C.byref(h2)) == B.GLD_ERR_INVALID_ARG
    assert lib.gld_destroy(h1) == B.GLD_OK
    assert lib.gld_create_static(C.byref(ref.params), dp(R), dp(V), C.c_void_p(stream.cuda_stream),
                                 C.byref(h2)) == B.GLD_OK
    assert lib.gld_step(h2, 3) == B.GLD_OK
    assert lib.gld_sync(h2) == B.GLD_OK
    assert lib.gld_destroy(h2) == B.GLD_OK
    ref.close()
