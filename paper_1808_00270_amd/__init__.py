"""MI355X generalized Langevin dynamics (GLD) time stepping.

Python front end of libgld.so (C ABI in include/gld.h): argument marshalling
and device memory/stream plumbing through PyTorch only.  The integrator
itself (neighbour build, memory convolution, pair contraction, colored noise,
update) runs entirely in the HIP kernels of the library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B

__all__ = ["System", "GLDError", "lib", "white_noise", "noise_filters"]

_lib = None


def lib():
    """The loaded libgld.so (raises ImportError if it is not built)."""
    global _lib
    if _lib is None:
        _lib = B.load()
    return _lib


class GLDError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().gld_status_string(status).decode()
        detail = lib().gld_last_error().decode()
        super().__init__(f"{what}: {msg} ({status}) {detail}")
        self.status = status


def _check(status: int, what: str):
    if status != B.GLD_OK:
        raise GLDError(status, what)


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class System:
    """One GLD system on the current GPU.

    Tables are the discrete kernels: ``k_self[m] = K^s_m``, pair memory
    ``K^p_m(r) = w(r) g_m`` with ``w`` on the grid ``r0 + b dr``.
    ``verlet_skin`` defaults to 0.1 r_cut (0: rebuild the lists every step).
    ``noise_window`` W > 1 computes the random forces of W consecutive steps
    together at the positions of the window's first step (the variant of
    Sec. II.C for positions that barely move over W steps); W must divide
    the filter block of the noise plan.
    """

    def __init__(self, *, n, box, dt, mass, kT, k_self, r, v, k_pair_g=None, k_pair_w=None, r0=0.0, dr=0.01,
                 r_cut=5.0, r_cut_min=0.0, parallel=False, fp64=False, wca_sigma=1.0, wca_eps=1.0, seed=0,
                 noise_tol=0.0, lam_lo=0.0, lam_hi=0.0, max_neighbors=0, check_interval=0, verlet_skin=None,
                 noise_window=1, k_pair=None, dk_self=None, noise_filters=None, check_iters=0, rebuild_period=0,
                 device=None, stream=None):
        import torch

        self._keep = []
        k_self = np.ascontiguousarray(k_self, dtype=np.float64)
        m_max = k_self.shape[0]
        g = w = kp = dks = fa = fb = None
        if k_pair_g is not None:
            g = np.ascontiguousarray(k_pair_g, dtype=np.float64)
            w = np.ascontiguousarray(k_pair_w, dtype=np.float64)
            assert g.shape == (m_max,)
        if k_pair is not None:  # the general table [n_r][m_max]
            kp = np.ascontiguousarray(k_pair, dtype=np.float64)
            assert kp.ndim == 2 and kp.shape[1] == m_max
        if dk_self is not None:
            dks = np.ascontiguousarray(dk_self, dtype=np.float64)
        if noise_filters is not None:  # (taps [rank][2 m_max - 1], mixing weights [K][rank])
            fa = np.ascontiguousarray(noise_filters[0], dtype=np.float64)
            fb = np.ascontiguousarray(noise_filters[1], dtype=np.float64)
            assert fa.shape[1] == 2 * m_max - 1 and fb.shape[1] == fa.shape[0]
        n_r = int(w.shape[0]) if w is not None else (int(kp.shape[0]) if kp is not None else 2)
        self._keep += [k_self, g, w, kp, dks, fa, fb]
        box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
        self.params = B.gld_params(
            n=int(n), box=(C.c_double * 3)(*box), dt=dt, mass=mass, kT=kT, m_max=m_max, n_r=n_r,
            k_self=_dp(k_self), k_pair_g=_dp(g), k_pair_w=_dp(w), r0=r0, dr=dr, r_cut=r_cut, r_cut_min=r_cut_min,
            pair_tensor=B.GLD_PAIR_PARALLEL if parallel else B.GLD_PAIR_ISOTROPIC,
            precision=B.GLD_FP64 if fp64 else B.GLD_FP32_MIXED, wca_sigma=wca_sigma, wca_eps=wca_eps,
            seed=int(seed) & 0xFFFFFFFFFFFFFFFF, noise_tol=noise_tol, lam_lo=lam_lo, lam_hi=lam_hi,
            max_neighbors=max_neighbors, check_interval=check_interval,
            verlet_skin=0.1 * r_cut if verlet_skin is None else float(verlet_skin), noise_window=int(noise_window),
            k_pair=_dp(kp), dk_self=_dp(dks), noise_a=_dp(fa), noise_b=_dp(fb),
            noise_rank=int(fa.shape[0]) if fa is not None else 0, noise_terms=int(fb.shape[0]) if fb is not None else 0,
            check_iters=int(check_iters), rebuild_period=int(rebuild_period))
        self.n, self.m_max, self.fp64 = int(n), m_max, fp64
        nbytes = C.c_size_t()
        _check(lib().gld_workspace_size(C.byref(self.params), C.byref(nbytes)), "gld_workspace_size")
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(self.n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, 3)
        h = C.c_void_p()
        _check(lib().gld_create(C.byref(self.params), _dp(r), _dp(v), C.c_void_p(self.workspace.data_ptr()),
                                nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)), "gld_create")
        self.handle = h

    @classmethod
    def from_workload(cls, wl, *, fp64=False, **kw):
        """Build from a :class:`workloads.Workload` (its tables and initial state)."""
        k_self, g, w, r0, dr = wl.tables()
        R, V = wl.initial_state()
        args = dict(n=wl.n, box=wl.box, dt=wl.dt, mass=wl.mass, kT=wl.kT, k_self=k_self, k_pair_g=g, k_pair_w=w,
                    r0=r0, dr=dr, r_cut=wl.r_cut, parallel=wl.parallel, fp64=fp64, wca_sigma=wl.wca_sigma,
                    wca_eps=wl.wca_eps, seed=wl.seed, r=R, v=V)
        args.update(kw)
        return cls(**args)

    def close(self):
        if getattr(self, "handle", None):
            lib().gld_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping ---------------------------------------------------------
    def step(self, n_steps=1):
        _check(lib().gld_step(self.handle, int(n_steps)), "gld_step")

    def sync(self):
        _check(lib().gld_sync(self.handle), "gld_sync")

    def set_graph(self, enable: bool):
        _check(lib().gld_set_graph(self.handle, int(bool(enable))), "gld_set_graph")

    def set_timing(self, enable: bool):
        _check(lib().gld_set_timing(self.handle, int(bool(enable))), "gld_set_timing")

    def kernel_times(self):
        ms = (C.c_double * B.GLD_K_COUNT)()
        cnt = (C.c_int64 * B.GLD_K_COUNT)()
        _check(lib().gld_kernel_times(self.handle, ms, cnt), "gld_kernel_times")
        return {B.KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(B.GLD_K_COUNT)}

    def list_stats(self):
        """(directed pairs within r_cut in the current list, most per particle)."""
        pairs, most = C.c_int64(), C.c_int32()
        _check(lib().gld_list_stats(self.handle, C.byref(pairs), C.byref(most)), "gld_list_stats")
        return pairs.value, most.value

    def noise_info(self):
        o = B.gld_noise_info()
        _check(lib().gld_noise_parameters(self.handle, C.byref(o)), "gld_noise_parameters")
        return {f: getattr(o, f) for f, _ in o._fields_}

    # -- state --------------------------------------------------------------
    def read_state(self, history=False, check=True):
        n3 = (self.n, 3)
        out = {k: np.zeros(n3) for k in ("r", "v", "f_c", "f_d", "f_r")}
        hist = np.zeros((max(self.m_max - 1, 0), self.n, 3)) if history else None
        st = B.gld_state(r=_dp(out["r"]), v=_dp(out["v"]), f_c=_dp(out["f_c"]), f_d=_dp(out["f_d"]),
                         f_r=_dp(out["f_r"]), history=_dp(hist) if hist is not None and hist.size else None)
        rc = lib().gld_read_state(self.handle, C.byref(st))
        if check:
            _check(rc, "gld_read_state")
        out["history"] = hist
        out["step"] = st.step
        out["flags"] = st.flags
        out["flag_step"] = st.flag_step
        out["status"] = rc
        return out

    def write_state(self, r, v, step=0, history=None):
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(self.n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, 3)
        h = None
        if history is not None:
            h = np.ascontiguousarray(history, dtype=np.float64)
            assert h.shape == (max(self.m_max - 1, 0), self.n, 3)
        st = B.gld_state(r=_dp(r), v=_dp(v), history=_dp(h) if h is not None and h.size else None, step=int(step))
        _check(lib().gld_write_state(self.handle, C.byref(st)), "gld_write_state")


def noise_filters(params, lam_lo, lam_hi, tol=0.0):
    """The one-off noise construction for [lam_lo, lam_hi] (host only):
    (taps [rank][2 m_max - 1], mixing weights [K][rank], info dict)."""
    P = 2 * params.m_max - 1
    A = np.zeros(32 * P)
    Bm = np.zeros(512 * 32)
    info = B.gld_noise_info()
    _check(lib().gld_build_noise_filters(C.byref(params), float(lam_lo), float(lam_hi), float(tol), _dp(A), A.size,
                                         _dp(Bm), Bm.size, C.byref(info)), "gld_build_noise_filters")
    r, K = info.rank, info.cheb_terms
    return A[:r * P].reshape(r, P).copy(), Bm[:K * r].reshape(K, r).copy(), {f: getattr(info, f) for f, _ in info._fields_}


def white_noise(seed, n, t0, n_t, device="cuda"):
    """(W[n_t, n, 3] float64, raw Philox words[n_t, n, 4] uint32) as drawn by the integrator."""
    import torch
    out = torch.empty((n_t, n, 3), dtype=torch.float64, device=device)
    raw = torch.empty((n_t, n, 4), dtype=torch.int32, device=device)
    s = torch.cuda.current_stream(device)
    _check(lib().gld_white_noise(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(n), int(t0), int(n_t),
                                 C.c_void_p(out.data_ptr()), C.c_void_p(raw.data_ptr()), C.c_void_p(s.cuda_stream)),
           "gld_white_noise")
    return out.cpu().numpy(), raw.cpu().numpy().view(np.uint32)
