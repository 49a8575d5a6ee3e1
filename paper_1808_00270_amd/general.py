"""The general memory model on the GPU (C ABI in include/gld_general.h).

Argument marshalling only: the all-pairs search, F^D' with tabulated pair
kernels of any rank and the distance-dependent self memory, the window
transform of the white noise, the per-frequency Lanczos square roots
(Algorithm 1) and the integrator run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from . import _check, _dp, lib

__all__ = ["GeneralSystem"]


class GeneralSystem:
    """One GLD system with general kernel tables (FP64) on the current GPU.

    ``k_pair[b][m] = K^p_m(r_b)`` (any rank; or the separable ``k_pair_w``,
    ``k_pair_g``), ``dk_self[b][m] = Delta K^s_m(r_b)`` (optional), on the
    grid ``r0 + b dr``.  ``max_iters`` caps the Krylov dimension of each
    frequency's Lanczos process (0: 96); ``noise_tol`` is its stopping
    tolerance (0: 1e-12).
    """

    def __init__(self, *, n, box, dt, mass, kT, k_self, r, v, k_pair=None, k_pair_g=None, k_pair_w=None,
                 dk_self=None, r0=0.0, dr=0.01, r_cut=5.0, r_cut_min=0.0, parallel=False, wca_sigma=1.0,
                 wca_eps=1.0, seed=0, noise_tol=0.0, max_neighbors=0, max_iters=0, device=None, stream=None):
        import torch

        k_self = np.ascontiguousarray(k_self, dtype=np.float64)
        m_max = k_self.shape[0]
        kp = g = w = dks = None
        if k_pair is not None:
            kp = np.ascontiguousarray(k_pair, dtype=np.float64)
            assert kp.ndim == 2 and kp.shape[1] == m_max
        if k_pair_g is not None:
            g = np.ascontiguousarray(k_pair_g, dtype=np.float64)
            w = np.ascontiguousarray(k_pair_w, dtype=np.float64)
        if dk_self is not None:
            dks = np.ascontiguousarray(dk_self, dtype=np.float64)
        n_r = int(kp.shape[0]) if kp is not None else (int(w.shape[0]) if w is not None else
                                                       (int(dks.shape[0]) if dks is not None else 2))
        if dks is not None:
            assert dks.shape == (n_r, m_max)
        self._keep = [k_self, kp, g, w, dks]
        box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
        self.params = B.gld_params(
            n=int(n), box=(C.c_double * 3)(*box), dt=dt, mass=mass, kT=kT, m_max=m_max, n_r=n_r,
            k_self=_dp(k_self), k_pair_g=_dp(g), k_pair_w=_dp(w), r0=r0, dr=dr, r_cut=r_cut, r_cut_min=r_cut_min,
            pair_tensor=B.GLD_PAIR_PARALLEL if parallel else B.GLD_PAIR_ISOTROPIC, precision=B.GLD_FP64,
            wca_sigma=wca_sigma, wca_eps=wca_eps, seed=int(seed) & 0xFFFFFFFFFFFFFFFF, noise_tol=noise_tol,
            max_neighbors=max_neighbors, k_pair=_dp(kp), dk_self=_dp(dks))
        self.n, self.m_max, self.max_iters = int(n), m_max, int(max_iters)
        nbytes = C.c_size_t()
        _check(lib().gld_general_workspace_size(C.byref(self.params), self.max_iters, C.byref(nbytes)),
               "gld_general_workspace_size")
        self.workspace_bytes = nbytes.value
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(self.n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, 3)
        h = C.c_void_p()
        _check(lib().gld_general_create(C.byref(self.params), self.max_iters, _dp(r), _dp(v),
                                        C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)), "gld_general_create")
        self.handle = h

    @staticmethod
    def workspace_size(params, max_iters=0):
        nbytes = C.c_size_t()
        _check(lib().gld_general_workspace_size(C.byref(params), int(max_iters), C.byref(nbytes)),
               "gld_general_workspace_size")
        return nbytes.value

    def close(self):
        if getattr(self, "handle", None):
            lib().gld_general_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n_steps=1):
        _check(lib().gld_general_step(self.handle, int(n_steps)), "gld_general_step")

    def sync(self):
        _check(lib().gld_general_sync(self.handle), "gld_general_sync")

    def info(self):
        o = B.gld_general_info()
        _check(lib().gld_general_get_info(self.handle, C.byref(o)), "gld_general_get_info")
        return {f: getattr(o, f) for f, _ in o._fields_}

    def frequency_vectors(self, w0=0, w1=None):
        """x_w = sqrt(K_hat_w) Re W_hat_w of the last completed step, [w1 - w0][n][3]."""
        w1 = self.m_max if w1 is None else int(w1)
        out = np.zeros((w1 - w0, self.n, 3))
        _check(lib().gld_general_frequency_vectors(self.handle, int(w0), w1, _dp(out)),
               "gld_general_frequency_vectors")
        return out

    def set_timing(self, enable: bool):
        _check(lib().gld_general_set_timing(self.handle, int(bool(enable))), "gld_general_set_timing")

    def kernel_times(self):
        ms = (C.c_double * B.GLD_G_COUNT)()
        cnt = (C.c_int64 * B.GLD_G_COUNT)()
        _check(lib().gld_general_kernel_times(self.handle, ms, cnt), "gld_general_kernel_times")
        return {B.GENERAL_KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(B.GLD_G_COUNT)}

    def read_state(self, history=False, check=True):
        n3 = (self.n, 3)
        out = {k: np.zeros(n3) for k in ("r", "v", "f_c", "f_d", "f_r")}
        hist = np.zeros((max(self.m_max - 1, 0), self.n, 3)) if history else None
        st = B.gld_state(r=_dp(out["r"]), v=_dp(out["v"]), f_c=_dp(out["f_c"]), f_d=_dp(out["f_d"]),
                         f_r=_dp(out["f_r"]), history=_dp(hist) if hist is not None and hist.size else None)
        rc = lib().gld_general_read_state(self.handle, C.byref(st))
        if check:
            _check(rc, "gld_general_read_state")
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
        _check(lib().gld_general_write_state(self.handle, C.byref(st)), "gld_general_write_state")

