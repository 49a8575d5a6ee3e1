"""Python front end of the batched engine (include/gld_batch.h): many
independent GLD systems advanced together on one GPU.

Argument marshalling only: every step of every system runs in the HIP
kernels of libgld.so.  Each system is described as for :class:`System`
(keyword arguments or a workload); all systems of a batch share its
precision.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from . import lib, _check, _dp, GLDError  # noqa: F401


def system_params(*, n, box, dt, mass, kT, k_self, k_pair_g=None, k_pair_w=None, r0=0.0, dr=0.01, r_cut=5.0,
                  r_cut_min=0.0, fp64=False, wca_sigma=1.0, wca_eps=1.0, seed=0, noise_tol=0.0, lam_lo=0.0,
                  lam_hi=0.0, max_neighbors=0, k_pair=None):
    """(gld_params, arrays to keep alive) for one system of a batch."""
    k_self = np.ascontiguousarray(k_self, dtype=np.float64)
    m_max = k_self.shape[0]
    g = w = kp = None
    if k_pair_g is not None:
        g = np.ascontiguousarray(k_pair_g, dtype=np.float64)
        w = np.ascontiguousarray(k_pair_w, dtype=np.float64)
    if k_pair is not None:
        kp = np.ascontiguousarray(k_pair, dtype=np.float64)
    n_r = int(w.shape[0]) if w is not None else (int(kp.shape[0]) if kp is not None else 2)
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    p = B.gld_params(
        n=int(n), box=(C.c_double * 3)(*box), dt=dt, mass=mass, kT=kT, m_max=m_max, n_r=n_r, k_self=_dp(k_self),
        k_pair_g=_dp(g), k_pair_w=_dp(w), r0=r0, dr=dr, r_cut=r_cut, r_cut_min=r_cut_min,
        pair_tensor=B.GLD_PAIR_ISOTROPIC, precision=B.GLD_FP64 if fp64 else B.GLD_FP32_MIXED,
        wca_sigma=wca_sigma, wca_eps=wca_eps, seed=int(seed) & 0xFFFFFFFFFFFFFFFF, noise_tol=noise_tol,
        lam_lo=lam_lo, lam_hi=lam_hi, max_neighbors=max_neighbors, k_pair=_dp(kp))
    return p, [k_self, g, w, kp]


def workload_params(wl, fp64=False, **kw):
    k_self, g, w, r0, dr = wl.tables()
    kw2 = dict(n=wl.n, box=wl.box, dt=wl.dt, mass=wl.mass, kT=wl.kT, k_self=k_self, k_pair_g=g, k_pair_w=w, r0=r0,
               dr=dr, r_cut=wl.r_cut, fp64=fp64, wca_sigma=wl.wca_sigma, wca_eps=wl.wca_eps, seed=wl.seed)
    kw2.update(kw)
    return system_params(**kw2)


def base_size(capacity):
    """Device bytes of a batch's own tables (descriptors, launch maps)."""
    nb = C.c_size_t()
    _check(lib().gld_batch_base_size(int(capacity), C.byref(nb)), "gld_batch_base_size")
    return nb.value


class Batch:
    """A batch of up to `capacity` systems in one device workspace of
    `workspace_bytes` (a torch uint8 tensor)."""

    def __init__(self, capacity, workspace_bytes, fp64=False, device=None, stream=None):
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        self.fp64 = fp64
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        _check(lib().gld_batch_create(B.GLD_FP64 if fp64 else B.GLD_FP32_MIXED, int(capacity),
                                      C.c_void_p(self.workspace.data_ptr()), int(workspace_bytes),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)), "gld_batch_create")
        self.handle = h
        self.n = {}
        self.m_max = {}
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().gld_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, params, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        nb = C.c_size_t()
        _check(lib().gld_batch_footprint(self.handle, C.byref(params), _dp(r), C.byref(nb)), "gld_batch_footprint")
        return nb.value

    def add(self, systems, strict=True):
        """systems: list of (params, keep, r, v).  Returns their slots (-1 for
        a system that could not be added) and statuses; strict: raise unless
        every system was added."""
        k = len(systems)
        P = (C.POINTER(B.gld_params) * k)(*[C.pointer(s[0]) for s in systems])
        rs = [np.ascontiguousarray(s[2], dtype=np.float64).reshape(-1, 3) for s in systems]
        vs = [np.ascontiguousarray(s[3], dtype=np.float64).reshape(-1, 3) for s in systems]
        R = (C.POINTER(C.c_double) * k)(*[_dp(a) for a in rs])
        V = (C.POINTER(C.c_double) * k)(*[_dp(a) for a in vs])
        slots = (C.c_int32 * k)()
        stat = (C.c_int32 * k)()
        rc = lib().gld_batch_add(self.handle, k, P, R, V, slots, stat)
        if strict:
            _check(rc, "gld_batch_add")
        out = list(slots)
        for s, (p, keep, _, _) in zip(out, systems):
            if s >= 0:
                self.n[s] = p.n
                self.m_max[s] = p.m_max
                self._keep[s] = (p, keep)
        return (out, list(stat)) if not strict else out

    def remove(self, slot):
        _check(lib().gld_batch_remove(self.handle, int(slot)), "gld_batch_remove")
        self.n.pop(slot, None)
        self._keep.pop(slot, None)

    def step(self, n_steps=1):
        _check(lib().gld_batch_step(self.handle, int(n_steps)), "gld_batch_step")

    def sync(self):
        _check(lib().gld_batch_sync(self.handle), "gld_batch_sync")

    def read_state(self, slot, history=False):
        n = self.n[slot]
        out = {k: np.zeros((n, 3)) for k in ("r", "v", "f_c", "f_d", "f_r")}
        hist = np.zeros((max(self.m_max[slot] - 1, 0), n, 3)) if history else None
        st = B.gld_state(r=_dp(out["r"]), v=_dp(out["v"]), f_c=_dp(out["f_c"]), f_d=_dp(out["f_d"]),
                         f_r=_dp(out["f_r"]), history=_dp(hist) if hist is not None and hist.size else None)
        _check(lib().gld_batch_read_state(self.handle, int(slot), C.byref(st)), "gld_batch_read_state")
        out.update(history=hist, step=st.step, flags=st.flags, flag_step=st.flag_step)
        return out

    def write_state(self, slot, r, v, step=0, history=None):
        n = self.n[slot]
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        h = None if history is None else np.ascontiguousarray(history, dtype=np.float64)
        st = B.gld_state(r=_dp(r), v=_dp(v), history=_dp(h) if h is not None and h.size else None, step=int(step))
        _check(lib().gld_batch_write_state(self.handle, int(slot), C.byref(st)), "gld_batch_write_state")

    def noise_info(self, slot):
        o = B.gld_noise_info()
        _check(lib().gld_batch_noise_parameters(self.handle, int(slot), C.byref(o)), "gld_batch_noise_parameters")
        return {f: getattr(o, f) for f, _ in o._fields_}

    def autotune(self, trial_steps=3):
        s = B.gld_batch_schedule()
        ms = (C.c_double * B.GLD_BATCH_CANDIDATES)()
        _check(lib().gld_batch_autotune(self.handle, int(trial_steps), C.byref(s), ms), "gld_batch_autotune")
        return list(s.lanes_threshold), list(ms)

    def set_schedule(self, thresholds):
        s = B.gld_batch_schedule()
        s.lanes_threshold[:] = [int(x) for x in thresholds]
        _check(lib().gld_batch_set_schedule(self.handle, C.byref(s)), "gld_batch_set_schedule")

    def set_timing(self, enable):
        _check(lib().gld_batch_set_timing(self.handle, int(bool(enable))), "gld_batch_set_timing")

    def kernel_times(self):
        ms = (C.c_double * B.GLD_K_COUNT)()
        cnt = (C.c_int64 * B.GLD_K_COUNT)()
        _check(lib().gld_batch_kernel_times(self.handle, ms, cnt), "gld_batch_kernel_times")
        return {B.KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(B.GLD_K_COUNT)}

    def stats(self):
        ns, npart, pairs = C.c_int32(), C.c_int64(), C.c_int64()
        _check(lib().gld_batch_stats(self.handle, C.byref(ns), C.byref(npart), C.byref(pairs)), "gld_batch_stats")
        return ns.value, npart.value, pairs.value

    def system_stats(self, slot):
        """(directed pairs, lanes per particle) of one system."""
        pairs, lanes = C.c_int64(), C.c_int32()
        _check(lib().gld_batch_system_stats(self.handle, int(slot), C.byref(pairs), C.byref(lanes)),
               "gld_batch_system_stats")
        return pairs.value, lanes.value


class Server:
    """Continuous-batching server (include/gld_serve.h): requests are queued
    with their arrival times, then :meth:`run` serves them all."""

    def __init__(self, max_systems, workspace_bytes, chunk_steps=50, thresholds=None, fp64=False, device=None,
                 stream=None):
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        sched = None
        if thresholds is not None:
            sched = B.gld_batch_schedule()
            sched.lanes_threshold[:] = [int(x) for x in thresholds]
        h = C.c_void_p()
        _check(lib().gld_server_create(B.GLD_FP64 if fp64 else B.GLD_FP32_MIXED, int(max_systems),
                                       C.c_void_p(self.workspace.data_ptr()), int(workspace_bytes),
                                       C.c_void_p(self.stream.cuda_stream), int(chunk_steps),
                                       C.byref(sched) if sched is not None else None, C.byref(h)),
               "gld_server_create")
        self.handle = h
        self.n = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().gld_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, params, r, v, steps, arrival_s):
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        rid, foot = C.c_int64(), C.c_size_t()
        _check(lib().gld_server_submit(self.handle, C.byref(params), _dp(r), _dp(v), int(steps), float(arrival_s),
                                       C.byref(rid), C.byref(foot)), "gld_server_submit")
        self.n[rid.value] = params.n
        return rid.value, foot.value

    def run(self):
        _check(lib().gld_server_run(self.handle), "gld_server_run")

    def request(self, rid, state=True):
        info = B.gld_request_info()
        out = None
        st = None
        if state:
            n = self.n[rid]
            out = {k: np.zeros((n, 3)) for k in ("r", "v", "f_c", "f_d", "f_r")}
            st = B.gld_state(r=_dp(out["r"]), v=_dp(out["v"]), f_c=_dp(out["f_c"]), f_d=_dp(out["f_d"]),
                             f_r=_dp(out["f_r"]))
        _check(lib().gld_server_request(self.handle, int(rid), C.byref(info), C.byref(st) if st is not None else None),
               "gld_server_request")
        rec = {f: getattr(info, f) for f, _ in info._fields_}
        if out is not None:
            out.update(step=st.step, flags=st.flags)
        return rec, out

    def stats(self):
        t, k = C.c_double(), C.c_int64()
        _check(lib().gld_server_stats(self.handle, C.byref(t), C.byref(k)), "gld_server_stats")
        return t.value, k.value
