"""ctypes front end of the FP64 CPU oracle (``gld_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` import this
module.  It shares nothing with the HIP path of the package.

The C source follows the paper (arXiv:1808.00270) section by section; see
its header for the equations covered and the readings taken.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gld_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_ERR_INVALID, ORC_ERR_NOT_PD, ORC_ERR_NO_CONV, ORC_ERR_OOM = 0, -1, -2, -3, -5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3 without fast-math: IEEE semantics and
    the source's order of every floating-point operation; OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=c99", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("dt", C.c_double), ("mass", C.c_double), ("kT", C.c_double),
        ("m_max", C.c_int32), ("n_r", C.c_int32),
        ("k_self", C.POINTER(C.c_double)),
        ("k_pair", C.POINTER(C.c_double)),
        ("r0", C.c_double), ("dr", C.c_double),
        ("r_cut", C.c_double), ("r_cut_min", C.c_double),
        ("parallel", C.c_int32), ("lanczos_max_iter", C.c_int32),
        ("wca_sigma", C.c_double), ("wca_eps", C.c_double),
        ("seed", C.c_uint64),
        ("lanczos_tol", C.c_double),
        ("dk_self", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # GLD_ORACLE_LIB lets a mutation check load a deliberately altered build
        _lib = C.CDLL(os.environ.get("GLD_ORACLE_LIB") or build())
        d = C.POINTER(C.c_double)
        P = C.POINTER(OrcParams)
        _lib.orc_create.restype = C.c_void_p
        _lib.orc_create.argtypes = [P]
        _lib.orc_destroy.argtypes = [C.c_void_p]
        _lib.orc_step.argtypes = [C.c_void_p, C.c_int64, d, d, d, d, d, d, d, d]
        _lib.orc_noise.argtypes = [C.c_void_p, C.c_int64, d, C.POINTER(C.c_uint32), C.c_int, C.c_int, d]
        _lib.orc_noise_dense_freq.argtypes = [C.c_void_p, C.c_int64, d, d]
        _lib.orc_noise_dense_time.argtypes = [C.c_void_p, C.c_int64, d, d]
        _lib.orc_dense_filters.argtypes = [C.c_void_p, d, d]
        _lib.orc_dense_sqrt_spectra.argtypes = [C.c_void_p, d, d, d]
        _lib.orc_corr_matrix.argtypes = [C.c_void_p, d, C.c_int, d]
        _lib.orc_spectra.argtypes = [C.c_void_p, d, d]
        _lib.orc_forces_rows.argtypes = [C.c_void_p, d, d, d, C.POINTER(C.c_int64), C.c_int64, d, d]
        _lib.orc_pairs.argtypes = [P, d, C.c_int, C.c_int64, C.POINTER(C.c_int64), d, C.POINTER(C.c_int64)]
        _lib.orc_wca_energy.restype = C.c_double
        _lib.orc_wca_energy.argtypes = [P, d]
        _lib.orc_wca_forces.argtypes = [P, d, d]
        _lib.orc_ab.argtypes = [P, d, d]
        _lib.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        _lib.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, d]
        _lib.orc_tridiag_eig.argtypes = [C.c_int, d, d, d]
        _lib.orc_last_iters.argtypes = [C.c_void_p]
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int]
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(rc: int, what: str):
    if rc != ORC_OK:
        raise OracleError(rc, what)


class Oracle:
    """One GLD system description for the oracle.

    ``k_self[m]``: K^s_m; ``k_pair[b, m]``: K^p_m(r0 + b dr) (general table;
    a separable kernel is passed as the outer product w_b g_m).
    """

    def __init__(self, *, n, box, dt, mass, kT, k_self, k_pair, r0, dr, r_cut,
                 r_cut_min=0.0, parallel=False, wca_sigma=1.0, wca_eps=1.0, seed=0,
                 lanczos_tol=1e-13, lanczos_max_iter=300, dk_self=None):
        box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
        self.k_self = np.ascontiguousarray(k_self, dtype=np.float64)
        self.k_pair = np.ascontiguousarray(k_pair, dtype=np.float64)
        self.dk_self = None if dk_self is None else np.ascontiguousarray(dk_self, dtype=np.float64)
        m_max = self.k_self.shape[0]
        assert self.k_pair.ndim == 2 and self.k_pair.shape[1] == m_max
        assert self.dk_self is None or self.dk_self.shape == self.k_pair.shape
        self.n, self.m_max, self.n_r = int(n), int(m_max), int(self.k_pair.shape[0])
        self.p = OrcParams(
            n=self.n, box=(C.c_double * 3)(*box), dt=dt, mass=mass, kT=kT,
            m_max=self.m_max, n_r=self.n_r, k_self=_dp(self.k_self), k_pair=_dp(self.k_pair),
            r0=r0, dr=dr, r_cut=r_cut, r_cut_min=r_cut_min, parallel=int(bool(parallel)),
            lanczos_max_iter=int(lanczos_max_iter), wca_sigma=wca_sigma, wca_eps=wca_eps,
            seed=int(seed) & 0xFFFFFFFFFFFFFFFF, lanczos_tol=lanczos_tol,
            dk_self=_dp(self.dk_self) if self.dk_self is not None else None)
        self.box = np.array(box)
        self.ctx = lib().orc_create(C.byref(self.p))
        if not self.ctx:
            raise OracleError(ORC_ERR_INVALID, "create")

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().orc_destroy(self.ctx)
            self.ctx = None

    # -- integrator -----------------------------------------------------
    def ab(self):
        a, b = C.c_double(), C.c_double()
        lib().orc_ab(C.byref(self.p), C.byref(a), C.byref(b))
        return a.value, b.value

    def step(self, step, R, V, hist):
        """Advance (R, V, hist) in place by one step; returns (FC, FD, FR) of step n."""
        n3 = 3 * self.n
        FC, FD, FR = (np.zeros(n3) for _ in range(3))
        tfd, tfr = C.c_double(), C.c_double()
        _check(lib().orc_step(self.ctx, int(step), _dp(R), _dp(V), _dp(hist), _dp(FC), _dp(FD), _dp(FR),
                              C.byref(tfd), C.byref(tfr)), "step")
        self.t_fd, self.t_fr = tfd.value, tfr.value
        return FC.reshape(-1, 3), FD.reshape(-1, 3), FR.reshape(-1, 3)

    def empty_history(self):
        return np.zeros((max(self.m_max - 1, 0), self.n, 3))

    # -- forces ----------------------------------------------------------
    def noise(self, step, R, ids=None, w0=0, w1=None):
        w1 = self.m_max if w1 is None else w1
        FR = np.zeros(3 * self.n)
        idp = None
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.uint32)
            idp = ids.ctypes.data_as(C.POINTER(C.c_uint32))
        _check(lib().orc_noise(self.ctx, int(step), _dp(np.ascontiguousarray(R, dtype=np.float64)), idp,
                               int(w0), int(w1), _dp(FR)), "noise")
        return FR.reshape(-1, 3)

    def last_iters(self):
        return lib().orc_last_iters(self.ctx)

    def noise_dense_freq(self, step, R):
        FR = np.zeros(3 * self.n)
        _check(lib().orc_noise_dense_freq(self.ctx, int(step), _dp(np.ascontiguousarray(R)), _dp(FR)), "dense noise")
        return FR.reshape(-1, 3)

    def noise_dense_time(self, step, R):
        FR = np.zeros(3 * self.n)
        _check(lib().orc_noise_dense_time(self.ctx, int(step), _dp(np.ascontiguousarray(R)), _dp(FR)), "dense noise")
        return FR.reshape(-1, 3)

    def dense_filters(self, R):
        n3 = 3 * self.n
        A = np.zeros((2 * self.m_max - 1, n3, n3))
        _check(lib().orc_dense_filters(self.ctx, _dp(np.ascontiguousarray(R)), _dp(A)), "filters")
        return A

    def dense_sqrt_spectra(self, R):
        n3 = 3 * self.n
        A = np.zeros((self.m_max, n3, n3))
        lmin = C.c_double()
        rc = lib().orc_dense_sqrt_spectra(self.ctx, _dp(np.ascontiguousarray(R)), _dp(A), C.byref(lmin))
        return rc, A, lmin.value

    def corr_matrix(self, R, m):
        n3 = 3 * self.n
        K = np.zeros((n3, n3))
        _check(lib().orc_corr_matrix(self.ctx, _dp(np.ascontiguousarray(R)), int(m), _dp(K)), "corr matrix")
        return K

    def spectra(self):
        S = np.zeros(self.m_max)
        Kp = np.zeros((self.n_r, self.m_max))
        lib().orc_spectra(self.ctx, _dp(S), _dp(Kp))
        return S, Kp

    def forces_rows(self, R, V, hist, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        FC = np.zeros((len(rows), 3))
        FD = np.zeros((len(rows), 3))
        _check(lib().orc_forces_rows(self.ctx, _dp(R), _dp(V), _dp(hist),
                                     rows.ctypes.data_as(C.POINTER(C.c_int64)), len(rows), _dp(FC), _dp(FD)),
               "forces_rows")
        return FC, FD

    def wca_forces(self, R):
        F = np.zeros(3 * self.n)
        _check(lib().orc_wca_forces(C.byref(self.p), _dp(np.ascontiguousarray(R)), _dp(F)), "wca")
        return F.reshape(-1, 3)

    def wca_energy(self, R):
        return lib().orc_wca_energy(C.byref(self.p), _dp(np.ascontiguousarray(R)))

    def pairs(self, R, use_cells=False, cap=None):
        cap = cap or max(1024, self.n * 600)
        ij = np.zeros(2 * cap, dtype=np.int64)
        r = np.zeros(cap)
        cnt = C.c_int64()
        _check(lib().orc_pairs(C.byref(self.p), _dp(np.ascontiguousarray(R)), int(use_cells), cap,
                               ij.ctypes.data_as(C.POINTER(C.c_int64)), _dp(r), C.byref(cnt)), "pairs")
        k = cnt.value
        return ij[:2 * k].reshape(-1, 2), r[:k]


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def gauss3(seed, pid, t):
    z = np.zeros(3)
    lib().orc_gauss3(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(pid), int(t), _dp(z))
    return z


def tridiag_eig(d, e):
    d = np.array(d, dtype=np.float64)
    e = np.array(list(e) + [0.0], dtype=np.float64)
    n = len(d)
    Q = np.zeros(n * n)
    rc = lib().orc_tridiag_eig(n, _dp(d), _dp(e), _dp(Q))
    _check(rc, "tridiag_eig")
    return d, Q.reshape(n, n)


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    """Threads of the oracle's OpenMP loops (1: single core)."""
    lib().orc_set_threads(int(n))
