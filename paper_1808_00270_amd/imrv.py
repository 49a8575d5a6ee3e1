"""Iterative memory reconstruction targeting velocity correlations (IMRV).

Sec. III.B of the paper reconstructs the memory kernels iteratively: a GLD
simulation with the current kernel K_n gives a velocity correlation function
Y_n(t), and the kernel is corrected by the difference of a mapping of that
function and the same mapping of the target,

    K_{n+1}(t) = K_n(t) + h_n(t) [ phi(Y_target)(t) - phi(Y_n)(t) ],
    phi(Y)(t)  = -alpha (M^2 / kT) (Y(t + dt) - Y(t)) / dt          (eq. phi),

with a relaxation parameter alpha and a filter h_n(t).  The paper leaves h
open (it refers to earlier work for it); here h is a fixed window, 1 up to a
correction time t_cor and decaying as exp(-(t - t_cor) / t_cor) after it
(t_cor = infinity: h = 1), the same at every iteration.

A kernel is only usable if its noise exists, i.e. if the spectrum of the
discrete correlation sequence (Sec. II.C, eq. FT) is positive.  The
correction of a measured (noisy) correlation function can push that
spectrum below zero at some frequencies; the paper does not say what to do
then.  :func:`reconstruct` projects each corrected kernel onto positive
spectra by default (:func:`project_positive`: the spectrum clipped from
below at a small fraction of its largest value, transformed back).

The driver is host logic around GLD runs: `simulate(k_of_t)` is any callable
that runs the GLD engine with the continuous kernel samples K(m dt),
m = 0..m_max-1, and returns the velocity correlation Y(m dt) it measured
(:func:`gpu_vacf` runs the library's integrator on the GPU).  The continuous
kernel maps onto the library's discrete tables by the trapezoid weights used
throughout (K_0 = dt K(0) / 2, K_m = dt K(m dt)).

:func:`pair_kernels_from_decoupled` is Sec. III.A's last step: the self and
pair kernels from the kernels K_+- of the decoupled two-particle modes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np


def to_table(k_of_t: np.ndarray, dt: float) -> np.ndarray:
    """Continuous kernel samples K(m dt) -> the library's discrete K_m."""
    k = dt * np.asarray(k_of_t, dtype=np.float64)
    k = k.copy()
    k[0] *= 0.5
    return k


def phi(y: np.ndarray, dt: float, mass: float, kT: float, alpha: float) -> np.ndarray:
    """The mapping of eq. (phi) at t = m dt, m = 0..len(y)-2."""
    y = np.asarray(y, dtype=np.float64)
    return -alpha * mass * mass / kT * (y[1:] - y[:-1]) / dt


def window(m_max: int, dt: float, t_cor: float = math.inf) -> np.ndarray:
    t = np.arange(m_max) * dt
    if not math.isfinite(t_cor):
        return np.ones(m_max)
    return np.where(t <= t_cor, 1.0, np.exp(-(t - t_cor) / t_cor))


def spectrum(k_of_t: np.ndarray) -> np.ndarray:
    """S_w = K(0) + 2 sum_{m>=1} K(m dt) cos(2 pi w m / P), w = 0..M-1,
    P = 2M - 1: the DFT of the even continuation of the samples, which is
    kT / dt times the library's per-frequency self spectrum of to_table(K)."""
    k = np.asarray(k_of_t, dtype=np.float64)
    M = len(k)
    P = 2 * M - 1
    c = np.concatenate([k, k[:0:-1]])  # K_0..K_{M-1}, K_{M-1}..K_1: period P
    return np.fft.rfft(c, n=P).real[:M]


def project_positive(k_of_t: np.ndarray, floor: float = 1e-3) -> np.ndarray:
    """The kernel whose spectrum is max(S_w, floor max_w |S_w|): unchanged
    when the spectrum already clears the floor."""
    k = np.asarray(k_of_t, dtype=np.float64)
    M = len(k)
    P = 2 * M - 1
    S = spectrum(k)
    lo = floor * float(np.max(np.abs(S)))
    if np.all(S >= lo):
        return k.copy()
    S = np.maximum(S, lo)
    full = np.concatenate([S, S[:0:-1]])  # even spectrum of period P
    return np.fft.ifft(full).real[:M] * 1.0


@dataclasses.dataclass
class IMRVResult:
    kernels: List[np.ndarray]      # K_n(t_m), n = 0..iterations
    responses: List[np.ndarray]    # Y_n(t_m) of each K_n
    errors: List[float]            # ||Y_n - Y_target|| / ||Y_target|| over the fitted range


def reconstruct(target: np.ndarray, k0: np.ndarray, simulate: Callable[[np.ndarray], np.ndarray], *, dt: float,
                mass: float = 1.0, kT: float = 1.0, alpha: float = 6.0, iterations: int = 20,
                t_cor: float = math.inf, callback: Optional[Callable[[int, np.ndarray, float], None]] = None,
                positive: bool = True) -> IMRVResult:
    """Run `iterations` IMRV corrections from the kernel samples k0 towards
    the target correlation function (target[m] = Y(m dt), at least
    len(k0) + 1 points).  Returns every kernel, its correlation function and
    its error.  positive: project every corrected kernel onto positive
    spectra (project_positive)."""
    m_max = len(k0)
    target = np.asarray(target, dtype=np.float64)
    assert len(target) >= m_max + 1, "the target needs m_max + 1 points"
    h = window(m_max, dt, t_cor)
    phi_t = phi(target[:m_max + 1], dt, mass, kT, alpha)
    k = np.asarray(k0, dtype=np.float64).copy()
    res = IMRVResult([], [], [])
    norm = np.linalg.norm(target[:m_max + 1])
    for it in range(iterations + 1):
        y = np.asarray(simulate(k), dtype=np.float64)[:m_max + 1]
        err = float(np.linalg.norm(y - target[:m_max + 1]) / norm)
        res.kernels.append(k.copy())
        res.responses.append(y)
        res.errors.append(err)
        if callback:
            callback(it, k, err)
        if it == iterations:
            break
        k = k + h * (phi_t - phi(y, dt, mass, kT, alpha))
        if positive:
            k = project_positive(k)
    return res


def pair_kernels_from_decoupled(k_plus: np.ndarray, k_minus: np.ndarray):
    """Sec. III.A: K^s(t) + Delta K^s(R, t) = (K_+ + K_-) / 2 and
    K^p(R, t) = (K_+ - K_-) / 2 from the kernels of the two decoupled modes
    V_+- of a pair at distance R."""
    kp, km = np.asarray(k_plus, dtype=np.float64), np.asarray(k_minus, dtype=np.float64)
    return 0.5 * (kp + km), 0.5 * (kp - km)


def vacf(v: np.ndarray, lags: int) -> np.ndarray:
    """Velocity autocorrelation <v(t + s) . v(t)> / 3 for s = 0..lags-1 from
    velocities v[t, i, c] (every particle and time origin, by FFT)."""
    T = v.shape[0]
    x = v.reshape(T, -1)
    nfft = 1 << int(math.ceil(math.log2(2 * T)))
    f = np.fft.rfft(x, n=nfft, axis=0)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=0)[:lags]
    counts = T - np.arange(lags)
    return ac.sum(axis=1) / counts / (x.shape[1] / 3.0) / 3.0


def gpu_vacf(k_of_t: np.ndarray, *, n: int = 4096, dt: float = 0.01, mass: float = 1.0, kT: float = 1.0,
             steps: int = 3000, burn_in: int = 500, lags: Optional[int] = None, seed: int = 7,
             fp64: bool = False) -> np.ndarray:
    """Velocity autocorrelation of N non-interacting particles (no pair memory,
    no conservative force) with the self kernel K(t) = k_of_t, integrated by
    the library on the GPU; every particle then follows the single-particle
    GLE, so the average over particles and time origins is the
    single-particle correlation function."""
    from . import System
    m_max = len(k_of_t)
    lags = lags or (m_max + 1)
    box = 40.0  # non-interacting: any box holding the cutoff
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.0, box, size=(n, 3))
    V = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 3))
    s = System(n=n, box=box, dt=dt, mass=mass, kT=kT, k_self=to_table(k_of_t, dt), r=R, v=V, wca_eps=0.0,
               seed=seed, fp64=fp64, r_cut=5.0, verlet_skin=0.5)
    s.step(burn_in)
    vs = np.empty((steps, n, 3))
    for t in range(steps):
        s.step(1)
        vs[t] = s.read_state()["v"]
    s.close()
    return vacf(vs, lags)
