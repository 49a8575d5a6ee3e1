"""Seeded synthetic GLD workloads: kernel tables, boxes and initial states.

This module holds input generation only (no part of the integrator, the
memory convolution or the noise construction).  Both the HIP path and the
CPU oracle receive the arrays it produces.

Kernel shapes (self and separable pair memory) follow the synthetic
benchmark definitions; the paper's own kernels were reconstructed from
molecular dynamics data that is not available, so these stand in for them.

* self kernel      K^s(t)   = 10 exp(-t/0.5) cos(4 t)
* pair kernel      K^p(r,t) = w(r) g(t),  w(r) = (1 - r/r_c)^2,
                   g(t) = 3 exp(-t/0.3) cos(5 t)
* discrete tables  K_0 = dt K(0) / 2, K_m = dt K(m dt) (trapezoid weights,
                   so that kT a_m K_m / dt = kT K(m dt), the FDT target)
* initial state    simple-cubic lattice (n_side = ceil(N^(1/3)), x fastest,
                   first N sites) with uniform jitter +-0.1 per coordinate;
                   Maxwell velocities N(0, kT/M) per component.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def self_kernel(t):
    return 10.0 * np.exp(-t / 0.5) * np.cos(4.0 * t)


def pair_time_kernel(t):
    return 3.0 * np.exp(-t / 0.3) * np.cos(5.0 * t)


def pair_weight(r, r_cut):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < r_cut, (1.0 - r / r_cut) ** 2, 0.0)


def discretize(kernel, dt, m_max):
    """Trapezoid map of a continuous memory kernel onto the lags m = 0..m_max-1."""
    t = np.arange(m_max) * dt
    k = dt * kernel(t)
    k[0] *= 0.5
    return k


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    rho: float
    m_max: int
    steps: int
    dt: float = 0.01
    mass: float = 1.0
    kT: float = 1.0
    r_cut: float = 5.0
    n_r: int = 501
    wca_sigma: float = 1.0
    wca_eps: float = 1.0
    seed: int = 0
    parallel: bool = False

    @property
    def box(self) -> float:
        return (self.n / self.rho) ** (1.0 / 3.0)

    def tables(self):
        """(k_self[m_max], g[m_max], w[n_r], r0, dr): separable pair kernel."""
        k_self = discretize(self_kernel, self.dt, self.m_max)
        g = discretize(pair_time_kernel, self.dt, self.m_max)
        dr = self.r_cut / (self.n_r - 1)
        r = np.arange(self.n_r) * dr
        w = pair_weight(r, self.r_cut)
        w[-1] = 0.0
        return k_self, g, w, 0.0, dr

    def k_pair_table(self):
        """General table K^p_m(r_b) = w_b g_m (outer product), shape [n_r, m_max]."""
        _, g, w, _, _ = self.tables()
        return np.outer(w, g)

    def initial_state(self):
        rng = np.random.default_rng(self.seed)
        L = self.box
        ns = int(math.ceil(self.n ** (1.0 / 3.0) - 1e-9))
        a = L / ns
        idx = np.arange(self.n)
        lat = np.stack([idx % ns, (idx // ns) % ns, idx // (ns * ns)], axis=1).astype(np.float64)
        R = lat * a + rng.uniform(-0.1, 0.1, size=(self.n, 3))
        V = rng.normal(0.0, math.sqrt(self.kT / self.mass), size=(self.n, 3))
        return R, V


def slab_state(w: Workload, frac: float):
    """All particles in the slab z < frac L (density rho / frac there, empty
    elsewhere): a simple lattice of n_xy x n_xy x n_z sites filled in order,
    jittered +-0.1; Maxwell velocities as in Workload.initial_state."""
    rng = np.random.default_rng(w.seed + 7)
    L = w.box
    nxy = int(math.ceil((w.n / frac) ** (1.0 / 3.0) - 1e-9))
    nz = int(math.ceil(w.n / (nxy * nxy)))
    idx = np.arange(w.n)
    R = np.stack([(idx % nxy) * (L / nxy), ((idx // nxy) % nxy) * (L / nxy),
                  (idx // (nxy * nxy)) * (frac * L / nz)], axis=1)
    R += rng.uniform(-0.1, 0.1, size=(w.n, 3))
    V = rng.normal(0.0, math.sqrt(w.kT / w.mass), size=(w.n, 3))
    return R, V


def config(k: int, **over) -> Workload:
    """The synthetic configurations (1-based, as listed in the benchmark set).

    1: N=64,     rho=0.05, m_max=200,  1000 steps   (parity, statistics)
    2: N=10^4,   rho=0.05, m_max=500,  10^4 steps   (single GPU, cache resident)
    3: N=2x10^5, rho=0.5,  m_max=1000, 10^3 steps   (headline, HBM bound)
    """
    table = {
        1: dict(name="cfg1_n64_rho0.05_m200", n=64, rho=0.05, m_max=200, steps=1000),
        2: dict(name="cfg2_n1e4_rho0.05_m500", n=10_000, rho=0.05, m_max=500, steps=10_000),
        3: dict(name="cfg3_n2e5_rho0.5_m1000", n=200_000, rho=0.5, m_max=1000, steps=1000),
    }
    d = dict(table[k])
    d["seed"] = 1000 + k
    d.update(over)
    return Workload(**d)


def random_history(rng, m_max, n, scale=0.01):
    """A seeded displacement history dR_{n-m}, m = 1..m_max-1, shape [m_max-1, n, 3]."""
    return rng.normal(0.0, scale, size=(max(m_max - 1, 0), n, 3))


def batch_system(i: int, attempt: int = 0) -> "Workload":
    """System i of the batched benchmark (256 independent systems): N
    log-uniform in [100, 2e4], density uniform in [0.005, 0.5], m_max from
    {200, 500, 1000}, the self and pair kernels scaled by independent factors
    uniform in [0.5, 2]; seeded by (2000 + i, attempt).  A draw whose box is
    below 10 (r_c = 5 needs L > 2 r_c) is drawn again with the next attempt;
    so is one that the library reports not positive definite (the caller
    passes the attempt)."""
    while True:
        rng = np.random.default_rng([2000 + i, attempt])
        n = int(round(math.exp(rng.uniform(math.log(100.0), math.log(2e4)))))
        rho = float(rng.uniform(0.005, 0.5))
        m_max = int(rng.choice([200, 500, 1000]))
        fs, fp = (float(x) for x in rng.uniform(0.5, 2.0, size=2))
        w = ScaledWorkload(name=f"batch{i}", n=n, rho=rho, m_max=m_max, steps=1000, seed=2000 + i,
                           f_self=fs, f_pair=fp)
        if w.box > 10.0:
            w.attempt = attempt
            return w
        attempt += 1


@dataclasses.dataclass
class ScaledWorkload(Workload):
    """A workload whose self and pair kernels are scaled by f_self and f_pair."""
    f_self: float = 1.0
    f_pair: float = 1.0
    attempt: int = 0

    def tables(self):
        k_self, g, w, r0, dr = super().tables()
        return self.f_self * k_self, self.f_pair * g, w, r0, dr


def serve_requests(count: int, steps_scale: float = 1.0, seed: int = 5000):
    """The first `count` requests of the serving workload: Poisson arrivals at
    20 per second, N log-uniform in [64, 5e4], steps log-uniform in
    [1e3, 1e5] (times steps_scale, at least 1), m_max from {200, 500, 1000},
    density uniform in [0.005, 0.5] (a box below 10 is drawn again).
    Returns [(arrival_s, steps, Workload)]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / 20.0))
        steps = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e5))) * steps_scale))
        while True:
            n = int(round(math.exp(rng.uniform(math.log(64.0), math.log(5e4)))))
            rho = float(rng.uniform(0.005, 0.5))
            m_max = int(rng.choice([200, 500, 1000]))
            w = Workload(name=f"req{i}", n=n, rho=rho, m_max=m_max, steps=steps, seed=seed + 1 + i)
            if w.box > 10.0:
                break
        out.append((t, max(1, steps), w))
    return out


def general_tables(m_max: int, n_r: int, r_cut: float, dt: float, pair2: float = 0.3, dk: float = 2.0,
                   f_pair: float = 1.0, t_scale: float = 1.0):
    """Tables of the general memory model (a pair kernel of rank two and a
    distance-dependent self memory) on the grid r_b = b r_cut / (n_r - 1):

    * K^s(t)      = self_kernel(t)
    * K^p(r, t)   = f_pair [w(r) g(t) + pair2 w2(r) g2(t)],  w, g as above,
                    w2(r) = 4 (r/r_c)(1 - r/r_c) (largest at r_c/2),
                    g2(t) = exp(-t/0.15)
    * dK^s(r, t)  = (dk / 10) w(r) K^s(t)

    t_scale < 1 compresses every kernel in time, K(t) -> K(t / t_scale)
    (for short memories: a kernel cut off well before it has decayed can
    have a non-positive spectrum).

    Returns (k_self[m_max], k_pair[n_r][m_max], dk_self[n_r][m_max] or None,
    r0 = 0, dr); the last grid point is zeroed like the separable tables."""
    dr = r_cut / (n_r - 1)
    r = np.arange(n_r) * dr
    x = np.clip(r / r_cut, 0.0, 1.0)
    w = (1.0 - x) ** 2
    w2 = 4.0 * x * (1.0 - x)
    w[-1] = 0.0
    w2[-1] = 0.0
    ts = float(t_scale)
    k_self = discretize(lambda t: self_kernel(t / ts), dt, m_max)
    g = discretize(lambda t: pair_time_kernel(t / ts), dt, m_max)
    g2 = discretize(lambda t: np.exp(-t / (0.15 * ts)), dt, m_max)
    k_pair = f_pair * (np.outer(w, g) + pair2 * np.outer(w2, g2))
    dks = np.outer(w, (dk / 10.0) * k_self) if dk else None
    return k_self, k_pair, dks, 0.0, dr
