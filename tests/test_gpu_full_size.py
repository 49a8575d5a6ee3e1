"""GPU parity at the benchmark sizes.

cfg2 (N = 1e4, m_max = 500): the FP64 GPU path runs from the initial state;
at steps 0, 10 and 100 its state (positions, velocities, history ring) is
handed to a fresh GPU system of each precision and to the oracle, and one
step is compared in full (F^D', F^R, the state increments).

cfg3 (N = 2e5, m_max = 1000, the benchmark workload and launch shape): the
oracle cannot run a whole step in test time, so the check is on outputs it
computes one by one and on properties that hold at any size:
  - F^C and F^D' of sampled particles against the oracle, at R_n and R_{n+1};
  - the position and velocity update of every particle against
    eq. (GLD_integrator) evaluated with the step's own forces;
  - the colored noise of every particle: its per-component variance equals
    the lag-0 correlation kT a_0 K^s_0 / dt and its covariance between
    neighbours equals kT a_0 g_0 / dt w(R_ij) (eq. stochastic_force2); with
    6e5 components and 5e7 pairs the sampling error is a fraction of a percent.
"""
import math

import numpy as np
import pytest

from paper_1808_00270_amd import workloads as wl
from test_gpu_parity import TOL, assert_close, log, one_step, oracle_for, pkg  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("step", [0, 10, 100])
def test_cfg2_one_step_from_gpu_fp64_state(pkg, oracle_mod, step):
    w = wl.config(2)
    R, V = w.initial_state()
    hist = np.zeros((w.m_max - 1, w.n, 3))
    if step > 0:
        log(f"  cfg2: FP64 GPU run to step {step}")
        s = pkg.System.from_workload(w, fp64=True, noise_tol=1e-13)
        s.step(step)
        st = s.read_state(history=True)
        s.close()
        assert st["step"] == step
        R, V, hist = st["r"], st["v"], st["history"]
    for fp64 in (True, False):
        one_step(pkg, oracle_mod, w, fp64, step=step, state=(R, V), hist=hist)


def _full_size_state(w, seed=21):
    R, V = w.initial_state()
    rng = np.random.default_rng(seed)
    # a seeded displacement history of the size of the ring (2.4 / 4.8 GB)
    hist = rng.standard_normal(size=(w.m_max - 1, w.n, 3))
    hist *= 0.01
    return R, V, hist


@pytest.mark.parametrize("fp64", [True, False])
def test_cfg3_full_size_rows_update_and_noise_moments(pkg, oracle_mod, fp64):
    w = wl.config(3)
    step = 9
    log(f"  cfg3 full size, fp64={fp64}: building the state")
    R, V, hist = _full_size_state(w)
    s = pkg.System.from_workload(w, fp64=fp64, r=R, v=V)
    s.write_state(R, V, step=step, history=hist)
    FC0 = s.read_state()["f_c"]
    s.step(1)
    g = s.read_state()
    s.close()
    assert g["step"] == step + 1
    tol = TOL[fp64]
    o = oracle_for(oracle_mod, w)
    rows = np.sort(np.random.default_rng(5).choice(w.n, size=300, replace=False))
    log("  oracle rows at R_n")
    FCo, FDo = o.forces_rows(R, V, hist, rows)
    assert_close("F^C rows (R_n)", FC0[rows], FCo, 1e-12)
    assert_close("F^D' rows", g["f_d"][rows], FDo, tol)
    # F^C at the new positions, same rows
    FCo1, _ = o.forces_rows(g["r"], g["v"], hist, rows)
    assert_close("F^C rows (R_n+1)", g["f_c"][rows], FCo1, 1e-12)
    # eq. (GLD_integrator) with the step's own forces, every particle
    a, b = o.ab()
    dt, M = w.dt, w.mass
    dR = dt * b * V + dt * dt / (2 * M) * b * (FC0 + g["f_d"] + g["f_r"])
    dV = (a - 1.0) * V + dt / (2 * M) * (a * FC0 + g["f_c"]) + dt / M * b * (g["f_d"] + g["f_r"])
    atol = 4 * np.finfo(np.float64).eps * np.abs(R).max()
    assert_close("dR (update)", g["r"] - R, dR, 1e-12, atol)
    assert_close("dV (update)", g["v"] - V, dV, 1e-12, atol)
    # colored noise moments at lag 0
    k_self, gk, wt, r0, dr = w.tables()
    c0 = w.kT * 2.0 * k_self[0] / dt   # a_0 = 2
    cp0 = w.kT * 2.0 * gk[0] / dt
    F = g["f_r"]
    var = float(np.mean(F * F))
    se_var = c0 * math.sqrt(2.0 / F.size) * 1.5   # neighbour correlations inflate it (< 1.5x here)
    log(f"    noise variance {var:.5f} vs {c0:.5f} (+- {se_var:.5f})")
    assert abs(var - c0) < 5 * se_var
    log("  oracle pair list at R_n")
    ij, r = o.pairs(R, use_cells=True, cap=300 * w.n)  # ordered pairs, both directions
    wij = np.interp(r, r0 + dr * np.arange(len(wt)), wt)
    prod = np.sum(F[ij[:, 0]] * F[ij[:, 1]], axis=1)
    sw2 = float(np.sum(wij * wij))
    est = float(np.sum(wij * prod)) / (3.0 * sw2)
    # independent-pair error, x3 for the ordered duplicates and for pairs that
    # share a particle (correlated products)
    se = math.sqrt(3.0 * (c0 * c0 + cp0 * cp0) * sw2) / (3.0 * sw2) * 3.0
    log(f"    neighbour covariance / w: {est:.5f} vs {cp0:.5f} (+- {se:.5f}), {len(r)} pairs")
    assert abs(est - cp0) < 5 * se


def test_cfg3_run_keeps_the_tight_noise_plan(pkg):
    """Over 300 steps from the lattice start (the benchmark's run), the
    largest row sum of |w| stays below the tight plan's upper end at every
    step: each chain uses the shorter expansion (the wide one would be exact
    too, only slower), and nothing is latched."""
    w = wl.config(3)
    s = pkg.System.from_workload(w)
    info = s.noise_info()
    log(f"  tight plan K {info['cheb_terms_tight']} up to {info['lam_hi_tight']:.3f} (wide K {info['cheb_terms']})")
    assert 0 < info["cheb_terms_tight"] < info["cheb_terms"]
    t0 = info["tight_steps"]
    s.step(300)
    st = s.read_state()
    assert st["status"] == 0 and st["step"] == 300
    assert s.noise_info()["tight_steps"] - t0 == 300
    s.close()
