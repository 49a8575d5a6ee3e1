"""Element-wise parity at the noise plan the benchmark runs.

The benchmark system (N = 2e5, rho = 0.5, m_max = 1000) is too large for the
oracle's Algorithm 1 on every particle; the noise plan, however, depends on
the density, the memory and the tolerance, not on N.  At N = 1200 and the
same density and memory the library builds the same plan shape (rank 6,
Chebyshev terms 27 tight / 33 wide, filter block 10, window h = 699 in
FP32-mixed at the default tolerance 4e-6; rank 13, K 69 / 86, h = 999 in
FP64 at the default 1e-12), so these tests compare, particle by particle,
exactly the noise construction the benchmark times:

* one step on the tight plan (the lattice start) and on the wide plan (a
  compressed slab whose row-sum bound lies between the two plans' upper
  ends), in both precisions at their default noise tolerances;
* a run written two steps before a step where both the history's block
  product (blocks of 32 steps in FP32, 16 in FP64) and the filter bank
  (blocks of 10 and 4 steps) start a new block by themselves (160 and 32),
  without the forced products that gld_write_state runs, and stepped past
  it; every step is compared with one oracle step from the GPU's own state.

Tolerances as in the other parity tests: 1e-12 (FP64) and 1e-5 (FP32-mixed),
normwise relative plus an element-wise bound.
"""
import math
import sys

import numpy as np
import pytest

from paper_1808_00270_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {True: 1e-12, False: 1e-5}
N = 1200


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


def workload():
    return wl.config(3, n=N)


def oracle_for(oracle_mod, w):
    k_self, g, wt, r0, dr = w.tables()
    return oracle_mod.Oracle(n=w.n, box=w.box, dt=w.dt, mass=w.mass, kT=w.kT, k_self=k_self,
                             k_pair=np.outer(wt, g), r0=r0, dr=dr, r_cut=w.r_cut, wca_sigma=w.wca_sigma,
                             wca_eps=w.wca_eps, seed=w.seed, lanczos_tol=1e-13, lanczos_max_iter=400)


def assert_close(name, a, b, tol, atol=0.0):
    d = np.abs(a - b)
    nb = np.linalg.norm(b)
    r = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)
    rms = math.sqrt(np.mean(b ** 2)) if b.size else 0.0
    emax = d.max() / rms if rms > 0 else d.max()
    log(f"    {name}: rel {r:.2e}  max/rms {emax:.2e}")
    assert np.linalg.norm(a - b) <= tol * nb + atol * math.sqrt(b.size), f"{name}: rel {r:.3e} > {tol:.1e}"
    assert np.all(d <= 10 * tol * rms + atol), f"{name}: element error {emax:.3e} > {10 * tol:.1e} (x rms)"


def row_sum_bound(w, R):
    d = R[:, None, :] - R[None, :, :]
    d -= w.box * np.round(d / w.box)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    return wl.pair_weight(r, w.r_cut).sum(1).max()


def compare_step(o, s, fp64, step, R, V, hist, what):
    """One GPU step from the state just written/reached against one oracle step."""
    tol = TOL[fp64]
    s.step(1)
    g = s.read_state(history=True)
    Ro, Vo, Ho = R.copy(), V.copy(), hist.copy()
    _, FD, FR = o.step(step, Ro, Vo, Ho)
    atol = 4 * np.finfo(np.float64).eps * max(np.abs(R).max(), 1.0)
    assert_close(f"{what} F^D'", g["f_d"], FD, tol)
    assert_close(f"{what} F^R", g["f_r"], FR, tol)
    assert_close(f"{what} dR", g["r"] - R, Ro - R, tol, atol)
    assert_close(f"{what} dV", g["v"] - V, Vo - V, tol, atol)
    assert_close(f"{what} history lag 1", g["history"][0], Ho[0], tol, atol)
    assert g["step"] == step + 1
    return g


@pytest.mark.parametrize("fp64", [False, True])
def test_headline_plan_tight_and_wide_one_step(pkg, oracle_mod, fp64):
    w = workload()
    R, V = w.initial_state()
    log(f"  headline plan N={w.n} rho={w.rho} m_max={w.m_max} fp64={fp64} (default noise tolerance)")
    s = pkg.System.from_workload(w, fp64=fp64)
    info = s.noise_info()
    log(f"    plan: K {info['cheb_terms']} / tight {info['cheb_terms_tight']}, rank {info['rank']}, "
        f"block {info['block']}, h {info['window_half']}, err {info['err_estimate']:.2e}, "
        f"[{info['lam_lo']:.3f}, {info['lam_hi']:.3f}] tight up to {info['lam_hi_tight']:.3f}")
    # the benchmark's plan shape
    if fp64:
        assert (info["rank"], info["window_half"]) == (13, 999)
        assert info["err_estimate"] < 1e-12
    else:
        assert info["rank"] == 6 and 600 <= info["window_half"] <= 760
        assert info["err_estimate"] < 4e-6
    assert 0 < info["cheb_terms_tight"] < info["cheb_terms"]
    o = oracle_for(oracle_mod, w)
    hist = wl.random_history(np.random.default_rng(21), w.m_max, w.n, scale=0.01)
    s.write_state(R, V, step=7, history=hist)
    t0 = s.noise_info()["tight_steps"]
    compare_step(o, s, fp64, 7, R, V, hist, "tight")
    assert s.noise_info()["tight_steps"] == t0 + 1
    # a compressed slab whose row-sum bound lies between the two plans' upper ends
    for frac in (0.85, 0.8, 0.75, 0.7):
        Rs, Vs = wl.slab_state(w, frac)
        gs = row_sum_bound(w, Rs)
        log(f"    slab {frac}: row-sum bound {gs:.3f}")
        if info["lam_hi_tight"] < gs < info["lam_hi"]:
            break
    else:
        pytest.fail("no slab with a row-sum bound between the two plans")
    s.write_state(Rs, Vs, step=12, history=hist)
    t1 = s.noise_info()["tight_steps"]
    s.step(1)
    assert s.noise_info()["tight_steps"] == t1
    assert_close("wide F^R", s.read_state()["f_r"], o.noise(12, Rs), TOL[fp64])
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_headline_plan_steps_through_unforced_block_starts(pkg, oracle_mod, fp64):
    w = workload()
    R, V = w.initial_state()
    log(f"  block starts N={w.n} rho={w.rho} m_max={w.m_max} fp64={fp64}")
    s = pkg.System.from_workload(w, fp64=fp64)
    info = s.noise_info()
    # the first step past 0 where the history's block (32 or 16 steps) and the
    # filter block both start
    b0 = math.lcm(32, info["block"])
    log(f"    filter block {info['block']}: both blocks start at step {b0}")
    o = oracle_for(oracle_mod, w)
    hist = wl.random_history(np.random.default_rng(22), w.m_max, w.n, scale=0.01)
    s.write_state(R, V, step=b0 - 2, history=hist)
    cur = s.read_state(history=True)
    for step in range(b0 - 2, b0 + 2):
        nxt = compare_step(o, s, fp64, step, cur["r"], cur["v"], cur["history"], f"step {step}")
        cur = nxt
    s.close()
