"""Run-time guards of the colored noise (Sec. II.B: positive definiteness is
checked on the fly; the paper's algorithm fails when it is lost, as it
reports at high density in Sec. IV).

The Chebyshev route needs the spectrum of the pair-weight matrix P inside the
noise interval [lam_lo, lam_hi]; every step's pair refresh checks the
Gershgorin row-sum bound against lam_hi, a Lanczos check every
check_interval steps checks the extreme Ritz values against both ends and
against the singular points of the correlation, and gld_write_state checks
a written configuration the same way.  These tests drive two particles
towards each other (WCA off, so that they pass freely) and require each
guard to latch its status at the right step:

  P = [[0, w], [w, 0]] (x) 1_3 for two particles within r_c, eigenvalues +-w,
  row sum w, w = (1 - r / r_c)^2 growing as the pair closes in.

The expected step is read off the oracle's trajectory of the same system
(the FP64 CPU oracle, stepped from the same state with the same white
noise), and the NOT_PD verdict is confirmed by the oracle's Algorithm 1 on
the configuration the check saw.
"""
import math
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


M_MAX, DT, RC, BOX = 60, 0.01, 5.0, 12.0


def tables(g_scale=1.0):
    k_self = wl.discretize(wl.self_kernel, DT, M_MAX)
    g = g_scale * wl.discretize(wl.pair_time_kernel, DT, M_MAX)
    n_r = 501
    dr = RC / (n_r - 1)
    w = wl.pair_weight(np.arange(n_r) * dr, RC)
    w[-1] = 0.0
    return k_self, g, w, 0.0, dr


def singular_point(k_self, g, kT=1.0):
    """Largest lambda at which S_w + G_w lambda vanishes for some frequency:
    S_w, G_w are the length-(2 m_max - 1) cosine transforms of the correlation
    sequences kT a_m K_m / dt (eq. stochastic_force2, a_0 = 2, a_m = 1)."""
    M = len(k_self)
    P = 2 * M - 1
    a = np.ones(M)
    a[0] = 2.0
    cs, cg = kT * a * k_self / DT, kT * a * g / DT
    m = np.arange(1, M)
    S, G = [], []
    for om in range(M):
        c = np.cos(2 * np.pi * om * m / P)
        S.append(cs[0] + 2 * (cs[1:] * c).sum())
        G.append(cg[0] + 2 * (cg[1:] * c).sum())
    S, G = np.array(S), np.array(G)
    return max(-s / q for s, q in zip(S, G) if q > 0)


def pair_state(r_init, speed):
    R = np.array([[3.0, 6.0, 6.0], [3.0 + r_init, 6.0, 6.0]])
    V = np.array([[speed, 0.0, 0.0], [-speed, 0.0, 0.0]])
    return R, V


def make(pkg, fp64, tabs, R, V, **kw):
    k_self, g, w, r0, dr = tabs
    return pkg.System(n=2, box=BOX, dt=DT, mass=1.0, kT=1.0, k_self=k_self, k_pair_g=g, k_pair_w=w, r0=r0,
                      dr=dr, r_cut=RC, wca_eps=0.0, seed=77, fp64=fp64, r=R, v=V,
                      **({"noise_tol": 1e-12} if fp64 else {}), **kw)


def oracle_traj(oracle_mod, tabs, R, V, steps, kT=1.0):
    """Positions R_0 .. R_steps of the oracle from (R, V) at step 0 with zero history."""
    k_self, g, w, r0, dr = tabs
    o = oracle_mod.Oracle(n=2, box=BOX, dt=DT, mass=1.0, kT=kT, k_self=k_self, k_pair=np.outer(w, g), r0=r0,
                          dr=dr, r_cut=RC, wca_eps=0.0, seed=77, lanczos_tol=1e-13, lanczos_max_iter=400)
    Rc, Vc, H = R.copy(), V.copy(), o.empty_history()
    out = [R.copy()]
    for n in range(steps):
        o.step(n, Rc, Vc, H)
        out.append(Rc.copy())
    return o, out


def weight(R):
    d = R[1] - R[0]
    d -= BOX * np.round(d / BOX)
    r = float(np.sqrt((d ** 2).sum()))
    return (1 - r / RC) ** 2 if r < RC else 0.0


@pytest.mark.parametrize("fp64", [True, False])
def test_row_sum_above_lam_hi_latches_interval_at_its_step(pkg, oracle_mod, fp64):
    tabs = tables()
    R, V = pair_state(4.0, 8.0)
    lam_hi = 0.3
    o, traj = oracle_traj(oracle_mod, tabs, R, V, 20)
    ws = [weight(x) for x in traj]
    # the refresh of step n sees R_{n+1}
    n_exp = next(n for n in range(20) if ws[n + 1] > lam_hi)
    log(f"  w along the oracle's path: {np.round(ws, 4)}; expected flag step {n_exp}")
    assert abs(ws[n_exp + 1] - lam_hi) > 1e-3 and abs(ws[n_exp] - lam_hi) > 1e-3
    s = make(pkg, fp64, tabs, R, V, lam_lo=-0.6, lam_hi=lam_hi)
    s.step(20)
    st = s.read_state(check=False)
    log(f"  status {st['status']} flag step {st['flag_step']}")
    assert st["status"] == pkg._binding.GLD_ERR_INTERVAL and st["flag_step"] == n_exp
    with pytest.raises(pkg.GLDError) as e:
        s.step(1)  # poisoned
    assert e.value.status == pkg._binding.GLD_ERR_INTERVAL
    s.close()


@pytest.mark.parametrize("fp64", [True, False])
def test_periodic_check_latches_interval_at_the_check_step(pkg, oracle_mod, fp64):
    """The lower end is guarded by the Lanczos check alone (the row sums only
    bound the top): with check_interval = 4 the first check whose
    configuration has -w below lam_lo latches GLD_ERR_INTERVAL at its step."""
    tabs = tables()
    R, V = pair_state(4.0, 8.0)
    lam_lo, every = -0.3, 4
    o, traj = oracle_traj(oracle_mod, tabs, R, V, 24)
    ws = [weight(x) for x in traj]
    # a check runs before step s (s > 0, s % every == 0) on R_s
    s_exp = next(s for s in range(every, 25, every) if -ws[s] < lam_lo)
    log(f"  w: {np.round(ws, 4)}; expected check step {s_exp}")
    assert abs(ws[s_exp] + lam_lo) > 1e-3
    assert ws[s_exp - every] < -lam_lo - 1e-3
    s = make(pkg, fp64, tabs, R, V, lam_lo=lam_lo, lam_hi=3.0, check_interval=every)
    s.step(24)
    st = s.read_state(check=False)
    log(f"  status {st['status']} flag step {st['flag_step']}")
    assert st["status"] == pkg._binding.GLD_ERR_INTERVAL and st["flag_step"] == s_exp
    s.close()


@pytest.mark.parametrize("fp64", [True, False])
def test_written_state_outside_the_interval_is_rejected(pkg, fp64):
    """gld_write_state checks the installed configuration against the noise
    interval and the singular points, as gld_create does."""
    tabs = tables()
    R, V = pair_state(4.0, 0.0)
    s = make(pkg, fp64, tabs, R, V, lam_lo=-0.3, lam_hi=3.0)
    R2, V2 = pair_state(1.5, 0.0)  # w = 0.49: the smallest eigenvalue -0.49 < lam_lo
    with pytest.raises(pkg.GLDError) as e:
        s.write_state(R2, V2, step=17)
    assert e.value.status == pkg._binding.GLD_ERR_INTERVAL
    st = s.read_state(check=False)
    assert st["flag_step"] == 17
    s.write_state(R, V, step=3)  # a good state clears it
    s.step(2)
    s.sync()
    s.close()


@pytest.mark.parametrize("fp64", [True, False])
def test_run_time_loss_of_positive_definiteness_is_not_pd(pkg, oracle_mod, fp64):
    """A strong pair memory (g scaled by 3) puts the singular point of the
    correlation near lambda = -0.486: once the closing pair has w beyond it,
    some K_hat_w = S_w + G_w P is indefinite.  The pair closes fast (w 0.46
    at step 6, 0.57 at step 7; the noise moves it by about 1e-4 per step), so
    the steps before the check at step 7 all stay inside the interval
    [-0.47, 1] and the check sees a configuration past the singular point:
    it latches GLD_ERR_NOT_PD at step 7, and the oracle's Algorithm 1
    reports NOT_PD for that same configuration (and not for the one before)."""
    tabs = tables(g_scale=3.0)
    sing = singular_point(tabs[0], tabs[1])
    log(f"  singular point {sing:.4f}")
    assert -0.49 < sing < -0.48
    R, V = pair_state(4.0, 20.0)
    every, lam_lo = 7, -0.47
    s = make(pkg, fp64, tabs, R, V, lam_lo=lam_lo, lam_hi=1.0, check_interval=every)
    s.step(every - 1)
    r_prev = s.read_state()["r"]
    s.step(1)
    r_chk = s.read_state()["r"]
    w_prev, w_chk = weight(r_prev), weight(r_chk)
    log(f"  w at steps {every - 1}, {every}: {w_prev:.4f}, {w_chk:.4f}")
    assert -w_prev > lam_lo + 5e-3 and -w_chk < sing - 0.05
    s.step(1)  # the check before step `every` sees r_chk
    st = s.read_state(check=False)
    log(f"  status {st['status']} flag step {st['flag_step']}")
    assert st["status"] == pkg._binding.GLD_ERR_NOT_PD and st["flag_step"] == every
    k_self, g, w, r0, dr = tabs
    o = oracle_mod.Oracle(n=2, box=BOX, dt=DT, mass=1.0, kT=1.0, k_self=k_self, k_pair=np.outer(w, g), r0=r0,
                          dr=dr, r_cut=RC, wca_eps=0.0, seed=77, lanczos_tol=1e-13, lanczos_max_iter=400)
    with pytest.raises(oracle_mod.OracleError) as e:
        o.noise(every, r_chk)
    assert e.value.code == oracle_mod.ORC_ERR_NOT_PD
    o.noise(every - 1, r_prev)  # positive definite one step earlier
    s.close()
