"""Statistical checks of the GPU path over many steps.

1. FDT of the colored noise on frozen positions (eq. stochastic_force2):
   with a huge mass the positions do not move, P is constant and F^R is a
   stationary Gaussian sequence whose lag covariances must be
   kT a_m K^s_m / dt on each component and kT a_m g_m / dt w(R_ij) between
   the same components of neighbours (a_0 = 2, a_m = 1).  m_max = 1000 makes
   the wrap error of the linear filter (reading A4) ~1e-9.  Error bars from
   block averages.
2. VACF and MSD of cfg1 trajectories against the FP64 oracle's
   (tests/golden/cfg1_vacf_msd.json, written by tests/golden/make_vacf_msd.py
   with the same seeds): agreement within 4 standard errors at every lag.
   The many-particle VACF has no closed form ("parity unpinned" beyond the
   oracle), so this is the check that the long-run statistics match.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1808_00270_amd import workloads as wl
from test_gpu_parity import log, pkg  # noqa: F401

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("fp64", [True, False])
def test_noise_fdt_on_frozen_positions(pkg, fp64):
    w = wl.config(1, m_max=1000, mass=1e12)
    R, V = w.initial_state()
    V[:] = 0.0
    s = pkg.System.from_workload(w, fp64=fp64, r=R, v=V)
    steps, nblk = 3000, 15
    F = np.empty((steps, w.n, 3))
    for t in range(steps):
        s.step(1)
        F[t] = s.read_state()["f_r"]
    R1 = s.read_state()["r"]
    s.close()
    assert np.abs(R1 - R).max() < 1e-9  # frozen
    k_self, g, wt, r0, dr = w.tables()
    # pairs at the frozen positions (minimum image), weights from the table
    L = w.box
    d = R[:, None, :] - R[None, :, :]
    d -= L * np.rint(d / L)
    r = np.sqrt(np.sum(d * d, axis=2))
    np.fill_diagonal(r, np.inf)
    wij = np.where(r < w.r_cut, np.interp(np.minimum(r, w.r_cut), r0 + dr * np.arange(len(wt)), wt), 0.0)
    sw2 = float(np.sum(wij * wij))
    blk = steps // nblk
    for m in (0, 1, 2, 5, 10, 20, 50):
        am = 2.0 if m == 0 else 1.0
        es = w.kT * am * k_self[m] / w.dt
        ep = w.kT * am * g[m] / w.dt
        self_b, pair_b = [], []
        for b in range(nblk):
            t0, t1 = b * blk, (b + 1) * blk - m
            A, B = F[t0 + m:t1 + m], F[t0:t1]
            self_b.append(np.mean(A * B))
            # sum_ij w_ij sum_c A_ic B_jc / (3 sum w^2), averaged over t
            pair_b.append(np.mean(np.einsum("ij,tic,tjc->t", wij, A, B)) / (3.0 * sw2))
        vs, vp = np.mean(self_b), np.mean(pair_b)
        ss, sp = np.std(self_b, ddof=1) / math.sqrt(nblk), np.std(pair_b, ddof=1) / math.sqrt(nblk)
        log(f"    lag {m:3d}: self {vs:9.4f} vs {es:9.4f} (+-{ss:.4f})   pair {vp:9.4f} vs {ep:9.4f} (+-{sp:.4f})")
        assert abs(vs - es) < 4.5 * ss + 1e-3 * abs(w.kT * 2 * k_self[0] / w.dt)
        assert abs(vp - ep) < 4.5 * sp + 1e-3 * abs(w.kT * 2 * g[0] / w.dt)


def _gpu_correlations(pkg, gold, fp64):
    lags, equil, stride, steps = gold["lags"], gold["equil"], gold["origin_stride"], gold["steps"]
    every = 10
    assert all(l % every == 0 for l in lags) and equil % every == 0 and stride % every == 0
    vacf, msd = [], []
    for seed in gold["seeds"]:
        w = wl.config(1, seed=seed)
        s = pkg.System.from_workload(w, fp64=fp64)
        st = s.read_state()
        Rs, Vs = [st["r"]], [st["v"]]
        for _ in range(steps // every):
            s.step(every)
            st = s.read_state()
            Rs.append(st["r"])
            Vs.append(st["v"])
        s.close()
        Rs, Vs = np.array(Rs), np.array(Vs)
        origins = range(equil, steps - lags[-1] + 1, stride)
        vacf.append([np.mean([np.mean(np.sum(Vs[(t + l) // every] * Vs[t // every], axis=1)) / 3.0
                              for t in origins]) for l in lags])
        msd.append([np.mean([np.mean(np.sum((Rs[(t + l) // every] - Rs[t // every]) ** 2, axis=1))
                             for t in origins]) for l in lags])
    return np.array(vacf), np.array(msd)


@pytest.mark.parametrize("fp64", [True, False])
def test_vacf_msd_match_oracle_statistics(pkg, fp64):
    with open(os.path.join(HERE, "golden", "cfg1_vacf_msd.json")) as f:
        gold = json.load(f)
    gv, gm = _gpu_correlations(pkg, gold, fp64)
    ov, om = np.array(gold["vacf"]), np.array(gold["msd"])
    ns = len(gold["seeds"])
    for name, a, b in (("VACF", gv, ov), ("MSD", gm, om)):
        ma, mb = a.mean(axis=0), b.mean(axis=0)
        se = np.sqrt(a.var(axis=0, ddof=1) / ns + b.var(axis=0, ddof=1) / ns)
        z = np.abs(ma - mb) / np.maximum(se, 1e-300)
        for k in (0, 1, 3, 10, len(gold["lags"]) - 1):
            log(f"    {name} lag {gold['lags'][k]:3d}: gpu {ma[k]:.5f} oracle {mb[k]:.5f} (+-{se[k]:.5f})")
        assert np.all(z < 4.0), f"{name}: largest deviation {z.max():.2f} standard errors at lag {gold['lags'][int(z.argmax())]}"
