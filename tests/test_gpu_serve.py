"""The continuous-batching server (include/gld_serve.h): requests arriving
over time with more of them than system slots; each request's final state
equals that of the same request run alone (a batch of one, same mat-vec
schedule), bit for bit, and the recorded times are consistent (admitted at
or after arrival, done after admission, no more than the slots at once)."""
import sys

import numpy as np
import pytest

from paper_1808_00270_amd import workloads as wl

pytestmark = pytest.mark.gpu
THR = [24, 64, 160]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bmod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_00270_amd as p
    p.lib()
    from paper_1808_00270_amd import batch
    return batch


def requests():
    base = [
        wl.ScaledWorkload(name="q0", n=64, rho=0.05, m_max=200, steps=0, seed=4001),
        wl.ScaledWorkload(name="q1", n=300, rho=0.2, m_max=60, steps=0, seed=4002, f_self=1.5),
        wl.ScaledWorkload(name="q2", n=900, rho=0.5, m_max=120, steps=0, seed=4003, f_pair=0.7),
        wl.ScaledWorkload(name="q3", n=250, rho=0.01, m_max=500, steps=0, seed=4004),
        wl.ScaledWorkload(name="q4", n=600, rho=0.3, m_max=200, steps=0, seed=4005, f_self=0.8),
    ]
    steps = [120, 75, 160, 90, 40]
    arrivals = [0.0, 0.02, 0.05, 0.3, 0.31]
    return list(zip(arrivals, steps, base))


@pytest.mark.parametrize("fp64", [False, True])
def test_each_result_is_the_same_alone_and_in_the_mix(bmod, fp64):
    reqs = requests()
    sv = bmod.Server(3, 1 << 30, chunk_steps=25, thresholds=THR, fp64=fp64)
    ids = []
    for t, steps, w in reqs:
        p, keep = bmod.workload_params(w, fp64=fp64)
        R, V = w.initial_state()
        rid, foot = sv.submit(p, R, V, steps, t)
        ids.append((rid, keep))
    sv.run()
    makespan, bsteps = sv.stats()
    log(f"  served {len(reqs)} requests in {makespan:.3f}s, {bsteps} batch steps")
    recs = []
    for (rid, _), (t, steps, w) in zip(ids, reqs):
        rec, st = sv.request(rid)
        recs.append(rec)
        log(f"  {w.name}: arrival {rec['arrival_s']:.3f} admitted {rec['admitted_s']:.3f} done {rec['done_s']:.3f} "
            f"steps {rec['steps']} footprint {rec['footprint'] / 2**20:.1f} MB")
        assert rec["admitted_s"] >= rec["arrival_s"] - 1e-9 and rec["done_s"] > rec["admitted_s"]
        assert st["step"] == steps and st["flags"] == 0
        # the same request alone
        b = bmod.Batch(1, 1 << 30, fp64=fp64)
        p, keep = bmod.workload_params(w, fp64=fp64)
        R, V = w.initial_state()
        s = b.add([(p, keep, R, V)])[0]
        b.set_schedule(THR)
        b.step(steps)
        a = b.read_state(s)
        b.close()
        for k in ("r", "v", "f_c", "f_d", "f_r"):
            assert np.array_equal(a[k], st[k]), (w.name, k)
    # at most three requests in the batch at any time
    events = sorted([(r["admitted_s"], 1) for r in recs] + [(r["done_s"], -1) for r in recs])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 3
    sv.close()
