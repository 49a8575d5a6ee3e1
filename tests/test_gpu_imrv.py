"""IMRV (Sec. III.B, eq. phi) with the library's GPU integrator as the GLD
engine: the target is the velocity autocorrelation measured in a GPU run of
non-interacting particles with a known self kernel K*; starting from K*/2,
the reconstruction's correlation approaches the target (to the statistical
error of the runs) and its kernel moves towards K*.  Parity unpinned: the
stochastic estimate has no exact value; the deterministic counterpart runs
on the CPU with the oracle (tests/test_imrv.py)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_self_kernel_reconstruction_on_the_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_00270_amd import imrv
    dt, M = 0.01, 100
    t = np.arange(M) * dt
    kstar = 10.0 * np.exp(-t / 0.5) * np.cos(4.0 * t)
    run = dict(n=4096, steps=1500, burn_in=300, dt=dt)
    target = imrv.gpu_vacf(kstar, seed=11, **run)
    log(f"  target VACF(0) {target[0]:.4f} (kT/M = 1)")
    assert abs(target[0] - 1.0) < 0.02
    res = imrv.reconstruct(target, 0.5 * kstar, lambda k: imrv.gpu_vacf(k, seed=13, **run), dt=dt, alpha=3.0,
                           iterations=10,
                           callback=lambda it, k, e: log(f"  iteration {it}: VACF error {e:.4f}"))
    kerr = [np.linalg.norm(k - kstar) / np.linalg.norm(kstar) for k in res.kernels]
    log(f"  kernel error {kerr[0]:.3f} -> {kerr[-1]:.3f}")
    assert res.errors[-1] < 0.25 * res.errors[0]
    assert kerr[-1] < kerr[0]
