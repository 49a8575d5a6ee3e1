"""IMRV (Sec. III.B, eq. phi) on deterministic responses, with the oracle as
the GLD engine: the noise-free response of a particle that starts with unit
velocity is the normalised equilibrium velocity autocorrelation (kT = 0
linear response), so these runs carry no statistical noise.

* the self kernel is reconstructed from the autocorrelation it produces;
* Sec. III.A's route: the decoupled modes V_+- of a pair at fixed distance
  have kernels K_+- = K^s +- K^p(R); each is reconstructed from the pair's
  C_+- (two-particle oracle runs) with single-particle runs, and
  K^s = (K_+ + K_-)/2, K^p(R) = (K_+ - K_-)/2 come out close to the truth.
"""
import numpy as np
import pytest

from paper_1808_00270_amd import imrv

DT, M = 0.01, 100


def single_response(oracle_mod, k_of_t):
    o = oracle_mod.Oracle(n=1, box=20.0, dt=DT, mass=1.0, kT=0.0, k_self=imrv.to_table(k_of_t, DT),
                          k_pair=np.zeros((2, M)), r0=0.0, dr=5.0, r_cut=5.0, wca_eps=0.0)
    R, V, H = np.array([[1.0, 1.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]), o.empty_history()
    ys = [1.0]
    for n in range(M):
        o.step(n, R, V, H)
        ys.append(V[0, 0])
    return np.array(ys)


def kstar():
    t = np.arange(M) * DT
    return 10.0 * np.exp(-t / 0.5) * np.cos(4.0 * t)


def test_self_kernel_from_its_velocity_autocorrelation(oracle_mod):
    ks = kstar()
    target = single_response(oracle_mod, ks)
    res = imrv.reconstruct(target, 0.5 * ks, lambda k: single_response(oracle_mod, k), dt=DT, alpha=3.0,
                           iterations=40)
    kerr = [np.linalg.norm(k - ks) / np.linalg.norm(ks) for k in res.kernels]
    assert res.errors[0] > 0.3 and res.errors[-1] < 0.01
    assert kerr[-1] < 0.6 * kerr[0]
    # the errors fall (up to small oscillations of the relaxation)
    assert max(res.errors[-10:]) < 0.05 * res.errors[0]


def test_pair_kernel_from_the_decoupled_two_particle_route(oracle_mod):
    ks = kstar()
    t = np.arange(M) * DT
    Rd, rc = 2.0, 5.0
    g = 4.0 * np.exp(-t / 0.3)              # K^p(R, t) = w(R) g(t), w(r) = 1 - r/rc
    w = np.clip(1 - np.linspace(0, rc, 51) / rc, 0, None)
    kp_true = (1 - Rd / rc) * g
    o = oracle_mod.Oracle(n=2, box=60.0, dt=DT, mass=1.0, kT=0.0, k_self=imrv.to_table(ks, DT),
                          k_pair=np.outer(w, imrv.to_table(g, DT)), r0=0.0, dr=rc / 50, r_cut=rc, wca_eps=0.0)
    # responses of the pair: unit velocity on particle 0 along the line of centres
    R = np.array([[10.0, 10.0, 10.0], [10.0 + Rd, 10.0, 10.0]])
    eps = 1e-7
    V = np.array([[eps, 0.0, 0.0], [0.0, 0.0, 0.0]])
    H = o.empty_history()
    v1, v2 = [eps], [0.0]
    for n in range(M):
        o.step(n, R, V, H)
        v1.append(V[0, 0])
        v2.append(V[1, 0])
    v1, v2 = np.array(v1) / eps, np.array(v2) / eps
    c_plus, c_minus = v1 + v2, v1 - v2      # V_+- = V_1 +- V_2 from V_+-(0) = 1
    fits = []
    for target in (c_plus, c_minus):
        res = imrv.reconstruct(target, ks, lambda k: single_response(oracle_mod, k), dt=DT, alpha=3.0,
                               iterations=40)
        assert res.errors[-1] < 0.02
        fits.append(res.kernels[-1])
    k_self, k_pair = imrv.pair_kernels_from_decoupled(*fits)
    e_self = np.linalg.norm(k_self - ks) / np.linalg.norm(ks)
    e_pair = np.linalg.norm(k_pair - kp_true) / np.linalg.norm(kp_true)
    # the first half of the memory, where the correlations constrain the kernels
    half = slice(0, M // 2)
    e_pair_early = np.linalg.norm((k_pair - kp_true)[half]) / np.linalg.norm(kp_true[half])
    print(f"self {e_self:.3f} pair {e_pair:.3f} pair (first half) {e_pair_early:.3f}")
    assert e_self < 0.2 and e_pair_early < 0.35


def test_decoupled_kernels_recombine_exactly():
    a, b = np.array([3.0, 1.0, -0.5]), np.array([1.0, 0.5, 0.25])
    ks, kp = imrv.pair_kernels_from_decoupled(a + b, a - b)
    assert np.allclose(ks, a) and np.allclose(kp, b)


def test_positive_projection():
    """The spectrum convention: S_w of K(t) = exp(-t/tau) samples equals the
    direct cosine sum; a kernel with a positive spectrum is left alone; one
    with negative values is mapped to one whose spectrum is the clipped one
    (inverse transform of an even real spectrum of period 2M - 1)."""
    t = np.arange(M) * DT
    k = np.exp(-t / 0.05)   # spectrum ratio min/max = ((1-q)/(1+q))^2 ~ 1e-2, q = exp(-DT/0.05)
    P = 2 * M - 1
    S = imrv.spectrum(k)
    w = np.arange(M)[:, None]
    direct = k[0] + 2 * (k[None, 1:] * np.cos(2 * np.pi * w * np.arange(1, M)[None, :] / P)).sum(axis=1)
    np.testing.assert_allclose(S, direct, rtol=1e-12, atol=1e-12)
    assert np.all(S > 0)
    np.testing.assert_array_equal(imrv.project_positive(k), k)
    bad = k - 0.3 * np.cos(2 * np.pi * 3 * np.arange(M) / P)  # dents the spectrum at w = 3
    Sb = imrv.spectrum(bad)
    assert Sb.min() < 0
    fixed = imrv.project_positive(bad, floor=1e-3)
    Sf = imrv.spectrum(fixed)
    lo = 1e-3 * np.abs(Sb).max()
    np.testing.assert_allclose(Sf, np.maximum(Sb, lo), rtol=1e-10, atol=1e-10)
