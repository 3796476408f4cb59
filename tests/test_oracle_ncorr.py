"""Pin the oracle's correlated-noise constrained realisation (Eq. 4, section 4.2).

The FFT-diagonal draw on the mirrored, padded segment must equal the dense
Gaussian posterior of the same extended-space model, written with numpy.linalg:
  mean  mu    = (I/sigma0^2 + C^-1)^-1 e / sigma0^2
  cov   Sigma = (I/sigma0^2 + C^-1)^-1,   C^-1 = F^H diag(1/P) F,  1/P_0 = 0.
"""
import numpy as np
import pytest

from oracle import tod as ot


def _dense_posterior(e, fsamp, sigma0, fknee, alpha):
    N = len(e)
    k = np.arange(N)
    kk = np.minimum(k, N - k)                       # two-sided spectrum
    f = kk * fsamp / N
    invP = np.zeros(N)
    invP[kk > 0] = 1.0 / (sigma0 ** 2 * (f[kk > 0] / fknee) ** alpha)
    F = np.exp(-2j * np.pi * np.outer(k, k) / N) / np.sqrt(N)
    Cinv = (F.conj().T @ np.diag(invP) @ F).real
    Sigma = np.linalg.inv(np.eye(N) / sigma0 ** 2 + Cinv)
    mu = Sigma @ e / sigma0 ** 2
    return mu, Sigma


CASES = [(23, 32.5, 1.0, 0.1, -1.5), (20, 78.8, 1.7, 2.0, -1.1), (31, 10.0, 0.6, 0.7, -1.8)]


@pytest.mark.parametrize("n,fs,s0,fk,al", CASES)
def test_mean_equals_dense_gls(n, fs, s0, fk, al):
    r = np.random.default_rng(n).normal(size=n) * 3 + 5
    N = ot.fft_length(n)
    mu, _ = _dense_posterior(ot.extend(r, N), fs, s0, fk, al)
    got = ot.sample_ncorr_segment(r, fs, s0, fk, al, 1, 0, 0, mean_only=True)
    assert np.allclose(got, mu[:n], rtol=0, atol=1e-12 * np.abs(mu).max())


@pytest.mark.parametrize("n,fs,s0,fk,al", CASES)
def test_draw_covariance_equals_dense_gls(n, fs, s0, fk, al, monkeypatch):
    """The fluctuation is linear in the unit normals; push every basis vector
    through the oracle and compare the exact covariance with the dense one."""
    N = ot.fft_length(n)
    K = N // 2 + 1
    r = np.zeros(n)
    _, Sigma = _dense_posterior(ot.extend(r, N), fs, s0, fk, al)
    cols = []
    for which in range(4):
        for k in range(K):
            if which in (1, 3) and k in (0, K - 1):
                continue                          # imaginary parts unused there
            z = [np.zeros(K) for _ in range(4)]
            z[which][k] = 1.0

            def fake(seed, seg, it, NN, z=z):
                W1 = (z[0] + 1j * z[1]) / np.sqrt(2.0)
                W2 = (z[2] + 1j * z[3]) / np.sqrt(2.0)
                W1[0], W2[0], W1[-1], W2[-1] = z[0][0], z[2][0], z[0][-1], z[2][-1]
                return W1, W2
            monkeypatch.setattr(ot, "white_modes", fake)
            cols.append(ot.sample_ncorr_segment(r, fs, s0, fk, al, 0, 0, 0))
    L = np.stack(cols, axis=1)
    assert np.allclose(L @ L.T, Sigma[:n, :n], rtol=0, atol=1e-12 * np.abs(Sigma).max())


def test_draw_variance_over_seeds():
    """Through the real Philox path: Var(n_t - mu_t) matches the posterior diagonal."""
    n, fs, s0, fk, al = 24, 32.5, 1.0, 0.5, -1.5
    r = np.random.default_rng(0).normal(size=n)
    N = ot.fft_length(n)
    mu, Sigma = _dense_posterior(ot.extend(r, N), fs, s0, fk, al)
    M = 3000
    X = np.stack([ot.sample_ncorr_segment(r, fs, s0, fk, al, 12345, 7, it) for it in range(M)])
    dev = X - mu[:n]
    v = dev.var(axis=0)
    target = np.diag(Sigma)[:n]
    assert np.all(np.abs(v - target) < 5 * target * np.sqrt(2.0 / M))
    assert np.all(np.abs(dev.mean(axis=0)) < 5 * np.sqrt(target / M))


def test_limits():
    r = np.random.default_rng(5).normal(size=40) + 2.0
    N = ot.fft_length(40)
    # f_knee -> 0: no correlated power except DC, the mean is the extension's mean
    lo = ot.sample_ncorr_segment(r, 10.0, 1.0, 1e-12, -1.5, 0, 0, 0, mean_only=True)
    assert np.allclose(lo, ot.extend(r, N).mean(), atol=1e-12)
    # f_knee -> infinity: the correlated part absorbs everything, mean = r
    hi = ot.sample_ncorr_segment(r, 10.0, 1.0, 1e9, -1.5, 0, 0, 0, mean_only=True)
    assert np.allclose(hi, r, atol=1e-9)


def test_mean_is_wiener_filter():
    """Mean-only output of a pure sinusoid at an exact mode k of the extension:
    scaled by P_k / (P_k + sigma0^2)."""
    n = 48
    N = ot.fft_length(n)               # 96
    k = 3
    t = np.arange(N)
    e = np.cos(2 * np.pi * k * (t + 0.5) / N)   # symmetric about (2n-1)/2 -> mirror exact
    r = e[:n]
    assert np.allclose(ot.extend(r, N), e)
    fs, s0, fk, al = 20.0, 1.3, 0.9, -1.2
    P = s0 ** 2 * ((k * fs / N) / fk) ** al
    got = ot.sample_ncorr_segment(r, fs, s0, fk, al, 0, 0, 0, mean_only=True)
    assert np.allclose(got, r * P / (P + s0 ** 2), atol=1e-13)
