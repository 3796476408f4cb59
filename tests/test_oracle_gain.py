"""Pins of the per-segment gain draw in the oracle.

A noiseless segment returns its gain exactly; a constant offset of the data
changes nothing (h_0 = 0 and K d, not (K t) . d); the FFT filter equals the
dense matrix C F^H diag(h) F E built from the DFT and an explicit extension
matrix; in the white-noise limit K is the mean-removed extension / sigma0^2;
the draw's standardised spread over iterations is a unit normal.
"""
import numpy as np
from scipy import stats

from oracle import gain as og
from oracle import tod as ot

PAR = dict(fsamp=32.5, sigma0=1.3, fknee=0.4, alpha=-1.5)


def _t(n, seed=0):
    rng = np.random.default_rng(seed)
    return 100.0 * np.sin(np.arange(n) * 2 * np.pi / 37.0) + rng.normal(size=n) * 20


def _args():
    return PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"]


def test_noiseless_gain_is_exact():
    t = _t(1000)
    for g in (0.97, 1.0, 1.013):
        got, sig, A, B = og.sample_gain_segment(g * t, t, *_args(), 1, 0, 0, mean_only=True)
        assert abs(got - g) <= 1e-12
        assert A > 0 and sig == 1.0 / np.sqrt(A)


def test_constant_offset_has_no_effect():
    rng = np.random.default_rng(5)
    t = _t(777, 1)
    d = 1.01 * t + rng.normal(size=777) * 2
    a = og.sample_gain_segment(d, t, *_args(), 3, 2, 1)[0]
    b = og.sample_gain_segment(d + 250.0, t, *_args(), 3, 2, 1)[0]
    assert abs(a - b) <= 1e-11


def test_filter_matches_dense_matrix():
    n = 23
    N = ot.fft_length(n)
    E = np.zeros((N, n))
    for j in range(n):
        E[j, j] = 1.0
        E[2 * n - 1 - j, j] = 1.0
    E[2 * n:, 0] = 1.0
    k = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(k, k) / N)
    h = og.gain_filter(N, *_args())
    full = np.concatenate([h, h[1:N - len(h) + 1][::-1]])
    H = (F.conj().T @ np.diag(full) @ F).real / N
    K = H[:n] @ E
    x = np.random.default_rng(2).normal(size=n)
    assert np.allclose(og.inv_noise(x, *_args()), K @ x, rtol=0, atol=1e-13 * np.abs(K @ x).max())


def test_white_noise_limit():
    n = 500
    x = np.random.default_rng(3).normal(size=n)
    N = ot.fft_length(n)
    e = ot.extend(x, N)
    ref = (e - e.mean())[:n] / PAR["sigma0"] ** 2
    got = og.inv_noise(x, PAR["fsamp"], PAR["sigma0"], 1e-12, -1.5)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_draw_is_mean_plus_unit_normal_scaled():
    t = _t(300, 4)
    d = 1.02 * t + np.random.default_rng(6).normal(size=300)
    mean, sig, _, _ = og.sample_gain_segment(d, t, *_args(), 9, 7, 0, mean_only=True)
    z = [(og.sample_gain_segment(d, t, *_args(), 9, 7, it)[0] - mean) / sig for it in range(2000)]
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_exact_mode_is_scaled_by_hand_computed_weight():
    """n = 500 gives N = 1000 with no pad; x_j = cos(2 pi k0 (j + 1/2) / N)
    extends to the pure mode k0.  With f_k0 = 2 f_knee and alpha = -1,
    P = sigma0^2 / 2, so K x = x / (1.5 sigma0^2)."""
    n, k0, fs = 500, 40, 32.5
    N = ot.fft_length(n)
    assert N == 1000
    fknee = 0.5 * k0 * fs / N
    j = np.arange(n)
    x = np.cos(2 * np.pi * k0 * (j + 0.5) / N)
    got = og.inv_noise(x, fs, 2.0, fknee, -1.0)
    assert np.abs(got - x / (1.5 * 4.0)).max() <= 1e-13
