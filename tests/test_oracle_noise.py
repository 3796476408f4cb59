"""Pins of the noise-parameter draw in the oracle.

Bins: contiguous, monotone, power-of-two widths with edge ratios <= 9/8, and
the vectorised form equals the scalar definition.  Periodogram: Parseval on
the extension.  alpha step: a binned spectrum that follows the model exactly
returns its alpha; the score vanishes at the mode and the curvature is
positive.  Wilson-Hilferty variates match scipy's chi^2 and Gamma quantiles.
End to end: n_corr synthesised with a known spectrum is recovered within its
posterior width; sigma0 of an exactly scaled residual is recovered.
"""
import numpy as np
from scipy import stats

from oracle import noise as on
from oracle import tod as ot


def test_bins_contiguous_and_logarithmic():
    k = np.arange(1, 1 << 20)
    b = on.bins_of(k)
    assert all(on.bin_of(int(x)) == int(y) for x, y in zip(k[::997], b[::997]))
    assert b[0] == 0 and (np.diff(b) >= 0).all() and (np.diff(b) <= 1).all()
    edges = k[np.flatnonzero(np.diff(b)) + 1]
    width = np.diff(edges)
    assert (width & (width - 1) == 0).all()           # powers of two
    assert (edges[8:] / edges[7:-1] <= 9 / 8 + 1e-12).all()
    assert on.bin_of((1 << 31) - 1) == on.NBIN - 1


def test_periodogram_parseval():
    rng = np.random.default_rng(1)
    nc = rng.normal(size=1234)
    N = ot.fft_length(1234)
    e = ot.extend(nc, N)
    I = np.abs(np.fft.rfft(e)) ** 2 / N
    J, c, f = on.periodogram_bins(nc, 10.0)
    # sum_k |X_k|^2 = N sum e^2 over all N modes; half spectrum k = 1..N/2
    assert abs((2 * J.sum() - I[-1]) - (e @ e - I[0])) <= 1e-10 * (e @ e)
    assert c.sum() == N // 2
    assert (np.diff(f) > 0).all()


def test_alpha_mode_of_an_exact_power_law():
    J, c, f = on.periodogram_bins(np.random.default_rng(2).normal(size=5000), 20.0)
    s0, fk, al = 1.7, 0.3, -1.3
    J = c * s0 ** 2 * (f / fk) ** al
    ah, H = on.alpha_mode(J, c, f, s0, fk)
    assert abs(ah - al) <= 1e-12
    x = np.log(f / fk)
    assert abs(np.sum(J / s0 ** 2 * x * np.exp(-ah * x) - c * x)) <= 1e-9 * np.sum(c * np.abs(x))
    assert H > 0


def test_wilson_hilferty_quantiles():
    for n in (1000, 50000):
        for z in (-2.0, 0.0, 1.5):
            ref = stats.chi2.ppf(stats.norm.cdf(z), n)
            assert abs(on.wilson_hilferty_chi2(n, z) / ref - 1) <= 1e-4
            refg = stats.gamma.ppf(stats.norm.cdf(z), n)
            assert abs(on.wilson_hilferty_gamma(n, z) / refg - 1) <= 1e-4


def _stationary(n, fsamp, s0, fk, al, seed):
    """Gaussian process with spectrum s0^2 (f/fk)^al on a long periodic grid,
    first n samples (unitary convention, DC dropped)."""
    Nl = 8 * n
    rng = np.random.default_rng(seed)
    f = np.arange(Nl // 2 + 1) * fsamp / Nl
    P = np.zeros(len(f))
    P[1:] = s0 ** 2 * (f[1:] / fk) ** al
    W = (rng.normal(size=len(f)) + 1j * rng.normal(size=len(f))) / np.sqrt(2)
    W[0] = 0
    W[-1] = rng.normal()
    return (np.sqrt(Nl) * np.fft.irfft(W * np.sqrt(P), n=Nl))[:n]


def test_recovers_known_spectrum():
    n, fs, s0, fk, al = 60000, 32.5, 1.0, 0.2, -1.4
    nc = _stationary(n, fs, s0, fk, al, 7)
    rng = np.random.default_rng(8)
    t = rng.normal(size=n) * 50
    d = 1.01 * t + nc + rng.normal(size=n) * s0
    # one sweep conditioned on the true f_knee
    sig, fkn, alpha = on.sample_noise_segment(d, t, 1.01, nc, fs, fk, 0, 0, 0, mean_only=True)
    assert abs(sig - s0) < 0.02
    J, c, f = on.periodogram_bins(nc, fs)
    _, H = on.alpha_mode(J, c, f, sig, fk)
    assert abs(alpha - al) < 6 / np.sqrt(H) + 0.01
    assert abs(np.log(fkn / fk)) < 0.05
    # repeated sweeps from a wrong f_knee climb towards the joint mode
    fkn, prev = 0.1, None
    for _ in range(20):
        _, fkn, alpha = on.sample_noise_segment(d, t, 1.01, nc, fs, fkn, 0, 0, 0, mean_only=True)
        if prev is not None:
            assert abs(alpha - al) <= abs(prev - al) + 1e-12
        prev = alpha


def test_sigma0_of_a_scaled_residual():
    rng = np.random.default_rng(3)
    n = 4000
    r = rng.normal(size=n)
    r *= 2.5 / np.sqrt(r @ r / n)          # sum r^2 = n 2.5^2 exactly
    nc = 0.1 * rng.normal(size=n)
    t = np.zeros(n)
    sig, _, _ = on.sample_noise_segment(r + nc, t, 1.0, nc, 10.0, 0.1, 0, 0, 0, mean_only=True)
    # median of chi^2_n by Wilson-Hilferty: n (1 - 2/(9n))^3
    assert abs(sig - 2.5 / (1 - 2 / (9 * n)) ** 1.5) <= 1e-12


def test_approximate_conditionals_at_workload_sizes():
    """How far the sampler's closed forms are from the exact conditionals
    they stand for (Eq. 5 step; readings of the noise draw): the
    Wilson-Hilferty chi^2 variate against scipy's exact quantiles, and the
    Laplace (Gaussian) form of alpha | f_knee, sigma0 against the exact
    conditional of the binned Whittle likelihood, inverted numerically on a
    fine grid, for a 30,000-sample stationary 1/f segment."""
    from scipy import stats
    from oracle import tod as ot
    z = np.array([-3.0, -1.0, 0.0, 1.0, 3.0])
    for n, tol in ((1e4, 1e-6), (2.6e5, 1e-8)):
        wh = on.wilson_hilferty_chi2(n, z)
        ex = stats.chi2.ppf(stats.norm.cdf(z), n)
        assert np.abs(wh / ex - 1).max() < tol
    rng = np.random.default_rng(1)
    n, fs, s0, fk, al = 30000, 78.8, 1.0, 0.1, -1.5
    N = ot.fft_length(n)
    k = np.arange(N // 2 + 1)
    f = k * fs / N
    P = np.zeros_like(f)
    P[1:] = s0 ** 2 * (f[1:] / fk) ** al
    X = (rng.normal(size=len(k)) + 1j * rng.normal(size=len(k))) * np.sqrt(P / 2)
    X[0] = 0
    nc = (np.fft.irfft(X, n=N) * np.sqrt(N))[:n]
    J, c, fb = on.periodogram_bins(nc, fs)
    ah, H = on.alpha_mode(J, c, fb, s0, fk)
    x, a = np.log(fb / fk), J / s0 ** 2
    grid = ah + np.linspace(-12, 12, 20001) / np.sqrt(H)
    lnL = np.array([-np.sum(a * np.exp(-g * x) + c * (2 * np.log(s0) + g * x)) for g in grid])
    p = np.exp(lnL - lnL.max())
    cdf = np.concatenate([[0.0], np.cumsum((p[1:] + p[:-1]) / 2 * np.diff(grid))])
    cdf /= cdf[-1]
    dev = [(np.interp(stats.norm.cdf(zz), cdf, grid) - (ah + zz / np.sqrt(H))) * np.sqrt(H) for zz in z]
    assert np.abs(dev).max() < 0.02   # in units of the conditional's width
