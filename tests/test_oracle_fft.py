"""Pin the FFT length rule, the extension and the FFT conventions the oracle uses."""
import numpy as np
import pytest

from oracle import tod as ot


def _five_smooth_upto(limit):
    s = set()
    a = 1
    while a <= limit:
        b = a
        while b <= limit:
            c = b
            while c <= limit:
                s.add(c)
                c *= 5
            b *= 3
        a *= 2
    return np.array(sorted(s))


def test_fft_length_brute_force():
    sm = _five_smooth_upto(20000)
    even = sm[sm % 2 == 0]
    for n in range(1, 5000):
        N = ot.fft_length(n)
        assert N == even[np.searchsorted(even, 2 * n)]


def test_fft_length_spot_values():
    # 2*4096 = 8192 is a power of two; 2*100000 = 200000 = 2^6 5^5
    assert ot.fft_length(4096) == 8192
    assert ot.fft_length(100000) == 200000
    assert ot.fft_length(262144) == 524288
    assert ot.fft_length(1) == 2


@pytest.mark.parametrize("N", [8, 30, 96, 250, 486, 1000])
def test_rfft_vs_direct_dft(N):
    x = np.random.default_rng(N).normal(size=N)
    k = np.arange(N // 2 + 1)[:, None]
    t = np.arange(N)[None, :]
    X = (x[None, :] * np.exp(-2j * np.pi * k * t / N)).sum(axis=1)
    assert np.allclose(np.fft.rfft(x), X, rtol=0, atol=1e-10 * np.abs(X).max())


def test_extension_periodic_and_symmetric():
    r = np.random.default_rng(0).normal(size=37)
    N = ot.fft_length(len(r))
    e = ot.extend(r, N)
    n = len(r)
    assert np.array_equal(e[:n], r)
    assert np.array_equal(e[n:2 * n], r[::-1])
    assert np.all(e[2 * n:] == r[0])
    # symmetric about (2n-1)/2 modulo N: e[j] == e[(2n-1-j) mod N]
    j = np.arange(N)
    assert np.array_equal(e, e[(2 * n - 1 - j) % N])


def test_whittle_periodogram_parseval():
    nc = np.random.default_rng(2).normal(size=501)
    I, P, f = ot.whittle_parts(nc, 10.0, 1.0, 0.1, -1.5)
    N = ot.fft_length(len(nc))
    e = ot.extend(nc, N)
    I0 = e.mean() ** 2 * N
    total = I0 + 2 * I[:-1].sum() + I[-1]
    assert np.isclose(total, np.sum(e * e), rtol=1e-12)
    assert np.isclose(f[-1], 5.0)  # Nyquist = fsamp / 2
