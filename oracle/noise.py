"""FP64 reference of the noise-parameter draw xi_n <- P(xi_n | d, g, n_corr, sky).

Test infrastructure: only tests/, the smoke check and the bench CPU baseline
use it; the product path never does.

The Gibbs chain draws the noise parameters after n_corr (Eq. 5); the paper
defers the sampler to a companion paper and notes that only low-volume power
spectrum data are involved.  Reading used here, per segment, with the sky
template t (unit gain), the gain g and the current n_corr:

1. White level.  r = d - g t - n_corr ~ N(0, sigma0^2 I); with a prior flat in
   ln sigma0, sigma0^2 = S / X with S = sum r^2 and X ~ chi^2_n, X drawn by the
   Wilson-Hilferty transform X = n (1 - 2/(9n) + z0 sqrt(2/(9n)))^3.
2. Correlated-noise spectrum.  The periodogram of n_corr on the n_corr draw's
   mirrored extension, I_k = |FFT(e)_k|^2 / N for k = 1..N/2, summed into
   integer log-frequency bins (`bin_of`): J_b = sum I_k, c_b = count,
   f_b = (f_samp/N) exp(mean ln k) (geometric-mean frequency).  Binned Whittle
   likelihood with P_b = sigma0^2 (f_b / f_knee)^alpha:
       ln L = - sum_b (J_b / P_b + c_b ln P_b).
3. alpha | f_knee, sigma0 (prior flat in alpha): ln L is strictly concave in
   alpha; alpha = alpha_hat + z1 / sqrt(H) with alpha_hat its maximiser and H
   the negative second derivative there (the Laplace form of the conditional).
   When ln L has no maximiser (every J_b = 0, as for a one-sample segment,
   whose mirrored extension is constant) the conditional is improper: no
   draw, alpha = f_knee = NaN.
4. f_knee | alpha, sigma0 (prior flat in ln f_knee): u = f_knee^alpha has the
   conditional Gamma(K, rate S_a / sigma0^2), K = sum c_b,
   S_a = sum_b J_b f_b^-alpha; u = G sigma0^2 / S_a with the Wilson-Hilferty
   Gamma variate G = K (1 - 1/(9K) + z2 / (3 sqrt K))^3, f_knee = u^(1/alpha).

z0, z1, z2: Box-Muller normals of the segment's Philox stream at counter word
k = 2^32 - 2 (no Fourier mode uses it); mean_only sets them to 0.
"""
import numpy as np
from scipy import optimize

from . import philox
from . import tod as ot

NOISE_COUNTER = 0xFFFFFFFE
NBIN = 7 + 8 * (31 - 3)   # bins of k = 1 .. 2^31 - 1


def bin_of(k):
    """Integer log-frequency bin of mode k >= 1: k = 1..7 one bin each; above,
    eight bins per octave split by the three bits after the leading one."""
    k = int(k)
    if k < 8:
        return k - 1
    e = k.bit_length() - 1
    return 7 + 8 * (e - 3) + ((k >> (e - 3)) - 8)


def bins_of(k):
    """bin_of over an integer array (exact: frexp of an integer < 2^53)."""
    k = np.asarray(k, dtype=np.int64)
    e = np.frexp(k.astype(np.float64))[1].astype(np.int64) - 1
    sh = np.maximum(e - 3, 0)
    return np.where(k < 8, k - 1, 7 + 8 * (e - 3) + (k >> sh) - 8)


def periodogram_bins(nc, fsamp):
    """(J, c, f) over the bins a segment's modes reach (empty bins dropped)."""
    n = len(nc)
    N = ot.fft_length(n)
    e = ot.extend(nc, N)
    I = np.abs(np.fft.rfft(e)) ** 2 / N
    M = N // 2
    k = np.arange(1, M + 1)
    b = bins_of(k)
    J = np.bincount(b, weights=I[1:], minlength=NBIN)
    c = np.bincount(b, minlength=NBIN).astype(np.float64)
    L = np.bincount(b, weights=np.log(k), minlength=NBIN)
    use = c > 0
    f = fsamp / N * np.exp(L[use] / c[use])
    return J[use], c[use], f


def alpha_mode(J, c, f, sigma0, fknee):
    """(alpha_hat, H): maximiser of the binned ln L in alpha and -d2 lnL/dalpha2;
    (nan, nan) when there is none."""
    x = np.log(f / fknee)
    a = J / sigma0 ** 2

    def score(al):
        with np.errstate(over="ignore", invalid="ignore"):  # far bracket ends of a flat ln L
            return float(np.sum(a * x * np.exp(-al * x) - c * x))

    # bracket the root by doubling, at most 60 times each way; no sign change
    # means ln L has no maximiser in alpha (all J_b = 0: a constant n_corr)
    lo, hi = -1.0, 1.0
    for _ in range(60):
        if not score(lo) < 0:
            break
        lo *= 2
    for _ in range(60):
        if not score(hi) > 0:
            break
        hi *= 2
    if not (score(lo) >= 0 and score(hi) <= 0):
        return np.nan, np.nan
    al = optimize.brentq(score, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    H = float(np.sum(a * x * x * np.exp(-al * x)))
    return al, H


def wilson_hilferty_chi2(n, z):
    return n * (1.0 - 2.0 / (9.0 * n) + z * np.sqrt(2.0 / (9.0 * n))) ** 3


def wilson_hilferty_gamma(K, z):
    return K * (1.0 - 1.0 / (9.0 * K) + z / (3.0 * np.sqrt(K))) ** 3


def noise_normals(seed, seg, it):
    z = philox.mode_normals(seed, seg, it, np.array([NOISE_COUNTER], dtype=np.uint64))
    return float(z[0][0]), float(z[1][0]), float(z[2][0])


def sample_noise_segment(d, t, g, nc, fsamp, fknee_old, seed, seg, it, mean_only=False):
    """(sigma0, fknee, alpha) of one segment."""
    d = np.asarray(d, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    nc = np.asarray(nc, dtype=np.float64)
    n = len(d)
    z0, z1, z2 = (0.0, 0.0, 0.0) if mean_only else noise_normals(seed, seg, it)
    r = d - g * t - nc
    S = float(r @ r)
    sigma0 = np.sqrt(S / wilson_hilferty_chi2(n, z0))
    J, c, f = periodogram_bins(nc, fsamp)
    ah, H = alpha_mode(J, c, f, sigma0, fknee_old)
    alpha = ah + z1 / np.sqrt(H)
    K = float(c.sum())
    Sa = float(np.sum(J * f ** (-alpha)))
    u = wilson_hilferty_gamma(K, z2) * sigma0 ** 2 / Sa
    fknee = u ** (1.0 / alpha)
    return sigma0, fknee, alpha


def sample_noise_all(ts, d, t, gain, nc, fknee_old, seed, it, mean_only=False, segs=None):
    out = np.full((3, ts.nseg), np.nan)
    for q in (range(ts.nseg) if segs is None else segs):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b == a:
            continue
        out[:, q] = sample_noise_segment(d[a:b], t[a:b], float(gain[q]), nc[a:b],
                                         float(ts.band_fsamp[ts.seg_band[q]]), float(fknee_old[q]),
                                         seed, q, it, mean_only)
    return out
