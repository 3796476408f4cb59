"""FP64 reference of the per-segment gain draw, g <- P(g | d, xi_n, sky).

Test infrastructure: only tests/, the smoke check and the bench CPU baseline
use it; the product path never does.

The Gibbs chain samples the gain first, conditioned on the data, the noise
parameters and the sky but not on n_corr (Eq. 3), so the correlated noise is
marginalised: its covariance joins the white noise in N.  The paper names the
step and its use of FFTs (section 4.2: FFTs serve both the correlated-noise
and the gain steps) and defers the gain model to a companion paper.  Reading
used here, per segment (one scan of one detector), with the sky template
t = P m (unit gain) and d = g t + n, n ~ N(0, N):

* N is stationary with spectrum sigma0^2 + P_k, P_k = sigma0^2 (f_k/f_knee)^alpha,
  and N^-1 acts on the same mirrored, padded extension as the n_corr draw:
      K x = first n samples of F^H diag(h) F ext(x),   h_k = 1/(sigma0^2 + P_k),
  h_0 = 0 (the DC mode is wholly correlated noise: no gain information);
* A = t . K t,  B = t . K d  (the GLS normal equations; K d rather than
  (K t) . d, so a constant offset of d has no effect);
* g = B/A + eta / sqrt(A), eta ~ N(0, 1) from the Philox stream of the segment
  at the counter word k = 2^32 - 1 (no Fourier mode uses it); mean_only: eta = 0;
* a flat prior; no smoothing of the gain across scans;
* A <= 0 (the template has no power outside the DC mode, as for a one-sample
  segment, or the segment is empty): no draw, g = NaN and sigma_g = inf.
"""
import numpy as np

from . import philox
from . import tod as ot

GAIN_COUNTER = 0xFFFFFFFF


def gain_filter(N, fsamp, sigma0, fknee, alpha):
    """h_k = 1 / (sigma0^2 + P_k) for k = 0..N/2, h_0 = 0."""
    k = np.arange(N // 2 + 1)
    f = k * fsamp / N
    h = np.zeros(len(k))
    h[1:] = 1.0 / (sigma0 ** 2 + sigma0 ** 2 * (f[1:] / fknee) ** alpha)
    return h


def inv_noise(x, fsamp, sigma0, fknee, alpha):
    """K x: N^-1 applied on the mirrored extension, first n samples."""
    n = len(x)
    N = ot.fft_length(n)
    e = ot.extend(x, N)
    h = gain_filter(N, fsamp, sigma0, fknee, alpha)
    return np.fft.irfft(h * np.fft.rfft(e), n=N)[:n]


def gain_normal(seed, seg, it):
    z0, _, _, _ = philox.mode_normals(seed, seg, it, np.array([GAIN_COUNTER], dtype=np.uint64))
    return float(z0[0])


def sample_gain_segment(d, t, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False):
    """(g, sigma_g, A, B) of one segment."""
    d = np.asarray(d, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    A = float(t @ inv_noise(t, fsamp, sigma0, fknee, alpha))
    B = float(t @ inv_noise(d, fsamp, sigma0, fknee, alpha))
    if not A > 0.0:  # no information outside the DC mode (e.g. one sample): no draw
        return np.nan, np.inf, A, B
    sig = 1.0 / np.sqrt(A)
    g = B / A
    if not mean_only:
        g += sig * gain_normal(seed, seg, it)
    return g, sig, A, B


def sample_gain_all(ts, d, t, seed, it, mean_only=False, segs=None):
    """Per-segment gains and sigmas (NaN for empty segments)."""
    g = np.full(ts.nseg, np.nan)
    sg = np.full(ts.nseg, np.nan)
    for q in (range(ts.nseg) if segs is None else segs):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b == a:
            continue
        band = int(ts.seg_band[q])
        g[q], sg[q], _, _ = sample_gain_segment(
            d[a:b], t[a:b], float(ts.band_fsamp[band]), float(ts.sigma0[q]), float(ts.fknee[q]),
            float(ts.alpha[q]), seed, q, it, mean_only)
    return g, sg
