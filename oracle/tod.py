"""FP64 reference of the TOD step: projection, correlated-noise draw, binning,
per-pixel solve, chi^2 and its gradients.

Test infrastructure only.  Everything is plain numpy in float64; the FFT is
numpy's pocketfft (any length), used as a library primitive.

Data model (Eq. 1 reduced to one pixelised sky, no beam, no orbital/sidelobe/
1 Hz terms):  d_t = g P_t m + n_corr,t + n_w,t, with the pointing row
P_t m = T[p_t] + Q[p_t] cos 2psi_t + U[p_t] sin 2psi_t and psi_t the centre
2 pi (b_t + 1/2)/4096 of the quantised angle bin b_t (section 4.1).

Correlated noise (the n_corr step of the Gibbs chain, Eq. 4) is drawn by a
Fourier-domain constrained realisation on the mirrored segment (section 4.2):

1. r = d - g P m
2. e = [r, reverse(r), r_0 ... r_0] of length N, the smallest even 5-smooth
   number >= 2n (mirroring makes the data periodic; the pad repeats r_0)
3. R = rfft(e) / sqrt(N)                      (unitary convention)
4. P_k = sigma0^2 (f_k / f_knee)^alpha, f_k = k f_samp / N, 1/P_0 := 0;
   nhat_k = (R_k/sigma0^2 + W1_k/sigma0 + W2_k sqrt(1/P_k)) / (1/sigma0^2 + 1/P_k)
   with W1, W2 independent unit complex white noise (real at k = 0, N/2)
5. n_corr = (sqrt(N) irfft(nhat))[0:n]

Binning (section 2.4: co-added on the fly, one synchronisation): with weight
w = g / sigma0^2 and v = d - n_corr,
  b_p = sum w v (1, c, s),   A_p = sum g w (1, c, s)^T (1, c, s),
(c, s) = (cos 2psi, sin 2psi); the map is A_p^-1 b_p where A_p is well
conditioned.

chi^2 (the likelihood evaluation) per segment:
  J = sum_t r_t^2 / sigma0^2 + sum_{k=1}^{N/2} (I_k / P_k + ln P_k),
with r = d - g P m - n_corr and I_k = |FFT(e(n_corr))_k|^2 / N.
"""
import numpy as np

from . import philox

NPSI = 4096


# ---------------------------------------------------------------- projection
def psi_angle(b):
    return 2.0 * np.pi * (np.asarray(b, dtype=np.float64) + 0.5) / NPSI


def pointing_rows(pix, psi):
    """(p, 1, cos 2psi, sin 2psi) for each sample."""
    a = psi_angle(psi)
    return np.asarray(pix, dtype=np.int64), np.cos(2.0 * a), np.sin(2.0 * a)


def project(maps, gp, psi, g):
    """s_t = g (T + Q cos 2psi + U sin 2psi) at global pixel gp."""
    p, c, s = pointing_rows(gp, psi)
    m = np.asarray(maps, dtype=np.float64)
    return np.asarray(g, dtype=np.float64) * (m[0, p] + m[1, p] * c + m[2, p] * s)


# ----------------------------------------------------------- FFT length & ext
def is_5smooth(m):
    m = int(m)
    if m < 1:
        return False
    for q in (2, 3, 5):
        while m % q == 0:
            m //= q
    return m == 1


def fft_length(n):
    """Smallest even 5-smooth integer >= 2n."""
    N = 2 * int(n)
    while not (N % 2 == 0 and is_5smooth(N)):
        N += 1
    return N


def extend(r, N):
    r = np.asarray(r, dtype=np.float64)
    n = len(r)
    e = np.empty(N)
    e[:n] = r
    e[n:2 * n] = r[::-1]
    e[2 * n:] = r[0]
    return e


# ------------------------------------------------------------ n_corr draw
def white_modes(seed, seg, it, N):
    """W1, W2 for modes k = 0..N/2 (complex; real at k = 0 and k = N/2)."""
    K = N // 2 + 1
    z0, z1, z2, z3 = philox.mode_normals(seed, seg, it, np.arange(K))
    W1 = (z0 + 1j * z1) / np.sqrt(2.0)
    W2 = (z2 + 1j * z3) / np.sqrt(2.0)
    W1[0], W2[0] = z0[0], z2[0]
    W1[-1], W2[-1] = z0[-1], z2[-1]
    return W1, W2


def inv_psd(N, fsamp, sigma0, fknee, alpha):
    k = np.arange(N // 2 + 1)
    f = k * fsamp / N
    invP = np.zeros(len(k))
    invP[1:] = 1.0 / (sigma0 ** 2 * (f[1:] / fknee) ** alpha)
    return invP


def sample_ncorr_segment(r, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False):
    n = len(r)
    if n == 0:  # an empty segment has nothing to draw
        return np.zeros(0)
    N = fft_length(n)
    e = extend(r, N)
    R = np.fft.rfft(e) / np.sqrt(N)
    invP = inv_psd(N, fsamp, sigma0, fknee, alpha)
    if mean_only:
        W1 = W2 = np.zeros(len(R))
    else:
        W1, W2 = white_modes(seed, seg, it, N)
    nhat = (R / sigma0 ** 2 + W1 / sigma0 + W2 * np.sqrt(invP)) / (1.0 / sigma0 ** 2 + invP)
    return (np.sqrt(N) * np.fft.irfft(nhat, n=N))[:n]


# ----------------------------------------------------------------- helpers
def global_pix(ts, pix):
    """Band-local pixel -> index into the concatenated maps."""
    off = np.repeat(ts.band_pix_off[ts.seg_band], np.diff(ts.seg_off))
    return np.asarray(pix, dtype=np.int64) + off


def per_sample(ts, arr):
    return np.repeat(np.asarray(arr), np.diff(ts.seg_off))


# -------------------------------------------------------------- full steps
def project_all(ts, maps, pix, psi):
    gp = global_pix(ts, pix)
    return project(maps, gp, psi, per_sample(ts, ts.gain))


def sample_ncorr_all(ts, d, s, seed, it, mean_only=False, segs=None):
    out = np.zeros(ts.nsamp)
    segs = range(ts.nseg) if segs is None else segs
    for q in segs:
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        r = np.asarray(d[a:b], dtype=np.float64) - np.asarray(s[a:b], dtype=np.float64)
        fs = ts.band_fsamp[ts.seg_band[q]]
        out[a:b] = sample_ncorr_segment(r, fs, ts.sigma0[q], ts.fknee[q], ts.alpha[q],
                                        seed, q, it, mean_only)
    return out


def bin_tod(ts, pix, psi, d, ncorr, gain=None, sigma0=None, accept=None):
    """(b [3][npix_total], A [6][npix_total] (TT,TQ,TU,QQ,QU,UU), hits)."""
    gain = ts.gain if gain is None else gain
    sigma0 = ts.sigma0 if sigma0 is None else sigma0
    acc = ts.seg_accept if accept is None else accept
    keep = per_sample(ts, acc).astype(bool)
    gp = global_pix(ts, pix)[keep]
    _, c, s = pointing_rows(gp, np.asarray(psi)[keep])
    g = per_sample(ts, gain)[keep]
    w = g / per_sample(ts, sigma0)[keep] ** 2
    v = np.asarray(d, dtype=np.float64)[keep] - np.asarray(ncorr, dtype=np.float64)[keep]
    npt = ts.npix_total
    b = np.zeros((3, npt))
    A = np.zeros((6, npt))
    one = np.ones_like(c)
    rows = (one, c, s)
    for i in range(3):
        np.add.at(b[i], gp, w * v * rows[i])
    pairs = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
    for q, (i, j) in enumerate(pairs):
        np.add.at(A[q], gp, g * w * rows[i] * rows[j])
    hits = np.bincount(gp, minlength=npt).astype(np.int64)
    return b, A, hits


def unpack_A(A):
    """[6][npix] -> [npix][3][3]."""
    TT, TQ, TU, QQ, QU, UU = A
    M = np.empty((A.shape[1], 3, 3))
    M[:, 0, 0], M[:, 0, 1], M[:, 0, 2] = TT, TQ, TU
    M[:, 1, 0], M[:, 1, 1], M[:, 1, 2] = TQ, QQ, QU
    M[:, 2, 0], M[:, 2, 1], M[:, 2, 2] = TU, QU, UU
    return M


def solve_maps(b, A, hits, rcond_min):
    """Per-pixel solve; NaN where hits < 3 or lambda_min/lambda_max < rcond_min."""
    M = unpack_A(A)
    npix = M.shape[0]
    ev = np.linalg.eigvalsh(M)
    with np.errstate(divide="ignore", invalid="ignore"):
        rc = np.where(ev[:, 2] > 0, ev[:, 0] / ev[:, 2], 0.0)
    ok = (np.asarray(hits) >= 3) & (rc >= rcond_min)
    m = np.full((3, npix), np.nan)
    if np.any(ok):
        m[:, ok] = np.linalg.solve(M[ok], b.T[ok][..., None])[..., 0].T
    return m, rc


# ---------------------------------------------------------------- chi^2
def whittle_parts(nc, fsamp, sigma0, fknee, alpha):
    """(I_k, P_k, f_k) for k = 1..N/2 on the extension of n_corr (no modes
    for an empty segment)."""
    n = len(nc)
    if n == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    N = fft_length(n)
    X = np.fft.rfft(extend(nc, N)) / np.sqrt(N)
    k = np.arange(1, N // 2 + 1)
    f = k * fsamp / N
    I = np.abs(X[1:]) ** 2
    P = sigma0 ** 2 * (f / fknee) ** alpha
    return I, P, f


def chisq_segment(r, nc, fsamp, sigma0, fknee, alpha):
    I, P, _ = whittle_parts(nc, fsamp, sigma0, fknee, alpha)
    return float(np.sum(r * r) / sigma0 ** 2 + np.sum(I / P + np.log(P)))


def chisq_all(ts, maps, pix, psi, d, ncorr, gain=None, sigma0=None, fknee=None, alpha=None):
    gain = ts.gain if gain is None else np.asarray(gain, dtype=np.float64)
    sigma0 = ts.sigma0 if sigma0 is None else np.asarray(sigma0, dtype=np.float64)
    fknee = ts.fknee if fknee is None else np.asarray(fknee, dtype=np.float64)
    alpha = ts.alpha if alpha is None else np.asarray(alpha, dtype=np.float64)
    gp = global_pix(ts, pix)
    out = np.zeros(ts.nseg)
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        sq = project(maps, gp[a:b], psi[a:b], gain[q])
        nc = np.asarray(ncorr[a:b], dtype=np.float64)
        r = np.asarray(d[a:b], dtype=np.float64) - sq - nc
        out[q] = chisq_segment(r, nc, ts.band_fsamp[ts.seg_band[q]], sigma0[q], fknee[q], alpha[q])
    return out


def chisq_grad_all(ts, maps, pix, psi, d, ncorr, gain=None, sigma0=None, fknee=None, alpha=None):
    """Analytic gradients of sum_seg J:
    dJ/dm = -2 P^T (g r / sigma0^2), dJ/dg = -2 sum (Pm) r / sigma0^2 per segment,
    dJ/dsigma0 = -2 sum r^2/sigma0^3 + sum_k (2/sigma0)(1 - I/P),
    dJ/df_knee = sum_k (1 - I/P)(-alpha/f_knee), dJ/dalpha = sum_k (1 - I/P) ln(f/f_knee),
    the last three per segment (sum over a detector's segments for per-detector
    parameters)."""
    gain = ts.gain if gain is None else np.asarray(gain, dtype=np.float64)
    sigma0 = ts.sigma0 if sigma0 is None else np.asarray(sigma0, dtype=np.float64)
    fknee = ts.fknee if fknee is None else np.asarray(fknee, dtype=np.float64)
    alpha = ts.alpha if alpha is None else np.asarray(alpha, dtype=np.float64)
    gp = global_pix(ts, pix)
    gm = np.zeros((3, ts.npix_total))
    gg = np.zeros(ts.nseg)
    gs = np.zeros(ts.nseg)
    gf = np.zeros(ts.nseg)
    ga = np.zeros(ts.nseg)
    m = np.asarray(maps, dtype=np.float64)
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        p, c, s = pointing_rows(gp[a:b], psi[a:b])
        Pm = m[0, p] + m[1, p] * c + m[2, p] * s
        nc = np.asarray(ncorr[a:b], dtype=np.float64)
        r = np.asarray(d[a:b], dtype=np.float64) - gain[q] * Pm - nc
        coef, gg[q], gs[q], gf[q], ga[q] = chisq_grad_segment(
            r, Pm, nc, ts.band_fsamp[ts.seg_band[q]], gain[q], sigma0[q], fknee[q], alpha[q])
        np.add.at(gm[0], p, coef)
        np.add.at(gm[1], p, coef * c)
        np.add.at(gm[2], p, coef * s)
    return gm, gg, gs, gf, ga


def chisq_grad_segment(r, Pm, nc, fsamp, gain, sigma0, fknee, alpha):
    """One segment's terms of chisq_grad_all, for the residual r = d - g Pm - nc:
    (coef, dJ/dg, dJ/dsigma0, dJ/df_knee, dJ/dalpha), coef = -2 g r / sigma0^2
    being the per-sample weight that P^T spreads into the map gradient."""
    coef = -2.0 * gain * r / sigma0 ** 2
    gg = -2.0 * np.sum(Pm * r) / sigma0 ** 2
    I, P, f = whittle_parts(nc, fsamp, sigma0, fknee, alpha)
    u = 1.0 - I / P
    gs = -2.0 * np.sum(r * r) / sigma0 ** 3 + np.sum(2.0 / sigma0 * u)
    gf = np.sum(u * (-alpha / fknee))
    ga = np.sum(u * np.log(f / fknee))
    return coef, float(gg), float(gs), float(gf), float(ga)
