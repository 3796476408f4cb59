"""FP64 reference of the masked correlated-noise draw: a constrained
realisation solved by preconditioned conjugate gradients (gap filling).

Test infrastructure: only tests/, the smoke check and the bench CPU baseline
use it; the product path never does.

The paper names the step (the correlated-noise draw needs FFTs inside a CG
solver for gap filling, most of all where scans cross large processing masks;
section 5 and the correlated-noise row of Table 2) and defers its form to a
companion paper.  Reading used here, on the same mirrored, padded extension
as the unmasked draw (length N = fft_length(n), e = [r, reverse(r), r0 ...]):

* the mask is extended the same way, mu = [m, reverse(m), 1 ...] (the pad
  counts as observed, exactly as the unmasked draw treats it);
* with F the unitary DFT, 1/P_k the prior's inverse spectrum (1/P_0 = 0) and
  W1, W2 the unmasked draw's Philox modes (Hermitian-extended),
      A = F^H diag(1/P) F + diag(mu) / sigma0^2,
      b = mu (e / sigma0^2 + w1 / sigma0) + F^H (W2 sqrt(1/P)),   w1 = F^H W1;
  Cov(b) = A, so x = A^-1 b is a draw from N(A^-1 mu e / sigma0^2, A^-1), the
  posterior of the correlated noise given the unmasked samples;
* n_corr = x[0:n];
* preconditioner F^H diag(1 / (1/sigma0^2 + 1/P)) F: the exact inverse of A
  when nothing is masked, so that case is the unmasked draw after one step.
"""
import numpy as np

from . import tod as ot


def extend_mask(m, N):
    """[m, reverse(m), 1 ...] of length N (float 0/1)."""
    m = np.asarray(m, dtype=np.float64)
    n = len(m)
    mu = np.ones(N)
    mu[:n] = m
    mu[n:2 * n] = m[::-1]
    return mu


def _fwd(x):          # unitary DFT of a real vector, modes 0..N/2
    return np.fft.rfft(x) / np.sqrt(len(x))


def _inv(X, N):       # unitary inverse of a Hermitian half spectrum
    return np.sqrt(N) * np.fft.irfft(X, n=N)


def operator(x, invP, mu, sigma0):
    """A x."""
    N = len(x)
    return _inv(invP * _fwd(x), N) + mu * x / sigma0 ** 2


def preconditioner(y, invP, sigma0):
    """F^H diag(1 / (1/sigma0^2 + 1/P)) F y."""
    N = len(y)
    return _inv(_fwd(y) / (1.0 / sigma0 ** 2 + invP), N)


def rhs(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False):
    """(b, e, mu, invP) of one segment."""
    n = len(r)
    N = ot.fft_length(n)
    e = ot.extend(r, N)
    mu = extend_mask(m, N)
    invP = ot.inv_psd(N, fsamp, sigma0, fknee, alpha)
    b = mu * e / sigma0 ** 2
    if not mean_only:
        W1, W2 = ot.white_modes(seed, seg, it, N)
        b = b + mu * _inv(W1, N) / sigma0 + _inv(W2 * np.sqrt(invP), N)
    return b, e, mu, invP


def pcg(b, invP, mu, sigma0, tol, maxiter):
    """Preconditioned CG for A x = b from x = 0; stops when ||r|| <= tol ||b||.
    Returns (x, iterations)."""
    x = np.zeros_like(b)
    res = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = preconditioner(res, invP, sigma0)
    p = z.copy()
    rz = res @ z
    for i in range(1, maxiter + 1):
        Ap = operator(p, invP, mu, sigma0)
        a = rz / (p @ Ap)
        x += a * p
        res -= a * Ap
        if np.linalg.norm(res) <= tol * nb:
            return x, i
        z = preconditioner(res, invP, sigma0)
        rz_new = res @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxiter


def cg_ncorr_segment(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False,
                     tol=1e-12, maxiter=2000):
    """Masked n_corr draw of one segment: (n_corr [n], CG iterations)."""
    b, e, mu, invP = rhs(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only)
    x, k = pcg(b, invP, mu, sigma0, tol, maxiter)
    return x[:len(r)], k


def cg_ncorr_all(ts, d, s, mask, seed, it, mean_only=False, tol=1e-12, maxiter=2000, segs=None):
    """Masked draw for every segment (or the listed ones); zeros elsewhere."""
    out = np.zeros(ts.nsamp)
    iters = {}
    for q in (range(ts.nseg) if segs is None else segs):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b == a:
            continue
        band = int(ts.seg_band[q])
        out[a:b], iters[q] = cg_ncorr_segment(
            d[a:b] - s[a:b], mask[a:b], float(ts.band_fsamp[band]), float(ts.sigma0[q]),
            float(ts.fknee[q]), float(ts.alpha[q]), seed, q, it, mean_only, tol, maxiter)
    return out, iters


def dense_system(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False):
    """(A, b) as dense N x N / N arrays (small N only): A from the unitary DFT
    matrix, for checking the matrix-free operator and the CG solution."""
    b, e, mu, invP = rhs(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only)
    N = len(b)
    k = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(k, k) / N) / np.sqrt(N)
    full = np.empty(N)
    half = N // 2 + 1
    full[:half] = invP
    full[half:] = invP[1:N - half + 1][::-1]
    A = (F.conj().T @ np.diag(full) @ F).real + np.diag(mu / sigma0 ** 2)
    return A, b


def gap_cg(b, invP, mu, sigma0, tol, maxiter):
    """The same system solved on the masked samples only (Woodbury).  With S
    the selection of the extended positions where mu = 0 and M the
    preconditioner above, A = M^-1 - S S^T / sigma0^2, so
        x = x0 + M S y,   x0 = M b,   (sigma0^2 I - S^T M S) y = S^T x0,
    and b - A x = S rho / sigma0^2 with rho the residual of the small system.
    Plain CG from y = 0 (x = x0), stopping when ||rho|| <= tol ||rho_0||: the
    full residual, which lives on the masked samples, has fallen by tol from
    its value at x0.  Returns (x, iterations)."""
    N = len(b)
    x0 = preconditioner(b, invP, sigma0)
    gap = np.flatnonzero(mu == 0)
    if len(gap) == 0:
        return x0, 0

    def H(v):
        u = np.zeros(N)
        u[gap] = v
        return sigma0 ** 2 * v - preconditioner(u, invP, sigma0)[gap]

    y = np.zeros(len(gap))
    rho = x0[gap].copy()
    p = rho.copy()
    rr = rho @ rho
    k = 0
    stop = tol * np.sqrt(rr)
    if rr == 0.0:  # x0 is the solution
        return x0, 0
    for k in range(1, maxiter + 1):
        q = H(p)
        a = rr / (p @ q)
        y += a * p
        rho -= a * q
        rr_new = rho @ rho
        if np.sqrt(rr_new) <= stop:
            break
        p = rho + (rr_new / rr) * p
        rr = rr_new
    u = np.zeros(N)
    u[gap] = y
    return x0 + preconditioner(u, invP, sigma0), k


def cg_ncorr_segment_gap(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only=False,
                         tol=1e-12, maxiter=2000):
    """Masked n_corr draw of one segment through gap_cg: (n_corr [n], iterations)."""
    b, e, mu, invP = rhs(r, m, fsamp, sigma0, fknee, alpha, seed, seg, it, mean_only)
    x, k = gap_cg(b, invP, mu, sigma0, tol, maxiter)
    return x[:len(r)], k


def cg_ncorr_all_gap(ts, d, s, mask, seed, it, mean_only=False, tol=1e-12, maxiter=2000, segs=None):
    out = np.zeros(ts.nsamp)
    iters = {}
    for q in (range(ts.nseg) if segs is None else segs):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b == a:
            continue
        band = int(ts.seg_band[q])
        out[a:b], iters[q] = cg_ncorr_segment_gap(
            d[a:b] - s[a:b], mask[a:b], float(ts.band_fsamp[band]), float(ts.sigma0[q]),
            float(ts.fknee[q]), float(ts.alpha[q]), seed, q, it, mean_only, tol, maxiter)
    return out, iters
