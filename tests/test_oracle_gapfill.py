"""Pins of the masked correlated-noise draw (CG gap filling) in the oracle.

The matrix-free operator equals the dense matrix built from the DFT; the CG
solution equals a dense solve; with nothing masked the draw is the unmasked
draw sample for sample (same Philox modes) after one preconditioned step; the
two-draw right-hand side has covariance A (so x ~ N(mean, A^-1)); masked
samples do not influence the result.
"""
import numpy as np

from oracle import gapfill as og
from oracle import tod as ot

PAR = dict(fsamp=32.5, sigma0=1.3, fknee=0.4, alpha=-1.5)


def _r(n, seed=0):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.normal(size=n)) * 0.2 + rng.normal(size=n)


def _mask(n, a, b):
    m = np.ones(n)
    m[a:b] = 0
    return m


def test_operator_matches_dense():
    n = 21
    r, m = _r(n), _mask(n, 5, 12)
    A, b = og.dense_system(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 7, 0, 2)
    N = len(b)
    _, _, mu, invP = og.rhs(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 7, 0, 2)
    x = np.random.default_rng(3).normal(size=N)
    assert np.allclose(og.operator(x, invP, mu, PAR["sigma0"]), A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())
    assert np.allclose(A, A.T, atol=1e-13)
    assert np.linalg.eigvalsh(A).min() > 0


def test_cg_matches_dense_solve():
    n = 37
    r, m = _r(n, 1), _mask(n, 9, 25)
    for mean_only in (True, False):
        A, b = og.dense_system(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 11, 3, 5,
                               mean_only)
        ref = np.linalg.solve(A, b)[:n]
        got, k = og.cg_ncorr_segment(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 11, 3, 5,
                                     mean_only, tol=1e-14)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        assert k < 200


def test_unmasked_is_the_fourier_draw():
    n = 300
    r = _r(n, 2)
    for mean_only in (True, False):
        ref = ot.sample_ncorr_segment(r, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 5, 4, 9,
                                      mean_only)
        got, k = og.cg_ncorr_segment(r, np.ones(n), PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"],
                                     5, 4, 9, mean_only, tol=1e-13)
        assert k == 1
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_rhs_covariance_is_A():
    """Push every unit normal of the Philox stream through the right-hand side's
    random part: the sum of the outer products is A (two-draw form)."""
    n = 12
    m = _mask(n, 3, 7)
    s0 = PAR["sigma0"]
    N = ot.fft_length(n)
    mu = og.extend_mask(m, N)
    invP = ot.inv_psd(N, PAR["fsamp"], s0, PAR["fknee"], PAR["alpha"])
    K = N // 2 + 1
    cols = []
    for which in (1, 2):
        for k in range(K):
            for part in ((1.0,) if k in (0, K - 1) else (1.0, 1j)):
                W = np.zeros(K, dtype=complex)
                W[k] = part if k in (0, K - 1) else part / np.sqrt(2.0)
                if which == 1:
                    cols.append(mu * og._inv(W, N) / s0)
                else:
                    cols.append(og._inv(W * np.sqrt(invP), N))
    J = np.array(cols).T
    A, _ = og.dense_system(np.zeros(n), m, PAR["fsamp"], s0, PAR["fknee"], PAR["alpha"], 0, 0, 0, True)
    assert np.allclose(J @ J.T, A, rtol=0, atol=1e-12 * np.abs(A).max())


def test_masked_samples_do_not_matter():
    n = 200
    r, m = _r(n, 4), _mask(n, 50, 120)
    r2 = r.copy()
    r2[50:120] += np.random.default_rng(9).normal(size=70) * 100
    a, _ = og.cg_ncorr_segment(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 1, 2, 3)
    b, _ = og.cg_ncorr_segment(r2, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 1, 2, 3)
    assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()


def test_gap_space_solver_matches_dense_and_full_cg():
    """The Woodbury form on the masked samples reaches the same solution as the
    dense solve and the full-system CG; no masked sample: x = M b, no iteration."""
    n = 64
    r, m = _r(n, 5), _mask(n, 10, 30)
    for mean_only in (True, False):
        A, b = og.dense_system(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 2, 1, 4,
                               mean_only)
        ref = np.linalg.solve(A, b)[:n]
        got, k = og.cg_ncorr_segment_gap(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 2, 1, 4,
                                         mean_only, tol=1e-14)
        full, kf = og.cg_ncorr_segment(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 2, 1, 4,
                                       mean_only, tol=1e-14)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(got - full).max() <= 1e-12 * np.abs(ref).max()
        assert 0 < k <= kf + 1
    un, k0 = og.cg_ncorr_segment_gap(r, np.ones(n), PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"],
                                     2, 1, 4)
    assert k0 == 0
    ref = ot.sample_ncorr_segment(r, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 2, 1, 4)
    assert np.abs(un - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gap_residual_identity():
    """b - A x = S rho / sigma0^2 for any y (the Woodbury algebra the stopping
    rule relies on)."""
    n = 40
    r, m = _r(n, 6), _mask(n, 7, 19)
    b, e, mu, invP = og.rhs(r, m, PAR["fsamp"], PAR["sigma0"], PAR["fknee"], PAR["alpha"], 3, 0, 1)
    s0 = PAR["sigma0"]
    N = len(b)
    gap = np.flatnonzero(mu == 0)
    x0 = og.preconditioner(b, invP, s0)
    y = np.random.default_rng(1).normal(size=len(gap))
    u = np.zeros(N)
    u[gap] = y
    x = x0 + og.preconditioner(u, invP, s0)
    rho = x0[gap] - (s0 ** 2 * y - og.preconditioner(u, invP, s0)[gap])
    full = b - og.operator(x, invP, mu, s0)
    expect = np.zeros(N)
    expect[gap] = rho / s0 ** 2
    assert np.abs(full - expect).max() <= 1e-11 * np.abs(b).max()
