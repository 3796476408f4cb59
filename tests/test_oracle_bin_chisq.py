"""Pin the oracle's projection, binning/solve and chi^2 with its gradients."""
import numpy as np
import pytest

import synth
from oracle import huffman as oh
from oracle import tod as ot


@pytest.fixture(scope="module")
def small():
    ts = synth.make(0, nscan=3, length=("uniform", 300, 420), keep_truth=True)
    rng = np.random.default_rng(11)
    ts.sigma0 = rng.uniform(0.5, 2.0, ts.nseg)        # exercise the weights
    ts.gain = 1.0 + 0.1 * rng.normal(size=ts.nseg)
    return ts


def test_projection_unit_maps(tiny):
    ts = tiny
    pix, psi = ts.pix, ts.psi
    g = ot.per_sample(ts, ts.gain)
    ang = 2 * np.pi * (psi + 0.5) / 4096
    for i, expect in enumerate([g, g * np.cos(2 * ang), g * np.sin(2 * ang)]):
        m = np.zeros((3, ts.npix_total))
        m[i] = 1.0
        assert np.allclose(ot.project_all(ts, m, pix, psi), expect, atol=1e-15)


def test_projection_stokes_rotation():
    """Rotating psi by 45 degrees turns Q into U: (0,1,0) at psi+pi/4 equals
    -(0,0,1) at psi... checked through sin/cos of 2psi on exact bin shifts."""
    gp = np.array([0, 1, 2])
    b = np.array([10, 700, 3000])
    m = np.array([[0.0] * 3, [1.0] * 3, [0.0] * 3])
    q = ot.project(m, gp, b + 1024, 1.0)            # +1024 bins = +pi/2 in psi
    assert np.allclose(q, -ot.project(m, gp, b, 1.0), atol=1e-14)


def test_noiseless_round_trip(small):
    ts = small
    d = ot.project_all(ts, ts.maps, ts.pix, ts.psi)
    b, A, hits = ot.bin_tod(ts, ts.pix, ts.psi, d, np.zeros(ts.nsamp))
    m, rc = ot.solve_maps(b, A, hits, 1e-3)
    ok = ~np.isnan(m[0])
    assert ok.sum() > 20
    assert np.all(np.abs(m[:, ok] - ts.maps[:, ok]) <= 1e-12 * np.abs(ts.maps).max())
    assert np.array_equal(hits, np.bincount(ot.global_pix(ts, ts.pix), minlength=ts.npix_total))
    M = ot.unpack_A(A)
    assert np.allclose(M, np.transpose(M, (0, 2, 1)))
    assert np.all(np.linalg.eigvalsh(M)[:, 0] >= -1e-12 * np.abs(M).max())


def test_rejected_segments_do_not_bin(small):
    ts = small
    acc = ts.seg_accept.copy()
    acc[1] = 0
    d = ot.project_all(ts, ts.maps, ts.pix, ts.psi)
    _, _, hits = ot.bin_tod(ts, ts.pix, ts.psi, d, np.zeros(ts.nsamp), accept=acc)
    assert hits.sum() == ts.nsamp - (ts.seg_off[2] - ts.seg_off[1])


def _J(ts, maps, d, nc, **kw):
    return ot.chisq_all(ts, maps, ts.pix, ts.psi, d, nc, **kw).sum()


@pytest.fixture(scope="module")
def chi_inputs(small):
    ts = small
    nc = ot.sample_ncorr_all(ts, ts.d, ot.project_all(ts, ts.maps, ts.pix, ts.psi), 99, 0)
    maps = ts.maps + np.random.default_rng(4).normal(size=ts.maps.shape)
    return ts, maps, nc


def test_map_gradient_is_binning_residual(chi_inputs):
    """dJ/dm = -2 (b - A m) with b, A from the binning of the same inputs."""
    ts, maps, nc = chi_inputs
    gm = ot.chisq_grad_all(ts, maps, ts.pix, ts.psi, ts.d, nc)[0]
    b, A, _ = ot.bin_tod(ts, ts.pix, ts.psi, ts.d, nc)
    M = ot.unpack_A(A)
    Am = np.einsum("pij,jp->ip", M, maps)
    assert np.allclose(gm, -2 * (b - Am), rtol=1e-10, atol=1e-9)


def test_finite_differences(chi_inputs):
    ts, maps, nc = chi_inputs
    gm, gg, gs, gf, ga = ot.chisq_grad_all(ts, maps, ts.pix, ts.psi, ts.d, nc)
    h = 1e-6

    def fd(fn, x0):
        return (fn(x0 + h) - fn(x0 - h)) / (2 * h)

    q = 1
    a, bq = ts.seg_off[q], ts.seg_off[q + 1]
    fs = ts.band_fsamp[0]
    gp = ot.global_pix(ts, ts.pix)

    def seg_J(g=None, s0=None, fk=None, al=None):
        g = ts.gain[q] if g is None else g
        s0 = ts.sigma0[q] if s0 is None else s0
        fk = ts.fknee[q] if fk is None else fk
        al = ts.alpha[q] if al is None else al
        sq = ot.project(maps, gp[a:bq], ts.psi[a:bq], g)
        r = ts.d[a:bq] - sq - nc[a:bq]
        return ot.chisq_segment(r, nc[a:bq], fs, s0, fk, al)

    for val, fn, x0 in [(gg[q], lambda x: seg_J(g=x), ts.gain[q]),
                        (gs[q], lambda x: seg_J(s0=x), ts.sigma0[q]),
                        (gf[q], lambda x: seg_J(fk=x), ts.fknee[q]),
                        (ga[q], lambda x: seg_J(al=x), ts.alpha[q])]:
        assert np.isclose(val, fd(fn, x0), rtol=1e-6, atol=1e-6)
    # a few single map coordinates, through the full objective
    for (i, p) in [(0, int(gp[5])), (1, int(gp[a + 7])), (2, int(gp[-3]))]:
        def Jm(x):
            mm = maps.copy()
            mm[i, p] = x
            return _J(ts, mm, ts.d, nc)
        assert np.isclose(gm[i, p], fd(Jm, maps[i, p]), rtol=1e-5, atol=1e-5)


def test_stationary_points(chi_inputs):
    """Gain and sigma0 gradients vanish at their closed-form optima."""
    ts, maps, nc = chi_inputs
    q = 0
    a, b = ts.seg_off[q], ts.seg_off[q + 1]
    gp = ot.global_pix(ts, ts.pix)
    Pm = ot.project(maps, gp[a:b], ts.psi[a:b], 1.0)
    v = ts.d[a:b] - nc[a:b]
    g_star = np.sum(Pm * v) / np.sum(Pm * Pm)
    gain = ts.gain.copy()
    gain[q] = g_star
    gg = ot.chisq_grad_all(ts, maps, ts.pix, ts.psi, ts.d, nc, gain=gain)[1]
    assert abs(gg[q]) < 1e-8 * np.sum(Pm * Pm)
    # sigma0^2 = (sum r^2 + sum_k I_k / q_k) / K with q_k = (f_k/f_knee)^alpha
    r = v - g_star * Pm
    I, P, f = ot.whittle_parts(nc[a:b], ts.band_fsamp[0], 1.0, ts.fknee[q], ts.alpha[q])
    K = len(I)
    s2 = (np.sum(r * r) + np.sum(I / P)) / K
    sig = ts.sigma0.copy()
    sig[q] = np.sqrt(s2)
    gs = ot.chisq_grad_all(ts, maps, ts.pix, ts.psi, ts.d, nc, gain=gain, sigma0=sig)[2]
    assert abs(gs[q]) < 1e-8 * K


def test_decode_then_project_pipeline(tiny):
    pix, psi = oh.decode_pointing(tiny)
    s = ot.project_all(tiny, tiny.maps, pix, psi)
    resid = tiny.d - s
    # the synthetic data are signal + noise: the residual has the noise's size
    assert 0.3 < resid.std() < 10.0
