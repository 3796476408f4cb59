"""The oracle on degenerate segment lengths.

The edge set: eight scans of 0, 1, 2, 3, 17, 130, 4097 and 0 samples, each
seen by the two radiometers of one horn at nside 16.  It holds empty
segments, one- to three-sample segments, segments shorter than one
side-index chunk, and ragged tails of every kind.  Pins:

* the four streams decode to the generator's arrays;
* a constant residual, of any length and hence every one-sample residual,
  has a mean-only n_corr equal to itself.  Its extension is constant, so all
  its power sits in the DC mode, which the prior leaves free (1/P_0 = 0);
* an empty segment has no n_corr, chi^2 = 0 with zero gradients, and NaN
  gain and noise parameters;
* a one-sample segment has no gain draw (NaN).  Its template has no power
  outside DC, so A = 0.  Its periodogram is zero, so alpha and f_knee have no
  conditional maximum (NaN);
* every other segment gives finite draws.
"""
import numpy as np
import pytest

import synth
from oracle import gain as og
from oracle import huffman as oh
from oracle import noise as on
from oracle import tod as ot
from synth.configs import Band

EDGE_LENGTHS = ("list", 0, 1, 2, 3, 17, 130, 4097, 0)


def make_edge():
    return synth.make(0, nscan=8, length=EDGE_LENGTHS, bands=(Band(16, 32.5, 2),), keep_truth=True,
                      tod_streams=True)


@pytest.fixture(scope="module")
def edge():
    ts = make_edge()
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, 91, 2)
    return ts, s, nc


def _lens(ts):
    return np.diff(ts.seg_off)


def test_edge_set_shape(edge):
    ts, _, _ = edge
    assert list(_lens(ts)) == [0, 0, 1, 1, 2, 2, 3, 3, 17, 17, 130, 130, 4097, 4097, 0, 0]


def test_edge_streams_decode(edge):
    ts, _, _ = edge
    pix, psi = oh.decode_pointing(ts)
    assert np.array_equal(pix, ts.pix) and np.array_equal(psi, ts.psi)
    assert np.array_equal(oh.decode_tod(ts), ts.d.astype(np.float64))
    fl = oh.decode_stream(ts, ts.flag_huff)
    assert fl.shape == (ts.nsamp,) and (fl >= 0).all()


@pytest.mark.parametrize("n", [1, 2, 5, 17, 4097])
def test_constant_residual_is_its_own_mean_draw(n):
    r = np.full(n, -2.75)
    for fs, s0, fk, al in [(32.5, 1.0, 0.1, -1.5), (78.8, 2.3, 0.05, -1.0)]:
        x = ot.sample_ncorr_segment(r, fs, s0, fk, al, 3, 0, 0, mean_only=True)
        assert np.allclose(x, r, rtol=0, atol=1e-12)


def test_empty_segments(edge):
    ts, s, nc = edge
    empty = np.flatnonzero(_lens(ts) == 0)
    assert len(empty) == 4
    J = ot.chisq_all(ts, ts.maps, ts.pix, ts.psi, ts.d, nc)
    gm, gg, gs, gf, ga = ot.chisq_grad_all(ts, ts.maps, ts.pix, ts.psi, ts.d, nc)
    assert np.all(J[empty] == 0) and np.all(gg[empty] == 0) and np.all(gs[empty] == 0)
    t = ot.project(ts.maps, ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    g, sg = og.sample_gain_all(ts, ts.d, t, 91, 2)
    assert np.isnan(g[empty]).all()
    xi = on.sample_noise_all(ts, ts.d, t, ts.gain, nc, ts.fknee, 91, 2)
    assert np.isnan(xi[:, empty]).all()


def test_one_sample_segments(edge):
    ts, s, nc = edge
    one = np.flatnonzero(_lens(ts) == 1)
    t = ot.project(ts.maps, ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    for q in one:
        a = ts.seg_off[q]
        _, _, A, _ = og.sample_gain_segment(ts.d[a:a + 1], t[a:a + 1], 32.5, ts.sigma0[q], ts.fknee[q],
                                            ts.alpha[q], 91, q, 2)
        assert A == 0.0
        J, c, f = on.periodogram_bins(nc[a:a + 1], 32.5)
        assert np.all(J == 0) and len(c) == 1
    g, _ = og.sample_gain_all(ts, ts.d, t, 91, 2)
    assert np.isnan(g[one]).all()
    with np.errstate(invalid="ignore"):
        xi = on.sample_noise_all(ts, ts.d, t, ts.gain, nc, ts.fknee, 91, 2)
    assert np.isnan(xi[1:, one]).all()


def test_longer_segments_finite(edge):
    ts, s, nc = edge
    big = np.flatnonzero(_lens(ts) >= 2)
    t = ot.project(ts.maps, ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    g, sg = og.sample_gain_all(ts, ts.d, t, 91, 2)
    assert np.isfinite(g[big]).all() and np.isfinite(sg[big]).all()
    xi = on.sample_noise_all(ts, ts.d, t, ts.gain, nc, ts.fknee, 91, 2, mean_only=True)
    assert np.isfinite(xi[:, big]).all()
    assert np.isfinite(nc).all()
