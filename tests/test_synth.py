"""Generator checks: determinism and the HEALPix pixelisation it relies on."""
import numpy as np
import pytest

import synth
from synth import healpix as hp


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 512])
def test_pixel_centres_round_trip(nside):
    p = np.arange(hp.npix_of(nside)) if nside <= 64 else \
        np.random.default_rng(0).integers(0, hp.npix_of(nside), 200000)
    th, ph = hp.pix2ang_ring(nside, p)
    assert np.array_equal(hp.ang2pix_ring(nside, th, ph), p)


@pytest.mark.parametrize("nside", [1, 4, 16])
def test_ring_layout(nside):
    """4*nside-1 rings; polar ring i has 4i pixels, equatorial rings 4*nside."""
    p = np.arange(hp.npix_of(nside))
    th, _ = hp.pix2ang_ring(nside, p)
    z = np.round(np.cos(th), 12)
    zs, counts = np.unique(z, return_counts=True)
    assert len(zs) == 4 * nside - 1
    counts = counts[::-1]  # north to south
    expect = [min(4 * i, 4 * nside, 4 * (4 * nside - i)) for i in range(1, 4 * nside)]
    assert list(counts) == expect


def test_equal_area():
    """Uniform points on the sphere fill the 768 pixels of nside 8 evenly (chi^2)."""
    rng = np.random.default_rng(1)
    n = 768 * 400
    z = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    c = np.bincount(hp.ang2pix_ring(8, np.arccos(z), phi), minlength=768)
    chi2 = np.sum((c - 400.0) ** 2 / 400.0)
    # 767 dof: mean 767, sd ~39
    assert abs(chi2 - 767) < 6 * 39.2


def test_neighbouring_points_neighbouring_pixels():
    """Walking along the latitude of a ring centre stays on that ring and moves at
    most one pixel per tiny step (the equatorial ring, z = 0, and a polar ring)."""
    nside = 32
    phi = np.linspace(0, 2 * np.pi, 20000, endpoint=False) + 1e-7
    p = hp.ang2pix_ring(nside, np.full_like(phi, np.pi / 2), phi)
    d = np.diff(p)
    assert set(np.unique(d)).issubset({0, 1, -(4 * nside - 1)})
    i = 5                                              # polar ring with 4i pixels
    z = 1.0 - i * i / (3.0 * nside * nside)
    p = hp.ang2pix_ring(nside, np.full_like(phi, np.arccos(z)), phi)
    assert p.min() == 2 * i * (i - 1) and p.max() == 2 * i * (i - 1) + 4 * i - 1
    assert set(np.unique(np.diff(p))).issubset({0, 1, -(4 * i - 1)})


def test_generator_deterministic():
    a = synth.make(0)
    b = synth.make(0)
    assert np.array_equal(a.d, b.d)
    assert np.array_equal(a.pix_huff.words, b.pix_huff.words)
    assert np.array_equal(a.psi_huff.words, b.psi_huff.words)
    assert np.array_equal(a.maps, b.maps)


def test_generator_shapes(tiny):
    ts = tiny
    assert ts.nseg == 8 and ts.nsamp == 8 * 4096
    assert ts.d.dtype == np.float64
    assert ts.pix.max() < 12 * 16 * 16 and ts.pix.min() >= 0
    assert ts.psi.max() < 4096
    assert np.allclose(ts.sigma0, 1.0) and np.allclose(ts.fknee, 0.1) and np.allclose(ts.alpha, -1.5)


def test_mixed_band_layout():
    ts = synth.make(4, nscan=6, length=("loguniform2", 10.0, 11.0))
    assert ts.nband == 3
    assert list(ts.band_pix_off) == [0, 12 * 256 ** 2, 12 * 256 ** 2 + 12 * 512 ** 2]
    # detectors per band 4/6/12, two scans per band
    assert ts.nseg == 2 * (4 + 6 + 12)
    assert ts.ndet == 22
