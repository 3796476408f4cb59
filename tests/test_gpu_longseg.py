"""Long segments: the largest transforms of the set against the oracle, and
the error for a segment beyond every FFT plan.

Segments of 524,288, 3,000,000 and 6,000,000 samples (one detector at
32.5 Hz, nside 16).  Their transforms have M = 2^19, 3e6 and 6e6 complex
points.  The FP32 plans split them into LDS column tiles of 128, 600 and
1200 points with rows of 4096 and 5000.  The FP64 plans reach
2048 x 2520 complex points, so the 6e6-sample segment has no FP64 plan: that
call fails on the host with TOD_ENOTSUP, before any launch.  The two shorter
segments run in FP64 on a layout without it, and carry the gain and
noise-parameter draws too.  Bars: 1e-5 relative per segment (FP32 path) and
1e-12 (FP64); the fused sweep's n_corr 3e-5 (its residual d - s is rounded to
FP32 before the transforms).
"""
import types

import numpy as np
import pytest
import torch

import synth
from oracle import tod as ot
from synth.configs import Band

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}
LONG = ("list", 524288, 3000000, 6000000)
_DATA = {}


def data():
    if not _DATA:
        _DATA["ts"] = synth.make(0, nscan=3, length=LONG, bands=(Band(16, 32.5, 1),), keep_truth=True)
    return _DATA["ts"]


def first_segments(ts, k):
    """A view of the set with its first k segments only (the streams stay whole)."""
    v = types.SimpleNamespace(**vars(ts))
    v.nseg = k
    v.seg_off = ts.seg_off[:k + 1].copy()
    v.nsamp = int(v.seg_off[-1])
    for a in ("seg_scan", "seg_det", "seg_band", "seg_accept", "gain", "sigma0", "fknee", "alpha"):
        setattr(v, a, getattr(ts, a)[:k].copy())
    v.d = ts.d[:v.nsamp]
    v.pix, v.psi = ts.pix[:v.nsamp], ts.psi[:v.nsamp]
    return v


def seg_rel(ts, got, ref):
    errs = []
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        errs.append(np.linalg.norm(got[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]))
    return max(errs)


def _ncorr(ts, prec):
    from paper_2201_03509_amd import ops
    nf, tf = (np.float32, torch.float32) if prec == "mixed" else (np.float64, torch.float64)
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi).astype(nf)
    seed, it = 41, 2
    ref = ot.sample_ncorr_all(ts, ts.d, s.astype(np.float64), seed, it)
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        out = torch.empty(ts.nsamp, dtype=tf, device="cuda")
        c.sample_ncorr(tod, prec, tod.d, torch.from_numpy(s).cuda(), seed, it, out)
        c.sync()
    finally:
        c.close()
    return seg_rel(ts, out.cpu().numpy().astype(np.float64), ref)


def test_long_ncorr_mixed():
    err = _ncorr(data(), "mixed")
    print("mixed max segment rel L2 %.2e" % err)
    assert err < TOL["mixed"]


def test_long_ncorr_fp64():
    err = _ncorr(first_segments(data(), 2), "fp64")
    print("fp64 max segment rel L2 %.2e" % err)
    assert err < TOL["fp64"]


def test_beyond_fp64_plans_rejected():
    from paper_2201_03509_amd import _lib as L
    from paper_2201_03509_amd import ops
    ts = data()
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        s = torch.zeros(ts.nsamp, dtype=torch.float64, device="cuda")
        out = torch.empty(ts.nsamp, dtype=torch.float64, device="cuda")
        with pytest.raises(ops.C3todError) as e:
            c.sample_ncorr(tod, "fp64", tod.d, s, 1, 0, out)
        assert e.value.status == L.TOD_ENOTSUP
        # the context stays usable: the mixed path takes the same layout
        s32 = torch.zeros(ts.nsamp, dtype=torch.float32, device="cuda")
        o32 = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        c.sample_ncorr(tod, "mixed", tod.d, s32, 1, 0, o32)
        c.sync()
        assert torch.isfinite(o32).all().item()
    finally:
        c.close()


def test_long_sweep_mixed():
    from paper_2201_03509_amd import ops
    ts = data()
    m = ts.maps.astype(np.float32)
    seed = 13
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        out = ops.new_outputs(tod, "mixed")
        c.tod_sweep(tod, "mixed", torch.from_numpy(m).cuda(), seed, 0, out["ncorr"], out["acc"], out["pix"],
                    out["psi"])
        c.sync()
        got = out["ncorr"].cpu().numpy().astype(np.float64)
        acc = out["acc"].cpu().numpy()
        assert np.array_equal(out["pix"].cpu().numpy(), ts.pix)
    finally:
        c.close()
    s = ot.project_all(ts, m.astype(np.float64), ts.pix, ts.psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, seed, 0)
    err = seg_rel(ts, got, nc)
    print("sweep n_corr max segment rel L2 %.2e" % err)
    assert err < TOL["mixed"]
    b, A, hits = ot.bin_tod(ts, ts.pix, ts.psi, ts.d, got)
    assert np.array_equal(acc[9], hits)
    assert np.abs(acc[0:3] - b).max() <= 1e-12 * np.abs(b).max()


def test_long_gain_noise_mixed():
    """Gain and noise-parameter draws on the long segments.  At these lengths
    the periodogram's high-frequency bins are wider than the 64 modes a wave
    covers, so the per-wave bin sums take their one-atomic path."""
    from paper_2201_03509_amd import ops
    from oracle import gain as og
    from oracle import noise as on
    ts = first_segments(data(), 2)
    t = ot.project(ts.maps, ot.global_pix(ts, ts.pix), ts.psi, 1.0).astype(np.float32)
    s = t.astype(np.float64) * np.repeat(ts.gain, np.diff(ts.seg_off))
    nc = ot.sample_ncorr_all(ts, ts.d, s, 41, 5).astype(np.float32)
    seed, it = 29, 3
    g_ref, _ = og.sample_gain_all(ts, ts.d, t.astype(np.float64), seed, it)
    xi_ref = on.sample_noise_all(ts, ts.d, t.astype(np.float64), ts.gain, nc.astype(np.float64), ts.fknee,
                                 seed, it)
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        g = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.sample_gain(tod, "mixed", tod.d, torch.from_numpy(t).cuda(), seed, it, g)
        xi = [torch.empty(ts.nseg, dtype=torch.float64, device="cuda") for _ in range(3)]
        c.sample_noise(tod, "mixed", tod.d, torch.from_numpy(t).cuda(), torch.from_numpy(nc).cuda(), seed, it,
                       *xi)
        c.sync()
    finally:
        c.close()
    eg = np.abs(g.cpu().numpy() - g_ref) / np.abs(g_ref)
    ex = np.stack([np.abs(x.cpu().numpy() - r) / np.abs(r) for x, r in zip(xi, xi_ref)])
    print("long segments: gain rel err %.2e, noise rel err %.2e" % (eg.max(), ex.max()))
    assert eg.max() < TOL["mixed"] and ex.max() < TOL["mixed"]
