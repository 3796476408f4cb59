"""Every entry point on the degenerate-length set against the oracle.

The set (see test_oracle_edge): scans of 0, 1, 2, 3, 17, 130, 4097 and 0
samples, two radiometers each.  So it has empty segments and one-, two- and
three-sample segments, whose transforms have N = 2, 4, 6 (one complex column,
no radix stage).  It also has segments shorter than a side-index chunk,
segments shorter than the revisit period, and ragged tails.  The strided
kernels are also run with revisit periods of 1, 3 and one longer than every
segment.  The masked draw gets a seeded random mask, with one three-sample
segment masked whole and one one-sample segment masked.

Bars as in the parity suites: bit-exact decodes; 1e-5 (FP32 path) and 1e-12
(FP64) relative per segment; the gain's bar is scaled by how far the
template's information A falls below t.t / sigma0^2 (a near-constant
three-sample template loses almost everything to the free DC mode, and FP32
rounding grows by the same ratio).  Where the method has no answer (an empty
segment's gain and noise parameters, a one-sample segment's gain, alpha and
f_knee) both sides return NaN at the same places.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import gain as og
from oracle import gapfill as gf
from oracle import huffman as oh
from oracle import noise as on
from oracle import tod as ot
from test_oracle_edge import make_edge

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}
_DATA = {}


def data():
    if not _DATA:
        ts = make_edge()
        _DATA["ts"] = ts
    return _DATA["ts"]


def _ctx(stride=None):
    from paper_2201_03509_amd import ops
    c = ops.Context(0)
    if stride is not None:
        c.set_bin_stride(0, stride)
    return c


def _ft(prec):
    return (np.float32, torch.float32) if prec == "mixed" else (np.float64, torch.float64)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _pointing(ts):
    return _dev(ts.pix.astype(np.int32)), _dev(ts.psi.astype(np.uint16))


def seg_rel(ts, got, ref):
    errs = [0.0]
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        if b > a:
            nr = np.linalg.norm(ref[a:b])
            errs.append(np.linalg.norm(got[a:b] - ref[a:b]) / max(nr, 1e-300))
    return max(errs)


def same_nan_and_close(got, ref, tol):
    """NaN at the same places, elsewhere within tol (a scalar or per element) relative."""
    assert np.array_equal(np.isnan(got), np.isnan(ref)), (got, ref)
    ok = ~np.isnan(ref)
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), ref.shape)[ok]
    assert np.all(np.abs(got[ok] - ref[ok]) <= tol * np.abs(ref[ok])), (got, ref)


def test_edge_decodes():
    from paper_2201_03509_amd import ops
    ts = data()
    c = _ctx()
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        pix = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
        psi = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
        c.decode_pointing(tod, pix, psi)
        d32 = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        d64 = torch.empty(ts.nsamp, dtype=torch.float64, device="cuda")
        c.decode_tod(tod, "mixed", d32)
        c.decode_tod(tod, "fp64", d64)
        flags = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
        mask = torch.empty(ts.nsamp, dtype=torch.uint8, device="cuda")
        c.decode_flags(tod, synth.FLAG_PLANE, flags, mask)
        c.sync()
    finally:
        c.close()
    assert np.array_equal(pix.cpu().numpy(), ts.pix) and np.array_equal(psi.cpu().numpy(), ts.psi)
    ref = oh.decode_tod(ts)
    assert np.array_equal(d64.cpu().numpy(), ref)
    assert np.array_equal(d32.cpu().numpy(), ref.astype(np.float32))
    fl = oh.decode_stream(ts, ts.flag_huff)
    assert np.array_equal(flags.cpu().numpy().astype(np.int64), fl)
    assert np.array_equal(mask.cpu().numpy(), ((fl & synth.FLAG_PLANE) == 0).astype(np.uint8))


@pytest.mark.parametrize("stride", [None, 1, 3, 5000])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_edge_project_bin_chisq(prec, stride):
    """project_sky, bin_tod and tod_chisq (+ adjoint): every
    strided kernel, at the probed revisit period and at forced ones."""
    ts = data()
    nf, tf = _ft(prec)
    m = ts.maps.astype(nf)
    m_ref = m.astype(np.float64)
    rng = np.random.default_rng(12)
    nc = (0.3 * rng.normal(size=ts.nsamp)).astype(nf)
    pix, psi = _pointing(ts)
    c = _ctx(stride)
    try:
        from paper_2201_03509_amd import ops
        tod = ops.DeviceTod(ts, "cuda:0")
        s = torch.empty(ts.nsamp, dtype=tf, device="cuda")
        c.project_sky(tod, prec, pix, psi, _dev(m), s)
        acc = ops.new_acc(ts.npix_total, "cuda")
        c.bin_tod(tod, prec, pix, psi, tod.d, _dev(nc), acc)
        J = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.tod_chisq(tod, prec, pix, psi, tod.d, _dev(nc), _dev(m), J)
        gm = torch.empty((3, ts.npix_total), dtype=torch.float64, device="cuda")
        gg = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.tod_chisq_backward(tod, prec, pix, psi, tod.d, _dev(nc), _dev(m), 1.0, gm, gg)
        c.sync()
    finally:
        c.close()
    s_ref = ot.project_all(ts, m_ref, ts.pix, ts.psi)
    assert seg_rel(ts, s.cpu().numpy().astype(np.float64), s_ref) < TOL[prec]
    b, A, hits = ot.bin_tod(ts, ts.pix, ts.psi, ts.d, nc.astype(np.float64))
    a = acc.cpu().numpy()
    assert np.array_equal(a[9], hits)
    assert np.abs(a[0:3] - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(a[3:9] - A).max() <= 1e-12 * np.abs(A).max()
    J_ref = ot.chisq_all(ts, m_ref, ts.pix, ts.psi, ts.d, nc.astype(np.float64))
    Jg = J.cpu().numpy()
    gm_ref, gg_ref, _, _, _ = ot.chisq_grad_all(ts, m_ref, ts.pix, ts.psi, ts.d, nc.astype(np.float64))
    ggg = gg.cpu().numpy()
    # J and dJ/dg sum terms of both signs: their errors are scaled by the
    # size of the terms; empty segments give exactly 0
    gp = ot.global_pix(ts, ts.pix)
    for q in range(ts.nseg):
        a0, b0 = ts.seg_off[q], ts.seg_off[q + 1]
        if b0 == a0:
            assert Jg[q] == 0.0 and ggg[q] == 0.0
            continue
        t = ot.project(m_ref, gp[a0:b0], ts.psi[a0:b0], 1.0)
        r = ts.d[a0:b0] - ts.gain[q] * t - nc[a0:b0]
        I, P, _ = ot.whittle_parts(nc[a0:b0].astype(np.float64), 32.5, ts.sigma0[q], ts.fknee[q], ts.alpha[q])
        J_terms = np.sum(r * r) / ts.sigma0[q] ** 2 + np.sum(I / P) + np.sum(np.abs(np.log(P)))
        assert abs(Jg[q] - J_ref[q]) <= TOL[prec] * J_terms, (q, Jg[q], J_ref[q])
        scale = 2.0 * np.sum(np.abs(t * r)) / ts.sigma0[q] ** 2
        assert abs(ggg[q] - gg_ref[q]) <= TOL[prec] * scale, (q, ggg[q], gg_ref[q])
    g = gm.cpu().numpy()
    assert np.abs(g - gm_ref).max() <= TOL[prec] * np.abs(gm_ref).max()


@pytest.mark.parametrize("mean_only", [True, False])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_edge_ncorr(prec, mean_only):
    ts = data()
    nf, tf = _ft(prec)
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi).astype(nf)
    seed, it = 77, 4
    ref = ot.sample_ncorr_all(ts, ts.d, s.astype(np.float64), seed, it, mean_only=mean_only)
    c = _ctx()
    try:
        from paper_2201_03509_amd import ops
        tod = ops.DeviceTod(ts, "cuda:0")
        out = torch.empty(ts.nsamp, dtype=tf, device="cuda")
        c.sample_ncorr(tod, prec, tod.d, _dev(s), seed, it, out, mean_only=mean_only)
        c.sync()
    finally:
        c.close()
    assert seg_rel(ts, out.cpu().numpy().astype(np.float64), ref) < TOL[prec]


@pytest.mark.parametrize("mean_only", [True, False])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_edge_gain_noise(prec, mean_only):
    ts = data()
    nf, tf = _ft(prec)
    t = ot.project(ts.maps, ot.global_pix(ts, ts.pix), ts.psi, 1.0).astype(nf)
    s = t.astype(np.float64) * np.repeat(ts.gain, np.diff(ts.seg_off))
    nc = ot.sample_ncorr_all(ts, ts.d, s, 77, 3).astype(nf)
    seed, it = 55, 6
    g_ref, sg_ref = og.sample_gain_all(ts, ts.d, t.astype(np.float64), seed, it, mean_only=mean_only)
    with np.errstate(invalid="ignore"):
        xi_ref = on.sample_noise_all(ts, ts.d, t.astype(np.float64), ts.gain, nc.astype(np.float64), ts.fknee,
                                     seed, it, mean_only=mean_only)
    c = _ctx()
    try:
        from paper_2201_03509_amd import ops
        tod = ops.DeviceTod(ts, "cuda:0")
        g = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        sg = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.sample_gain(tod, prec, tod.d, _dev(t), seed, it, g, sg, mean_only=mean_only)
        xi = [torch.empty(ts.nseg, dtype=torch.float64, device="cuda") for _ in range(3)]
        c.sample_noise(tod, prec, tod.d, _dev(t), _dev(nc), seed, it, *xi, mean_only=mean_only)
        c.sync()
    finally:
        c.close()
    # A = t.Kt loses what the template has outside DC: a near-constant short
    # template (three samples in one pixel) leaves A far below t.t / sigma0^2,
    # and the FP32 transforms' rounding grows by that ratio kappa
    kappa = np.ones(ts.nseg)
    for q in range(ts.nseg):
        a0, b0 = ts.seg_off[q], ts.seg_off[q + 1]
        if b0 > a0 and np.isfinite(sg_ref[q]):
            tq = t[a0:b0].astype(np.float64)
            kappa[q] = max(1.0, (tq @ tq) / ts.sigma0[q] ** 2 * sg_ref[q] ** 2)
    gg_, sgg = g.cpu().numpy(), sg.cpu().numpy()
    print("gain rel err / kappa:", np.abs(gg_ - g_ref) / np.abs(g_ref) / kappa)
    same_nan_and_close(gg_, g_ref, TOL[prec] * kappa)
    fin = np.isfinite(sg_ref)
    assert np.array_equal(np.isfinite(sgg), fin)
    assert np.all(np.abs(sgg[fin] - sg_ref[fin]) <= TOL[prec] * kappa[fin] * sg_ref[fin])
    for i in range(3):
        got = xi[i].cpu().numpy()
        print("noise param", i, "rel err", np.abs(got - xi_ref[i]) / np.abs(xi_ref[i]))
        same_nan_and_close(got, xi_ref[i], TOL[prec])


@pytest.mark.parametrize("mean_only", [True, False])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_edge_masked(prec, mean_only):
    ts = data()
    nf, tf = _ft(prec)
    rng = np.random.default_rng(31)
    mask = (rng.random(ts.nsamp) > 0.3).astype(np.uint8)
    for q in (6, 7):  # the three-sample segments, masked whole
        mask[ts.seg_off[q]:ts.seg_off[q + 1]] = 0
    mask[ts.seg_off[2]], mask[ts.seg_off[3]] = 0, 1  # one-sample segments: masked, kept
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi).astype(nf)
    seed, it = 5, 2
    # the plain definition: the full extended system by preconditioned CG
    ref, _ = gf.cg_ncorr_all(ts, ts.d, s.astype(np.float64), mask, seed, it, mean_only=mean_only, tol=1e-14)
    c = _ctx()
    try:
        from paper_2201_03509_amd import ops
        tod = ops.DeviceTod(ts, "cuda:0")
        out = torch.empty(ts.nsamp, dtype=tf, device="cuda")
        iters = torch.empty(ts.nseg, dtype=torch.int32, device="cuda")
        c.sample_ncorr_masked(tod, prec, tod.d, _dev(s), _dev(mask), seed, it, out, mean_only=mean_only,
                              tol=1e-6 if prec == "mixed" else 1e-15, iters=iters)
        c.sync()
    finally:
        c.close()
    got = out.cpu().numpy().astype(np.float64)
    assert seg_rel(ts, got, ref) < TOL[prec]
    # segments short enough for the dense system: numpy.linalg.solve (a
    # segment masked whole leaves its DC mode free, A singular: no unique x)
    for q in range(ts.nseg):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if not 0 < b - a <= 64 or not mask[a:b].any():
            continue
        band = int(ts.seg_band[q])
        A, rhs = gf.dense_system(ts.d[a:b] - s[a:b].astype(np.float64), mask[a:b], float(ts.band_fsamp[band]),
                                 float(ts.sigma0[q]), float(ts.fknee[q]), float(ts.alpha[q]), seed, q, it,
                                 mean_only)
        x = np.linalg.solve(A, rhs)[:b - a]
        assert np.linalg.norm(got[a:b] - x) <= TOL[prec] * max(np.linalg.norm(x), 1e-300), q


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_edge_sweep(prec):
    """The fused sweep (eager and as a replayed graph) on the edge set."""
    from paper_2201_03509_amd import ops
    ts = data()
    nf, _ = _ft(prec)
    m = ts.maps.astype(nf)
    seed = 9
    c = _ctx()
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        out = ops.new_outputs(tod, prec)
        outg = ops.new_outputs(tod, prec)
        for it in range(2):
            c.tod_sweep(tod, prec, _dev(m), seed, it, out["ncorr"], out["acc"], out["pix"], out["psi"])
            c.tod_sweep(tod, prec, _dev(m), seed, it, outg["ncorr"], outg["acc"], outg["pix"], outg["psi"],
                        use_graph=True)
            c.sync()
            assert np.array_equal(outg["ncorr"].cpu().numpy(), out["ncorr"].cpu().numpy())
        c.sync()
    finally:
        c.close()
    assert np.array_equal(out["pix"].cpu().numpy(), ts.pix)
    s = ot.project_all(ts, m.astype(np.float64), ts.pix, ts.psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, seed, 1)
    got = out["ncorr"].cpu().numpy().astype(np.float64)
    assert seg_rel(ts, got, nc) < TOL[prec]
    b, A, hits = ot.bin_tod(ts, ts.pix, ts.psi, ts.d, got)
    a = out["acc"].cpu().numpy()
    assert np.array_equal(a[9], hits)
    assert np.abs(a[0:3] - b).max() <= 1e-12 * np.abs(b).max()
