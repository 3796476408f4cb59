"""GPU path vs the oracle, element by element, through the C-ABI.

Tolerances (spec bar): decode and pixel indices bit-exact; maps and
n_corr within 1e-5 relative (FP32 path) or 1e-12 (FP64 path), measured as
||gpu - oracle||_2 / ||oracle||_2 per segment for per-sample outputs.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import huffman as oh
from oracle import tod as ot

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}


def _ctx():
    from paper_2201_03509_amd import ops
    return ops.Context(0)


@pytest.fixture(scope="module")
def ctx():
    c = _ctx()
    yield c
    c.close()


def _cases():
    # (config, nscan, length, side-index spacing) -- several chunks, ragged
    # tails, several bands, the default and a long side-index spacing
    return {
        "tiny": (0, None, None, None),
        "lfi30_small": (1, 3, ("uniform", 9000, 13000), None),
        "mixed_small": (4, 6, ("loguniform2", 11.0, 14.0), None),
        "lfi30_c256": (1, 2, ("uniform", 9000, 13000), 256),
    }


_CACHE = {}


def dataset(name):
    if name not in _CACHE:
        k, ns, ln, cl = _cases()[name]
        ts = synth.make(k, nscan=ns, length=ln, keep_truth=True, chunk_len=cl)
        pix, psi = oh.decode_pointing(ts)
        assert np.array_equal(pix, ts.pix) and np.array_equal(psi, ts.psi)
        _CACHE[name] = (ts, pix, psi)
    return _CACHE[name]


def dev_tod(ts):
    from paper_2201_03509_amd import ops
    return ops.DeviceTod(ts, "cuda:0")


def maps_for(ts, prec):
    m = ts.maps.astype(np.float32) if prec == "mixed" else ts.maps
    return torch.from_numpy(np.ascontiguousarray(m)).cuda(), m.astype(np.float64)


def seg_rel(ts, got, ref):
    errs = []
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        nr = np.linalg.norm(ref[a:b])
        errs.append(np.linalg.norm(got[a:b] - ref[a:b]) / max(nr, 1e-300))
    return max(errs)


@pytest.mark.parametrize("name", ["tiny", "lfi30_small", "mixed_small", "lfi30_c256"])
def test_decode_bit_exact(ctx, name):
    ts, pix, psi = dataset(name)
    tod = dev_tod(ts)
    p = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    q = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
    ctx.decode_pointing(tod, p, q)
    ctx.sync()
    assert np.array_equal(p.cpu().numpy(), pix)
    assert np.array_equal(q.cpu().numpy().astype(np.int64), psi)


def test_decode_detects_corruption(ctx):
    from paper_2201_03509_amd import ops
    import copy
    ts0, pix, psi = dataset("tiny")
    # flip bits in the middle of segment 2's psi stream
    ts = copy.copy(ts0)
    ts.psi_huff = copy.copy(ts0.psi_huff)
    w = ts0.psi_huff.words.copy()
    a = ts0.psi_huff.seg_word_off[2]
    w[a + 40: a + 60] ^= np.uint32(0x5A5A5A5A)
    ts.psi_huff.words = w
    tod = dev_tod(ts)
    p = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    q = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
    ctx.decode_pointing(tod, p, q)
    with pytest.raises(ops.CorruptStream):
        ctx.sync()
    assert ctx.device_error_bits() != 0
    ctx.clear_error()
    ctx.sync()


def test_invalid_arguments_rejected_on_host(ctx):
    from paper_2201_03509_amd import ops
    ts, _, _ = dataset("tiny")
    tod = dev_tod(ts)
    bad = ts.seg_off.copy()
    tod.h_seg_off[3] = tod.h_seg_off[4] + 5          # non-monotone offsets
    p = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    q = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
    with pytest.raises(ops.InvalidArgument):
        ctx.decode_pointing(tod, p, q)
    tod.h_seg_off[:] = bad


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["tiny", "lfi30_small", "mixed_small"])
def test_project(ctx, name, prec):
    ts, pix, psi = dataset(name)
    tod = dev_tod(ts)
    m_dev, m_ref = maps_for(ts, prec)
    ref = ot.project_all(ts, m_ref, pix, psi)
    ft = torch.float32 if prec == "mixed" else torch.float64
    s = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    ctx.project_sky(tod, prec, torch.from_numpy(pix.astype(np.int32)).cuda(),
                    torch.from_numpy(psi.astype(np.uint16)).cuda(), m_dev, s)
    ctx.sync()
    assert seg_rel(ts, s.cpu().numpy().astype(np.float64), ref) < TOL[prec]


@pytest.mark.parametrize("mean_only", [True, False])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["tiny", "lfi30_small", "mixed_small"])
def test_ncorr(ctx, name, prec, mean_only):
    ts, pix, psi = dataset(name)
    tod = dev_tod(ts)
    ft = torch.float32 if prec == "mixed" else torch.float64
    m_dev, m_ref = maps_for(ts, prec)
    s_ref = ot.project_all(ts, m_ref, pix, psi)
    # both sides take the same s (rounded to the path's precision) and d
    s_in = s_ref.astype(np.float32 if prec == "mixed" else np.float64)
    seed, it = synth.seed32(ts.config), 3
    ref = ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it, mean_only=mean_only)
    out = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    ctx.sample_ncorr(tod, prec, tod.d, torch.from_numpy(s_in).cuda(), seed, it, out,
                     mean_only=mean_only)
    ctx.sync()
    got = out.cpu().numpy().astype(np.float64)
    assert seg_rel(ts, got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["tiny", "lfi30_small", "mixed_small"])
def test_bin_and_solve(ctx, name, prec):
    from paper_2201_03509_amd import ops
    ts, pix, psi = dataset(name)
    tod = dev_tod(ts)
    rng = np.random.default_rng(5)
    nc = (rng.normal(size=ts.nsamp) * 0.3).astype(np.float32 if prec == "mixed" else np.float64)
    b, A, hits = ot.bin_tod(ts, pix, psi, ts.d, nc.astype(np.float64))
    acc = ops.new_acc(ts.npix_total, "cuda")
    ctx.bin_tod(tod, prec, torch.from_numpy(pix.astype(np.int32)).cuda(),
                torch.from_numpy(psi.astype(np.uint16)).cuda(), tod.d,
                torch.from_numpy(nc).cuda(), acc)
    ctx.sync()
    a = acc.cpu().numpy()
    assert np.array_equal(a[9], hits)
    scale_b = np.abs(b).max()
    scale_A = np.abs(A).max()
    assert np.abs(a[0:3] - b).max() <= 1e-12 * scale_b
    assert np.abs(a[3:9] - A).max() <= 1e-12 * scale_A
    # solve
    tau = 1e-3
    m_ref, rc_ref = ot.solve_maps(b, A, hits, tau)
    mdt = torch.float32 if prec == "mixed" else torch.float64
    m_out = torch.empty((3, ts.npix_total), dtype=mdt, device="cuda")
    rc = torch.empty(ts.npix_total, dtype=torch.float64, device="cuda")
    ctx.solve_maps(acc, tau, m_out, rc)
    ctx.sync()
    mg = m_out.cpu().numpy().astype(np.float64)
    ok = ~np.isnan(m_ref[0])
    near = np.abs(rc_ref - tau) < 1e-9
    assert np.array_equal(np.isnan(mg[0]) | near, ~ok | near)
    sel = ok & ~near
    for i in range(3):
        den = np.linalg.norm(m_ref[i, sel])
        assert np.linalg.norm(mg[i, sel] - m_ref[i, sel]) / den < (1e-6 if prec == "mixed" else 1e-12)
    assert np.allclose(rc.cpu().numpy(), rc_ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noiseless_round_trip(ctx, prec):
    """FP64 d = g P m exactly: the GPU bin + solve returns the input map."""
    from paper_2201_03509_amd import ops
    ts, pix, psi = dataset("tiny")
    tod = dev_tod(ts)
    d = ot.project_all(ts, ts.maps, pix, psi)
    acc = ops.new_acc(ts.npix_total, "cuda")
    ctx.bin_tod(tod, prec, torch.from_numpy(pix.astype(np.int32)).cuda(),
                torch.from_numpy(psi.astype(np.uint16)).cuda(), torch.from_numpy(d).cuda(), None,
                acc)
    m_out = torch.empty((3, ts.npix_total), dtype=torch.float64, device="cuda")
    ctx.solve_maps(acc, 1e-3, m_out)
    ctx.sync()
    m = m_out.cpu().numpy()
    ok = ~np.isnan(m[0])
    assert ok.sum() > 50
    assert np.abs(m[:, ok] - ts.maps[:, ok]).max() <= 1e-12 * np.abs(ts.maps).max()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["tiny", "lfi30_small"])
def test_sweep_matches_steps(ctx, name, prec):
    from paper_2201_03509_amd import ops
    ts, pix, psi = dataset(name)
    tod = dev_tod(ts)
    m_dev, m_ref = maps_for(ts, prec)
    seed, it = synth.seed32(ts.config), 0
    out = ops.new_outputs(tod, prec)
    ctx.tod_sweep(tod, prec, m_dev, seed, it, out["ncorr"], out["acc"], out["pix"], out["psi"])
    ctx.sync()
    assert np.array_equal(out["pix"].cpu().numpy(), pix)
    s = ot.project_all(ts, m_ref, pix, psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, seed, it)
    got = out["ncorr"].cpu().numpy().astype(np.float64)
    assert seg_rel(ts, got, nc) < TOL[prec]
    b, A, hits = ot.bin_tod(ts, pix, psi, ts.d, got)
    a = out["acc"].cpu().numpy()
    assert np.array_equal(a[9], hits)
    assert np.abs(a[0:3] - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(a[3:9] - A).max() <= 1e-12 * np.abs(A).max()


def test_sweep_graph_replays(ctx):
    """Captured sweep: replays with new iteration numbers equal eager sweeps."""
    from paper_2201_03509_amd import ops
    ts, pix, psi = dataset("lfi30_small")
    tod = dev_tod(ts)
    m_dev, _ = maps_for(ts, "mixed")
    seed = synth.seed32(1)
    eager = ops.new_outputs(tod, "mixed")
    graph = ops.new_outputs(tod, "mixed")
    for it in range(4):
        ctx.tod_sweep(tod, "mixed", m_dev, seed, it, eager["ncorr"], eager["acc"], eager["pix"],
                      eager["psi"], use_graph=False)
        ctx.sync()
        e_nc = eager["ncorr"].cpu().numpy().copy()
        e_acc = eager["acc"].cpu().numpy().copy()
        ctx.tod_sweep(tod, "mixed", m_dev, seed, it, graph["ncorr"], graph["acc"], graph["pix"],
                      graph["psi"], use_graph=True)
        ctx.sync()
        assert np.array_equal(graph["ncorr"].cpu().numpy(), e_nc)
        ga = graph["acc"].cpu().numpy()
        assert np.array_equal(ga[9], e_acc[9])
        assert np.allclose(ga[:9], e_acc[:9], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("runs", [2, 3, 16])
@pytest.mark.parametrize("stride", [None, 3, 1000])
@pytest.mark.parametrize("name", ["lfi30_small", "mixed_small"])
def test_bin_runs_across_scans(name, stride, runs):
    """Binning runs that walk one detector pair's consecutive scans at equal
    spin phase (tod_set_bin_runs), at forced run lengths and strides: every
    sample is binned once (hits exact), b and A match the oracle."""
    from paper_2201_03509_amd import ops
    ts, pix, psi = dataset(name)
    rng = np.random.default_rng(9)
    nc = (rng.normal(size=ts.nsamp) * 0.3).astype(np.float32)
    b, A, hits = ot.bin_tod(ts, pix, psi, ts.d, nc.astype(np.float64))
    c = ops.Context(0)
    try:
        c.set_bin_runs(runs)
        if stride:
            for band in range(ts.nband):
                c.set_bin_stride(band, stride)
        tod = dev_tod(ts)
        acc = ops.new_acc(ts.npix_total, "cuda")
        c.bin_tod(tod, "mixed", torch.from_numpy(pix.astype(np.int32)).cuda(),
                  torch.from_numpy(psi.astype(np.uint16)).cuda(), tod.d, torch.from_numpy(nc).cuda(), acc)
        c.sync()
        a = acc.cpu().numpy()
    finally:
        c.close()
    assert np.array_equal(a[9], hits)
    assert np.abs(a[0:3] - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(a[3:9] - A).max() <= 1e-12 * np.abs(A).max()
