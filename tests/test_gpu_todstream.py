"""Compressed TOD and flag streams on the GPU vs the oracle's decoder, through
the C-ABI.  Bar: bit-exact (integer decode; the TOD is quantum x integer, exact
in FP32 and FP64).  Also: a corrupted stream is reported, and the decoded
flag mask drives the masked n_corr draw exactly like the host-built mask.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import huffman as oh
from oracle import tod as ot

pytestmark = pytest.mark.gpu

_CASES = {
    "tiny": (0, None, None, None),
    "lfi30_small": (1, 3, ("uniform", 9000, 13000), None),
    "mixed_small": (4, 6, ("loguniform2", 11.0, 14.0), None),
    "lfi30_c256": (1, 2, ("uniform", 9000, 13000), 256),
}
_CACHE = {}


def dataset(name):
    if name not in _CACHE:
        k, ns, ln, cl = _CASES[name]
        _CACHE[name] = synth.make(k, nscan=ns, length=ln, keep_truth=True, chunk_len=cl, tod_streams=True)
    return _CACHE[name]


@pytest.fixture(scope="module")
def ctx():
    from paper_2201_03509_amd import ops
    c = ops.Context(0)
    yield c
    c.close()


def _tod(ts):
    from paper_2201_03509_amd import ops
    return ops.DeviceTod(ts, "cuda:0")


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(_CASES))
def test_decode_tod_bit_exact(ctx, name, prec):
    ts = dataset(name)
    tod = _tod(ts)
    ft = torch.float32 if prec == "mixed" else torch.float64
    d = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    ctx.decode_tod(tod, prec, d)
    ctx.sync()
    ref = oh.decode_tod(ts)
    got = d.cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, ts.d.astype(np.float64))


@pytest.mark.parametrize("name", list(_CASES))
def test_decode_flags_bit_exact(ctx, name):
    ts = dataset(name)
    tod = _tod(ts)
    f = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    m = torch.empty(ts.nsamp, dtype=torch.uint8, device="cuda")
    ctx.decode_flags(tod, synth.FLAG_PLANE | synth.FLAG_GLITCH, f, m)
    ctx.sync()
    ref = oh.decode_stream(ts, ts.flag_huff)
    assert np.array_equal(f.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(m.cpu().numpy(), (ref == 0).astype(np.uint8))


def test_corrupt_tod_stream_reported(ctx):
    """Flipped bits inside segment 2's TOD stream break the side index's
    chunk consistency."""
    import copy
    from paper_2201_03509_amd import ops
    ts0 = dataset("lfi30_small")
    ts = copy.copy(ts0)
    ts.tod_huff = copy.copy(ts0.tod_huff)
    w = ts0.tod_huff.words.copy()
    a = ts0.tod_huff.seg_word_off[2]
    w[a + 40: a + 60] ^= np.uint32(0x5A5A5A5A)
    ts.tod_huff.words = w
    tod = _tod(ts)
    d = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
    ctx.decode_tod(tod, "mixed", d)
    with pytest.raises(ops.CorruptStream):
        ctx.sync()
    assert ctx.device_error_bits() != 0
    ctx.clear_error()
    ctx.sync()


def test_flag_mask_drives_the_masked_draw(ctx):
    """Processing-mask bit only: the decoded mask equals the host plane mask,
    so the masked draws agree sample for sample."""
    from oracle import tod as ot
    ts = dataset("tiny")
    tod = _tod(ts)
    m_dev = torch.empty(ts.nsamp, dtype=torch.uint8, device="cuda")
    ctx.decode_flags(tod, synth.FLAG_PLANE, None, m_dev)
    ctx.sync()
    m_host = synth.plane_mask(ts, ts.pix)
    assert np.array_equal(m_dev.cpu().numpy(), m_host)
    s = torch.from_numpy(ot.project_all(ts, ts.maps, ts.pix, ts.psi)).cuda()
    outs = []
    for m in (m_dev, torch.from_numpy(m_host).cuda()):
        o = torch.empty(ts.nsamp, dtype=torch.float64, device="cuda")
        ctx.sample_ncorr_masked(tod, "fp64", tod.d, s, m, 5, 1, o, tol=1e-12)
        ctx.sync()
        outs.append(o.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_sweep_from_compressed_tod(prec):
    """tod_sweep_stream decodes the TOD inside the sweep: its d is the FP32 TOD
    bit for bit, and n_corr, hits and the binned sums equal those of the
    sweep that reads d (eager and graph-replayed), and the oracle's."""
    from paper_2201_03509_amd import ops
    ts = synth.make(1, nscan=2, length=("uniform", 9000, 13000), keep_truth=True, tod_streams=True)
    m = ts.maps.astype(np.float32 if prec == "mixed" else np.float64)
    seed = 21
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        maps = torch.from_numpy(m).cuda()
        a = ops.new_outputs(tod, prec)
        c.tod_sweep(tod, prec, maps, seed, 3, a["ncorr"], a["acc"], a["pix"], a["psi"])
        ft = torch.float32 if prec == "mixed" else torch.float64
        res = []
        for graph in (False, True, True):
            b = ops.new_outputs(tod, prec)
            dw = torch.empty(ts.nsamp, dtype=ft, device="cuda")
            c.tod_sweep_stream(tod, prec, maps, seed, 3, b["ncorr"], b["acc"], b["pix"], b["psi"], dw,
                               use_graph=graph)
            c.sync()
            res.append((b, dw))
        ea = a["acc"].cpu().numpy()
        for b, dw in res:
            assert np.array_equal(dw.cpu().numpy().astype(np.float64), ts.d.astype(np.float64))
            assert np.array_equal(b["ncorr"].cpu().numpy(), a["ncorr"].cpu().numpy())
            ba = b["acc"].cpu().numpy()
            assert np.array_equal(ba[9], ea[9])
            assert np.abs(ba[:9] - ea[:9]).max() <= 1e-12 * np.abs(ea[:9]).max()
        got = a["ncorr"].cpu().numpy().astype(np.float64)
    finally:
        c.close()
    s = ot.project_all(ts, m.astype(np.float64), ts.pix, ts.psi)
    ref = ot.sample_ncorr_all(ts, ts.d, s, seed, 3)
    tol = 1e-5 if prec == "mixed" else 1e-12
    for q in range(ts.nseg):
        lo, hi = ts.seg_off[q], ts.seg_off[q + 1]
        assert np.linalg.norm(got[lo:hi] - ref[lo:hi]) / np.linalg.norm(ref[lo:hi]) < tol


def test_decoder_block_boundaries(ctx):
    """Segments whose chunk counts straddle the decoders' 512-chunk blocks
    (511, 512 and 513 chunks of 32 symbols, the last of one symbol; 1025
    chunks), at odd and even sample offsets: the pointing (with and without
    allocation), TOD and flag streams bit-exact."""
    ts = synth.make(1, nscan=4, length=("list", 16352, 16384, 16385, 32800), keep_truth=True,
                    tod_streams=True)
    tod = _tod(ts)
    pix = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    psi = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
    ctx.decode_pointing(tod, pix, psi)
    ctx.sync()
    assert np.array_equal(pix.cpu().numpy(), ts.pix)
    assert np.array_equal(psi.cpu().numpy().astype(np.int64), ts.psi)
    pix.fill_(-1)
    psi.fill_(0)
    ctx.decode_pointing_noalloc(tod, pix, psi)
    ctx.sync()
    assert np.array_equal(pix.cpu().numpy(), ts.pix)
    assert np.array_equal(psi.cpu().numpy().astype(np.int64), ts.psi)
    d = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
    ctx.decode_tod(tod, "mixed", d)
    f = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    m = torch.empty(ts.nsamp, dtype=torch.uint8, device="cuda")
    ctx.decode_flags(tod, synth.FLAG_PLANE | synth.FLAG_GLITCH, f, m)
    ctx.sync()
    assert np.array_equal(d.cpu().numpy(), ts.d.astype(np.float32))
    ref = oh.decode_stream(ts, ts.flag_huff)
    assert np.array_equal(f.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(m.cpu().numpy(), (ref == 0).astype(np.uint8))
