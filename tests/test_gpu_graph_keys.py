"""A captured sweep is replayed only for the arguments it was captured with:
every device pointer the kernels receive (the layout's arrays, accept flags
included, and every array of both Huffman streams) and the plan's task lists
and binning tiles are part of the graph's key.  Each case changes one of them
between two graph sweeps and checks the replay against an eager sweep and
the oracle's hit counts."""
import numpy as np
import pytest
import torch

import synth
from oracle import tod as ot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    return synth.make(1, nscan=2, length=("uniform", 9000, 13000), keep_truth=True)


def _sweep(c, tod, maps, it, graph, **kw):
    from paper_2201_03509_amd import ops
    o = ops.new_outputs(tod, "mixed")
    c.tod_sweep(tod, "mixed", maps, 5, it, o["ncorr"], o["acc"], o["pix"], o["psi"], use_graph=graph, **kw)
    c.sync()
    return o["ncorr"].cpu().numpy(), o["acc"].cpu().numpy()


def _hits(ts, accept=None):
    h = np.zeros(ts.npix_total)
    for q in range(ts.nseg):
        if accept is not None and not accept[q]:
            continue
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        np.add.at(h, ot.global_pix(ts, ts.pix)[a:b], 1)
    return h


def _same(g, e):
    assert np.array_equal(g[0], e[0])
    assert np.array_equal(g[1][9], e[1][9])
    assert np.allclose(g[1][:9], e[1][:9], rtol=1e-12, atol=1e-9)


def test_accept_flags_null_and_array(data):
    from paper_2201_03509_amd import ops
    ts = data
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        maps = torch.from_numpy(ts.maps.astype(np.float32)).cuda()
        acc = np.ones(ts.nseg, dtype=np.uint8)
        acc[::3] = 0
        tod.seg_accept.copy_(torch.from_numpy(acc))
        for it in range(2):
            g = _sweep(c, tod, maps, it, True)
            _same(g, _sweep(c, tod, maps, it, False))
            assert np.array_equal(g[1][9], _hits(ts, acc))
        tod.layout.seg_accept = None          # NULL: every segment accepted
        for it in range(2):
            g = _sweep(c, tod, maps, it, True)
            _same(g, _sweep(c, tod, maps, it, False))
            assert np.array_equal(g[1][9], _hits(ts))
    finally:
        c.close()


def test_side_index_buffers_swapped(data):
    """Two graph sweeps whose pixel streams share words and tables but not
    the side index: the second must read its own side index (the first
    one's is overwritten after the capture)."""
    from paper_2201_03509_amd import ops
    ts = data
    c = ops.Context(0)
    try:
        a = ops.DeviceTod(ts, "cuda:0")
        b = ops.DeviceTod(ts, "cuda:0")
        maps = torch.from_numpy(ts.maps.astype(np.float32)).cuda()
        ref = _sweep(c, a, maps, 0, False)
        g1 = _sweep(c, a, maps, 0, True)
        _same(g1, ref)
        from paper_2201_03509_amd import _lib
        hyb = _lib.tod_huff()
        for name, _ in _lib.tod_huff._fields_:
            setattr(hyb, name, getattr(a.pix_huff, name))
        for k in ("chunk_bit", "chunk_prev", "seg_chunk_off"):
            setattr(hyb, k, b._pt[k].data_ptr())
        a._pt["chunk_bit"].zero_()           # the first capture's side index is gone
        a._pt["chunk_prev"].zero_()
        g2 = _sweep(c, a, maps, 0, True, pix_huff=hyb)
        c.sync()
        _same(g2, ref)
        assert np.array_equal(g2[1][9], _hits(ts))
    finally:
        c.close()


def test_stride_change_after_capture(data):
    """A binning stride set after a capture rebuilds the tiles, and the next
    graph sweep is captured anew with them."""
    from paper_2201_03509_amd import ops
    ts = data
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        maps = torch.from_numpy(ts.maps.astype(np.float32)).cuda()
        for stride in (0, 3, 1000, 7):
            c.set_bin_stride(0, stride)
            g = _sweep(c, tod, maps, 1, True)
            e = _sweep(c, tod, maps, 1, False)
            _same(g, e)
            assert np.array_equal(g[1][9], _hits(ts)), stride
    finally:
        c.close()
