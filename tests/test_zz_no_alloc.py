"""decode_pointing_noalloc: the decode entry point whose scratch (decoding
tables and work list) lives in a static device array instead of context
buffers.  Checked through the C-ABI against decode_pointing, bit for bit, on
two calls in a row, the second with a smaller input, and against the
oracle's decode; a request beyond the static array is refused on the host;
stream corruption is reported the same way."""
import numpy as np
import pytest
import torch

import synth
from oracle import huffman as oh

pytestmark = pytest.mark.gpu


def _decode_both(c, ts):
    from paper_2201_03509_amd import ops
    tod = ops.DeviceTod(ts, "cuda:0")
    p0 = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
    q0 = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
    c.decode_pointing(tod, p0, q0)
    p1 = torch.full((ts.nsamp,), -7, dtype=torch.int32, device="cuda")
    q1 = torch.full((ts.nsamp,), 12345, dtype=torch.int32, device="cuda").to(torch.uint16)
    c.decode_pointing_noalloc(tod, p1, q1)
    c.sync()
    return tod, (p0.cpu().numpy(), q0.cpu().numpy()), (p1.cpu().numpy(), q1.cpu().numpy())


def test_noalloc_matches_decode_pointing():
    from paper_2201_03509_amd import ops
    big = synth.make(1, nscan=3, length=("uniform", 9000, 13000), keep_truth=True)
    small = synth.make(4, nscan=2, length=("loguniform2", 8.0, 12.0), keep_truth=True)
    assert small.nsamp < big.nsamp and small.nseg != big.nseg
    c = ops.Context(0)
    try:
        for ts in (big, small):   # the second call reuses the array with a smaller input
            _, ref, got = _decode_both(c, ts)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            pix, psi = oh.decode_pointing(ts)
            assert np.array_equal(got[0], pix) and np.array_equal(got[1].astype(np.int64), psi)
    finally:
        c.close()


def test_noalloc_limits_and_errors():
    from paper_2201_03509_amd import ops, _lib
    import copy as _copy
    ts = synth.make(0, keep_truth=True)
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        p = torch.empty(ts.nsamp, dtype=torch.int32, device="cuda")
        q = torch.empty(ts.nsamp, dtype=torch.uint16, device="cuda")
        # more table blobs than the static array holds: refused before any launch
        big = _lib.tod_huff()
        for name, _ in _lib.tod_huff._fields_:
            setattr(big, name, getattr(tod.pix_huff, name))
        big.ntable = 100000
        with pytest.raises(ops.C3todError) as ei:
            c.decode_pointing_noalloc(tod, p, q, pix_huff=big)
        assert ei.value.status == _lib.TOD_ENOTSUP
        c.decode_pointing_noalloc(tod, p, q)
        c.sync()
        assert np.array_equal(p.cpu().numpy(), ts.pix)
        # a corrupt psi stream raises the sticky error as decode_pointing does
        bad = _copy.copy(ts)
        bad.psi_huff = _copy.copy(ts.psi_huff)
        w = ts.psi_huff.words.copy()
        a = ts.psi_huff.seg_word_off[2]
        w[a + 40: a + 60] ^= np.uint32(0x5A5A5A5A)
        bad.psi_huff.words = w
        tb = ops.DeviceTod(bad, "cuda:0")
        c.decode_pointing_noalloc(tb, p, q)
        with pytest.raises(ops.CorruptStream):
            c.sync()
        c.clear_error()
        c.sync()
    finally:
        c.close()
