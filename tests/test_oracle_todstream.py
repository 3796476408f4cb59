"""Pins of the compressed TOD and flag streams (section 4.1, Table 1).

The oracle's decoder (a bit-by-bit tree walk, independent of the generator's
encoder) returns the generator's quantised TOD exactly and its flag words;
the processing-mask flag bit is the pixel-level plane mask; the compression
ratios behave as Table 1 reports (flags compress about 32x against 32-bit
words: nearly all differences are zero, coded in one bit).
"""
import numpy as np

import synth
from oracle import huffman as oh


def _set():
    return synth.make(1, nscan=3, length=("uniform", 9000, 13000), keep_truth=True, tod_streams=True)


def test_tod_round_trip_exact():
    ts = _set()
    d = oh.decode_tod(ts)
    assert np.array_equal(d, ts.d.astype(np.float64))
    x = ts.d.astype(np.float64) / ts.tod_quantum
    assert np.array_equal(x, np.rint(x))          # integer multiples of the quantum


def test_flags_round_trip_and_plane_bit():
    ts = _set()
    f = oh.decode_stream(ts, ts.flag_huff)
    plane = 1 - synth.plane_mask(ts, ts.pix).astype(np.int64)
    assert np.array_equal(f & synth.FLAG_PLANE, plane)
    g = (f & synth.FLAG_GLITCH) != 0
    assert 0 < g.sum() < 1e-3 * ts.nsamp
    assert (f & ~3).max() == 0


def test_compression_ratios():
    ts = _set()
    tod_bits = 8.0 * ts.tod_huff.words.nbytes / ts.nsamp
    flag_bits = 8.0 * ts.flag_huff.words.nbytes / ts.nsamp
    assert 32.0 / flag_bits > 25.0
    assert 1.0 <= flag_bits < 1.3
    assert 32.0 / tod_bits > 2.0
