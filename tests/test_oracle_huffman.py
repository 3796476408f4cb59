"""Pins of the reference Huffman decoder (section 4.1, Fig. 3)."""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import huffman as oh
from synth import huffman_enc as enc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "huffman_fig3.txt")


def _fig3_codes():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        sym, code = line.split()
        out.append((int(sym), code))
    return out


def test_paper_fig3_codes_decode():
    """The printed codes, read top-down with 0 = left, decode a hand-made bitstring."""
    codes = _fig3_codes()
    # complete the truncated tree with filler leaves so the code is complete
    fill = [(100, "101"), (101, "1100"), (102, "11011"), (103, "1111"), (104, "1000")]
    allc = [(s, int(c, 2), len(c)) for s, c in codes + fill]
    tree = oh.build_tree(allc)
    assert oh.kraft_sum(np.bincount([L for _, _, L in allc], minlength=33)) == 1.0
    msg = [0, 1, -1, -2, 0, 0, -2, 1]
    lut = dict((s, c) for s, c in codes)
    bits = [int(b) for s in msg for b in lut[s]]
    assert oh.walk_decode_py(tree, bits) == msg
    # 0 -> a single bit 0, +-1 -> 4 bits, -2 -> 5 bits as printed
    assert len(lut[0]) == 1 and lut[0] == "0"
    assert len(lut[1]) == len(lut[-1]) == 4 and len(lut[-2]) == 5


def test_paper_fig3_one_bit_for_dominant_symbol():
    """A symbol holding ~42% of 861276 entries over 670 symbols gets a 1-bit code
    (Fig. 3); any probability above 2/5 forces this in a Huffman code."""
    rng = np.random.default_rng(3)
    n, nsym = 861276, 670
    n0 = int(0.42 * n)
    rest = rng.geometric(0.05, size=n - n0) * rng.choice([-1, 1], size=n - n0)
    vals = np.concatenate([np.zeros(n0, dtype=np.int64), rest])
    blob, (ss, sl, codes) = enc.build_table(vals)
    counts, syms = oh.parse_table(blob)
    cl = oh.canonical_code_list(counts, syms)
    L0 = [L for s, c, L in cl if s == 0][0]
    assert L0 == 1
    assert len(cl) <= nsym + 1000


def test_canonical_rule_textbook():
    """Lengths {A:1, B:2, C:3, D:3} give A=0, B=10, C=110, D=111."""
    counts = np.zeros(33, dtype=np.int64)
    counts[1], counts[2], counts[3] = 1, 1, 2
    cl = oh.canonical_code_list(counts, np.array([65, 66, 67, 68]))
    assert [(s, format(c, "0%db" % L)) for s, c, L in cl] == \
        [(65, "0"), (66, "10"), (67, "110"), (68, "111")]


def _round_trip(vals):
    vals = np.asarray(vals, dtype=np.int64)
    blob, lookup = enc.build_table(vals)
    words, pos = enc.encode_values(vals, lookup)
    counts, syms = oh.parse_table(blob)
    # Kraft equality for a full Huffman code (one symbol: single half-used code)
    k = oh.kraft_sum(counts)
    assert k == (0.5 if len(syms) == 1 else 1.0)
    # compressed size = sum(count * length)
    _, sl, _ = lookup
    uniq, cnt = np.unique(vals, return_counts=True)
    cl = oh.canonical_code_list(counts, syms)
    lens = dict((s, L) for s, c, L in cl)
    assert int(pos[-1]) == sum(int(c) * lens[int(u)] for u, c in zip(uniq, cnt))
    tree = oh.build_tree(cl)
    out, end = oh.walk_decode(tree, words, 0, len(vals))
    assert end == pos[-1]
    assert np.array_equal(out, vals)
    return cl


@settings(max_examples=60, deadline=None)
@given(st.lists(st.integers(-5000, 5000), min_size=1, max_size=2000))
def test_round_trip_random(vals):
    _round_trip(vals)


def test_round_trip_single_symbol():
    cl = _round_trip([7] * 100)
    assert cl == [(7, 0, 1)]


def test_round_trip_32bit_codes():
    """Fibonacci-weighted counts give the deepest possible tree: 32-bit codes."""
    fib = [1, 1]
    while len(fib) < 33:
        fib.append(fib[-1] + fib[-2])
    vals = np.repeat(np.arange(33) - 16, fib)
    np.random.default_rng(0).shuffle(vals)
    cl = _round_trip(vals)
    assert max(L for _, _, L in cl) == 32


def test_side_index_and_corruption(tiny):
    ts = tiny
    dec = oh.StreamDecoder(ts.psi_huff)
    n = int(ts.seg_off[1])
    full = dec.segment(0, n)
    C = ts.psi_huff.chunk_len
    for c in [0, 3, (n - 1) // C]:
        assert np.array_equal(dec.chunk(0, c, n), full[c * C:(c + 1) * C])
    # a truncated stream must be rejected
    hs = ts.psi_huff
    w = hs.words[hs.seg_word_off[0]:hs.seg_word_off[1]]
    with pytest.raises(ValueError):
        oh.walk_decode(dec.tree(0), w[: len(w) // 2], 0, n)


def test_decode_matches_truth(tiny):
    pix, psi = oh.decode_pointing(tiny)
    assert np.array_equal(pix, tiny.pix) and np.array_equal(psi, tiny.psi)
