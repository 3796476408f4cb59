"""Reference decoding of the Huffman-coded, sample-differenced pointing streams.

Test infrastructure only.  Follows section 4.1 of the paper: each pointing
stream (HEALPix pixel, quantised polarisation angle) was differenced sample by
sample, d(i) - d(i-1), and the differences Huffman coded; decoding reads the
code tree from the top (0 = left branch, 1 = right branch, Fig. 3) and then
undoes the differencing with a running sum.

Readings where the paper is silent: d(-1) = 0 at the start of every segment;
one canonical code table per scan and stream kind; codes MSB-first in uint32
words; a side index every ``chunk_len`` symbols gives the chunk's first bit and
the value before it (pure side information: the bitstream is unchanged).

The canonical table (counts per length + symbols in code order) is turned into
explicit codes here by the textbook rule -- the first code of length L is
(first code of length L-1 + number of codes of length L-1) << 1, and codes of
one length are consecutive -- then into a binary tree that is walked bit by bit.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_huffman_walk.so")
_lib = None


def build_c(force=False):
    """Compile the plain-C tree walker (gcc)."""
    src = os.path.join(_HERE, "huffman_walk.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build_c()
        lib = ctypes.CDLL(_SO)
        lib.walk_decode.restype = ctypes.c_int64
        lib.walk_decode.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] * 3 + [ctypes.c_void_p]
        _lib = lib
    return _lib


def parse_table(blob):
    """(counts[0..32], symbols in code order) from a table blob."""
    blob = np.asarray(blob, dtype=np.uint32)
    nsym = int(blob[0])
    counts = np.zeros(33, dtype=np.int64)
    counts[1:33] = blob[2:34]
    syms = blob[34:34 + nsym].view(np.int32).astype(np.int64)
    if counts.sum() != nsym:
        raise ValueError("table counts do not add up to nsym")
    return counts, syms


def canonical_code_list(counts, syms):
    """[(symbol, code, length)] by the canonical rule."""
    out = []
    code = 0
    i = 0
    for L in range(1, 33):
        for _ in range(int(counts[L])):
            out.append((int(syms[i]), code, L))
            code += 1
            i += 1
        code <<= 1
    return out


def kraft_sum(counts):
    return sum(int(counts[L]) * 2.0 ** -L for L in range(1, 33))


def build_tree(code_list):
    """Binary tree from (symbol, code, length); returns (left, right, leaf, symbols)."""
    left, right, leaf = [-1], [-1], [-1]
    symbols = []
    for si, (sym, code, L) in enumerate(code_list):
        node = 0
        for b in range(L - 1, -1, -1):
            if leaf[node] >= 0:
                raise ValueError("code list is not prefix-free")
            bit = (code >> b) & 1
            nxt = right[node] if bit else left[node]
            if nxt < 0:
                left.append(-1)
                right.append(-1)
                leaf.append(-1)
                nxt = len(leaf) - 1
                if bit:
                    right[node] = nxt
                else:
                    left[node] = nxt
            node = nxt
        if left[node] >= 0 or right[node] >= 0 or leaf[node] >= 0:
            raise ValueError("code list is not prefix-free")
        leaf[node] = si
        symbols.append(sym)
    return (np.array(left, np.int32), np.array(right, np.int32),
            np.array(leaf, np.int32), np.array(symbols, np.int64))


def walk_decode_py(tree, bits):
    """Pure-Python walk over a sequence of 0/1 bits (tiny inputs only)."""
    left, right, leaf, symbols = tree
    out, node = [], 0
    for b in bits:
        node = right[node] if b else left[node]
        if node < 0:
            raise ValueError("invalid code path")
        if leaf[node] >= 0:
            out.append(int(symbols[leaf[node]]))
            node = 0
    if node != 0:
        raise ValueError("bitstring ends inside a code")
    return out


def walk_decode(tree, words, start_bit, nsym):
    """Decode ``nsym`` codes from uint32 ``words`` starting at ``start_bit``.

    Returns (symbol values int64, bit position after the last code)."""
    left, right, leaf, symbols = tree
    words = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.empty(int(nsym), dtype=np.int32)
    lib = _load()
    end = lib.walk_decode(left.ctypes.data, right.ctypes.data, leaf.ctypes.data,
                          words.ctypes.data, len(words), int(start_bit), int(nsym),
                          out.ctypes.data)
    if end < 0:
        raise ValueError("corrupt stream: invalid code or read past the end")
    return symbols[out], int(end)


class StreamDecoder:
    """Decoder for one concatenated stream kind (pix or psi) of a TOD set."""

    def __init__(self, hs):
        self.hs = hs
        self._trees = {}

    def tree(self, t):
        if t not in self._trees:
            hs = self.hs
            blob = hs.tables[hs.table_off[t]:hs.table_off[t + 1]]
            counts, syms = parse_table(blob)
            self._trees[t] = build_tree(canonical_code_list(counts, syms))
        return self._trees[t]

    def segment(self, seg, n):
        """All n undifferenced values of one segment, with stream checks."""
        hs = self.hs
        w = hs.words[hs.seg_word_off[seg]:hs.seg_word_off[seg + 1]]
        diffs, end = walk_decode(self.tree(int(hs.seg_table[seg])), w, 0, n)
        x = np.cumsum(diffs)                       # d(-1) = 0
        # the remainder of the last word must be zero padding
        if end > 32 * len(w) or (32 * len(w) - end) >= 32:
            raise ValueError("stream length mismatch")
        if end % 32:
            if int(w[-1]) & ((1 << (32 - end % 32)) - 1):
                raise ValueError("non-zero padding")
        # side index consistency
        c0, c1 = hs.seg_chunk_off[seg], hs.seg_chunk_off[seg + 1]
        C = hs.chunk_len
        if c1 - c0 != (n + C - 1) // C:
            raise ValueError("chunk count mismatch")
        return x

    def chunk(self, seg, c, n):
        """Values of chunk c (0-based within the segment) from the side index."""
        hs = self.hs
        C = hs.chunk_len
        cg = hs.seg_chunk_off[seg] + c
        m = min(C, n - c * C)
        w = hs.words[hs.seg_word_off[seg]:hs.seg_word_off[seg + 1]]
        diffs, _ = walk_decode(self.tree(int(hs.seg_table[seg])), w, int(hs.chunk_bit[cg]), m)
        return int(hs.chunk_prev[cg]) + np.cumsum(diffs)


def decode_pointing(ts, segs=None):
    """Reference (pix, psi) for all samples (or for the listed segments only).

    Returns int64 arrays laid out like the flat sample arrays when ``segs`` is
    None, else a dict seg -> (pix, psi)."""
    dp, ds = StreamDecoder(ts.pix_huff), StreamDecoder(ts.psi_huff)
    if segs is None:
        pix = np.empty(ts.nsamp, dtype=np.int64)
        psi = np.empty(ts.nsamp, dtype=np.int64)
        for s in range(ts.nseg):
            a, b = ts.seg_off[s], ts.seg_off[s + 1]
            pix[a:b] = dp.segment(s, b - a)
            psi[a:b] = ds.segment(s, b - a)
        return pix, psi
    out = {}
    for s in segs:
        n = int(ts.seg_off[s + 1] - ts.seg_off[s])
        out[s] = (dp.segment(s, n), ds.segment(s, n))
    return out


def decode_stream(ts, hs, segs=None):
    """Undifferenced integers of any stream of the set (TOD, flags), flat."""
    dec = StreamDecoder(hs)
    out = np.zeros(ts.nsamp, dtype=np.int64)
    for q in (range(ts.nseg) if segs is None else segs):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b > a:
            out[a:b] = dec.segment(q, b - a)
    return out


def decode_tod(ts, segs=None):
    """The TOD of the set from its compressed stream: quantum x the integers
    (the paper's TOD are ADC integers, differenced and coded like the pointing)."""
    return ts.tod_quantum * decode_stream(ts, ts.tod_huff, segs).astype(np.float64)
