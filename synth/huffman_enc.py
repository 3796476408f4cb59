"""Huffman *encoder* for the synthetic compressed pointing (preprocessing only).

The paper stores pointing as sample-differenced integer streams that are
Huffman coded (section 4.1, Fig. 3).  This module produces such streams in the
format the decoders read; it holds no decoding logic.

Format (one table per scan and stream kind, shared by the scan's detectors):

* code lengths: ordinary Huffman lengths from symbol counts (merge the two
  lightest nodes; ties broken by lower count, then by smaller smallest symbol);
* canonical code assignment: symbols sorted by (length, value) receive
  consecutive codes, shifted left when the length grows;
* table blob (uint32 words): ``[nsym, maxlen, count[1..32], sym[0..nsym)]``
  where ``sym`` are int32 values in canonical order;
* each segment's bitstream is MSB-first in uint32 words, zero padded to a word;
* side index every ``chunk_len`` symbols: bit offset of the chunk's first
  code within the segment stream (uint32) and the undifferenced value just
  before the chunk (int32, 0 for the first chunk).
"""
import numpy as np

MAXLEN = 32
TABLE_HDR = 34  # nsym, maxlen, count[1..32]


def huffman_lengths(symbols, counts):
    """Code length per symbol.  ``symbols`` int array, ``counts`` > 0."""
    symbols = np.asarray(symbols, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    n = len(symbols)
    if n == 0:
        raise ValueError("empty alphabet")
    if n == 1:
        return np.ones(1, dtype=np.int64)
    # two-queue Huffman on leaves sorted by (count, symbol)
    order = np.lexsort((symbols, counts))
    leaf_w = counts[order].tolist()
    leaf_key = symbols[order].tolist()
    parent = [0] * (2 * n - 1)
    node_w = leaf_w + [0] * (n - 1)
    node_key = leaf_key + [0] * (n - 1)
    li, qi, qn = 0, n, n  # leaf cursor, internal-queue head, next internal id

    def pop():
        nonlocal li, qi
        if li < n and (qi >= qn or (node_w[li], node_key[li]) <= (node_w[qi], node_key[qi])):
            li += 1
            return li - 1
        qi += 1
        return qi - 1

    for _ in range(n - 1):
        a = pop()
        b = pop()
        node_w[qn] = node_w[a] + node_w[b]
        node_key[qn] = min(node_key[a], node_key[b])
        parent[a] = qn
        parent[b] = qn
        qn += 1
    root = qn - 1
    par = np.array(parent, dtype=np.int64)
    depth = np.zeros(2 * n - 1, dtype=np.int64)
    for v in range(root - 1, -1, -1):       # parents are created after children
        depth[v] = depth[par[v]] + 1
    lengths = np.empty(n, dtype=np.int64)
    lengths[order] = depth[:n]
    if lengths.max() > MAXLEN:
        raise ValueError("code length %d exceeds %d bits" % (lengths.max(), MAXLEN))
    return lengths


def canonical_codes(symbols, lengths):
    """Canonical codes.  Returns (sorted_symbols, sorted_lengths, codes)."""
    symbols = np.asarray(symbols, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    order = np.lexsort((symbols, lengths))
    ss, sl = symbols[order], lengths[order]
    codes = np.empty(len(ss), dtype=np.uint64)
    code = 0
    prev = int(sl[0])
    for i in range(len(ss)):
        L = int(sl[i])
        if i > 0:
            code = (code + 1) << (L - prev)
        prev = L
        codes[i] = code
    return ss, sl, codes


def build_table(values):
    """Table blob + lookup (symbol -> (code, length)) from an int array (an
    empty array gets the one-symbol table of 0, so every scan has a valid table)."""
    values = np.asarray(values, dtype=np.int64)
    if values.size == 0:
        values = np.zeros(1, dtype=np.int64)
    sym, cnt = np.unique(values, return_counts=True)
    lens = huffman_lengths(sym, cnt)
    ss, sl, codes = canonical_codes(sym, lens)
    nsym = len(ss)
    blob = np.zeros(TABLE_HDR + nsym, dtype=np.uint32)
    blob[0] = nsym
    blob[1] = int(sl.max())
    bc = np.bincount(sl, minlength=MAXLEN + 1)
    blob[2:2 + MAXLEN] = bc[1:MAXLEN + 1]
    blob[TABLE_HDR:] = ss.astype(np.int32).view(np.uint32)
    return blob, (ss, sl, codes)


def encode_values(diffs, lookup):
    """Pack the codes of ``diffs`` MSB-first into uint32 words.

    Returns (words, bit_len_of_each_symbol_prefix) where the second array is the
    bit offset of every symbol (int64, length n+1)."""
    ss, sl, codes = lookup
    vo = np.argsort(ss, kind="stable")
    sv = ss[vo]
    diffs = np.asarray(diffs, dtype=np.int64)
    j = np.searchsorted(sv, diffs)
    if np.any(j >= len(sv)) or np.any(sv[np.minimum(j, len(sv) - 1)] != diffs):
        raise ValueError("symbol missing from table")
    idx = vo[j]
    L = sl[idx].astype(np.int64)
    C = codes[idx].astype(np.uint64)
    pos = np.zeros(len(diffs) + 1, dtype=np.int64)
    np.cumsum(L, out=pos[1:])
    nbits = int(pos[-1])
    nwords = (nbits + 31) // 32
    p = pos[:-1]
    w = p >> 5
    sh = (p & 31).astype(np.int64)
    end = sh + L                                   # bit end within word w (1..63)
    # part that lands in word w
    first = np.where(end <= 32,
                     C << np.maximum(32 - end, 0).astype(np.uint64),
                     C >> np.maximum(end - 32, 0).astype(np.uint64)) & np.uint64(0xFFFFFFFF)
    spill = end > 32
    second = (C << np.maximum(64 - end, 0).astype(np.uint64)) & np.uint64(0xFFFFFFFF)
    acc = np.bincount(w, weights=first.astype(np.float64), minlength=nwords + 1)
    if np.any(spill):
        acc += np.bincount(w[spill] + 1, weights=second[spill].astype(np.float64),
                           minlength=nwords + 1)
    words = acc[:nwords].astype(np.uint64).astype(np.uint32)
    return words, pos


def difference(x):
    """Sample differencing d(i) - d(i-1) with d(-1) = 0 (section 4.1)."""
    x = np.asarray(x, dtype=np.int64)
    out = np.empty_like(x)
    if len(x):
        out[0] = x[0]
        out[1:] = x[1:] - x[:-1]
    return out


def chunk_index(x, pos, chunk_len):
    """Side index: bit offset and previous undifferenced value per chunk."""
    n = len(x)
    nch = (n + chunk_len - 1) // chunk_len
    starts = np.arange(nch, dtype=np.int64) * chunk_len
    bits = pos[starts].astype(np.uint32)
    prev = np.zeros(nch, dtype=np.int32)
    if nch > 1:
        prev[1:] = np.asarray(x, dtype=np.int64)[starts[1:] - 1].astype(np.int32)
    return bits, prev
