"""Every FFT kernel variant against the oracle's n_corr draw.

The split of each transform length is forced through a tuning file
(`tod_load_tuning`), so every compiled register column length, every row
radix (single-stage rows and multi-stage rows, whose first and last stages
touch memory directly), the LDS column tiles and the FP64 path each run once;
a file naming a radix without a compiled stage must fall back to a valid split.
"""
import json

import numpy as np
import pytest
import torch

import synth
from oracle import tod as ot

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}

# (prec, M1, M2, colreg, r1, r2): the register column lengths 16..100 paired with
# row lengths that use every FP32 row radix; LDS column tiles; the FP64 radices
CASES = [
    ("mixed", 16, 27, 1, [], [27]), ("mixed", 18, 25, 1, [], [25]), ("mixed", 20, 24, 1, [], [24]),
    ("mixed", 24, 20, 1, [], [20]), ("mixed", 25, 18, 1, [], [9, 2]), ("mixed", 27, 12, 1, [], [12]),
    ("mixed", 30, 10, 1, [], [10]), ("mixed", 32, 9, 1, [], [9]), ("mixed", 36, 8, 1, [], [8]),
    ("mixed", 40, 6, 1, [], [6]), ("mixed", 45, 5, 1, [], [5]), ("mixed", 48, 4, 1, [], [4]),
    ("mixed", 50, 3, 1, [], [3]), ("mixed", 54, 2, 1, [], [2]), ("mixed", 60, 30, 1, [], [6, 5]),
    ("mixed", 64, 36, 1, [], [9, 4]), ("mixed", 72, 40, 1, [], [8, 5]), ("mixed", 75, 48, 1, [], [12, 4]),
    ("mixed", 80, 50, 1, [], [25, 2]), ("mixed", 81, 54, 1, [], [27, 2]),
    ("mixed", 60, 600, 1, [], [24, 25]), ("mixed", 81, 729, 1, [], [27, 27]),
    ("mixed", 90, 32, 1, [], [8, 4]), ("mixed", 96, 45, 1, [], [9, 5]), ("mixed", 100, 27, 1, [], [27]),
    ("mixed", 96, 45, 0, [8, 4, 3], [9, 5]), ("mixed", 128, 30, 0, [8, 8, 2], [5, 6]),
    ("fp64", 96, 90, 0, [8, 4, 3], [10, 9]), ("fp64", 40, 36, 0, [8, 5], [6, 6]),
    ("fp64", 30, 64, 0, [5, 3, 2], [8, 8]),
]


def _case_id(c):
    return "%s-%dx%d-%s" % (c[0], c[1], c[2], "reg" if c[3] else "lds")


def _run(tmp_path, prec, M, choice):
    from paper_2201_03509_amd import ops
    ts = synth.make(0, nscan=1, length=("uniform", M, M), keep_truth=True)
    assert ts.nseg == 1 and int(ts.seg_off[1]) == M
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": [choice], "bin_stride": {}}))
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        m = ts.maps.astype(np.float32) if prec == "mixed" else ts.maps
        s_ref = ot.project_all(ts, m.astype(np.float64), ts.pix, ts.psi)
        s_in = s_ref.astype(np.float32 if prec == "mixed" else np.float64)
        seed, it = synth.seed32(ts.config), 7
        ref = ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it)
        out = torch.empty(ts.nsamp, dtype=torch.float32 if prec == "mixed" else torch.float64,
                          device="cuda")
        c.sample_ncorr(tod, prec, tod.d, torch.from_numpy(s_in).cuda(), seed, it, out)
        c.sync()
        got = out.cpu().numpy().astype(np.float64)
    finally:
        c.close()
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("case", CASES, ids=_case_id)
def test_forced_split(tmp_path, case):
    prec, M1, M2, colreg, r1, r2 = case
    M = M1 * M2
    choice = {"mixed": int(prec == "mixed"), "M": M, "M1": M1, "M2": M2,
              "B": 64 if colreg else 16, "colreg": colreg, "r1": r1, "r2": r2}
    assert _run(tmp_path, prec, M, choice) < TOL[prec]


def test_unsupported_radix_falls_back(tmp_path):
    """A cached split naming radix 16 (no compiled row stage) is ignored."""
    M1, M2 = 20, 32
    choice = {"mixed": 1, "M": M1 * M2, "M1": M1, "M2": M2, "B": 64, "colreg": 1, "r1": [],
              "r2": [16, 2]}
    assert _run(tmp_path, "mixed", M1 * M2, choice) < TOL["mixed"]


# row lengths with a compiled row kernel: every 5-smooth length in [2000, 5040]
def _smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


ROWC = [L for L in range(2000, 5041) if _smooth(L)]
F32_ROW_RADICES = [2, 3, 4, 5, 6, 8, 9, 10, 12, 20, 24, 25, 27]


def _generic_radices(L):
    r = []
    while L > 1:
        best = max(c for c in F32_ROW_RADICES if L % c == 0)
        r.append(best)
        L //= best
    return r


@pytest.mark.parametrize("L", ROWC)
def test_compiled_row_lengths(tmp_path, L):
    """Every compiled row length, as M = 16 x L: the n_corr draw (mode 0, with
    and without the draw) and the gain draw's filter (mode 2) against the
    oracle.  The rows 0 and M1/2 of each transform take the generic kernel."""
    from paper_2201_03509_amd import ops
    from oracle import gain as og
    M = 16 * L
    choice = {"mixed": 1, "M": M, "M1": 16, "M2": L, "B": 64, "colreg": 1, "r1": [],
              "r2": _generic_radices(L)}
    ts = synth.make(1, nscan=1, length=("uniform", M, M), keep_truth=True)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": [choice], "bin_stride": {}}))
    t = ot.project(ts.maps.astype(np.float32).astype(np.float64), ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    s_in = (t * np.repeat(ts.gain, np.diff(ts.seg_off))).astype(np.float32)
    seed, it = 31, 2
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        outs = []
        for mo in (False, True):
            out = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
            c.sample_ncorr(tod, "mixed", tod.d, torch.from_numpy(s_in).cuda(), seed, it, out, mean_only=mo)
            outs.append(out)
        g = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.sample_gain(tod, "mixed", tod.d, torch.from_numpy(t.astype(np.float32)).cuda(), seed, it, g)
        c.sync()
    finally:
        c.close()
    for mo, out in zip((False, True), outs):
        ref = ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it, mean_only=mo)
        got = out.cpu().numpy().astype(np.float64)
        for q in range(ts.nseg):
            a, b = ts.seg_off[q], ts.seg_off[q + 1]
            assert np.linalg.norm(got[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]) < TOL["mixed"], (L, mo, q)
    g_ref, _ = og.sample_gain_all(ts, ts.d, t.astype(np.float32).astype(np.float64), seed, it)
    assert np.all(np.abs(g.cpu().numpy() - g_ref) <= TOL["mixed"] * np.abs(g_ref))


def _next_5smooth(n):
    while not _smooth(n):
        n += 1
    return n


# register column splits with segments of ragged lengths: every length has
# M = M1 M2 as its next 5-smooth number, so one forced split serves them all;
# odd and even n, n = M and n < M (the pad repeats r_0), and, with several
# detectors per scan, odd and even sample offsets
RAGGED = [
    (27, 16, [8, 2], [431, 407, 432, 420]),
    (81, 25, [25], [2025, 2023, 2001, 2012]),
    (16, 135, [27, 5], [2160, 2159, 2053, 2100]),
    (100, 30, [6, 5], [3000, 2999, 2917, 2950]),
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: "%dx%d" % (c[0], c[1]))
def test_register_columns_ragged_lengths(tmp_path, case):
    """The forward column pass reads each pair of reals of the mirrored,
    padded extension with one load: adjacent samples, mirrored pairs, the last
    sample twice (odd n) and the pad's r_0.  Both of its inputs (d - s of a
    standalone draw, the sweep's residual) against the oracle per segment."""
    from paper_2201_03509_amd import ops
    M1, M2, r2, lengths = case
    M = M1 * M2
    assert all(_next_5smooth(n) == M for n in lengths)
    ts = synth.make(1, nscan=len(lengths), length=("list", *lengths), keep_truth=True)
    offs = np.asarray(ts.seg_off[:-1])
    assert (offs % 2 == 1).any() and (np.diff(ts.seg_off) % 2 == 1).any()
    choice = {"mixed": 1, "M": M, "M1": M1, "M2": M2, "B": 64, "colreg": 1, "r1": [], "r2": r2}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": [choice], "bin_stride": {}}))
    m32 = ts.maps.astype(np.float32)
    s_ref = ot.project_all(ts, m32.astype(np.float64), ts.pix, ts.psi)
    s_in = s_ref.astype(np.float32)
    seed, it = synth.seed32(ts.config), 3
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        draw = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        c.sample_ncorr(tod, "mixed", tod.d, torch.from_numpy(s_in).cuda(), seed, it, draw)
        out = ops.new_outputs(tod, "mixed")
        c.tod_sweep(tod, "mixed", torch.from_numpy(np.ascontiguousarray(m32)).cuda(), seed, it,
                    out["ncorr"], out["acc"], out["pix"], out["psi"])
        c.sync()
    finally:
        c.close()
    refs = {"draw": ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it),
            "sweep": ot.sample_ncorr_all(ts, ts.d, s_ref, seed, it)}
    gots = {"draw": draw.cpu().numpy().astype(np.float64),
            "sweep": out["ncorr"].cpu().numpy().astype(np.float64)}
    for key in refs:
        for q in range(ts.nseg):
            a, b = ts.seg_off[q], ts.seg_off[q + 1]
            ref, got = refs[key][a:b], gots[key][a:b]
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < TOL["mixed"], (key, q, b - a)


def _chisq_noise_case(tmp_path, ts, choice, seed, it):
    """tod_chisq (the row pass's Whittle sums, mode 1) and sample_noise (its
    periodogram, mode 4) under a forced split, against the oracle."""
    from paper_2201_03509_amd import ops
    from oracle import noise as on
    from chisq_bounds import magnitudes
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": [choice], "bin_stride": {}}))
    m32 = ts.maps.astype(np.float32)
    t = ot.project(m32.astype(np.float64), ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    s = t * np.repeat(ts.gain, np.diff(ts.seg_off))
    nc32 = ot.sample_ncorr_all(ts, ts.d, s, seed, it).astype(np.float32)
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        ncd = torch.from_numpy(nc32).cuda()
        J = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.tod_chisq(tod, "mixed", torch.from_numpy(ts.pix.astype(np.int32)).cuda(),
                    torch.from_numpy(ts.psi.astype(np.uint16)).cuda(), tod.d, ncd,
                    torch.from_numpy(m32).cuda(), J)
        outs = [torch.empty(ts.nseg, dtype=torch.float64, device="cuda") for _ in range(3)]
        fk_in = torch.from_numpy(np.asarray(ts.fknee, dtype=np.float64)).cuda()
        c.sample_noise(tod, "mixed", tod.d, torch.from_numpy(t.astype(np.float32)).cuda(), ncd, seed, it,
                       *outs, fknee=fk_in)
        c.sync()
    finally:
        c.close()
    nc_r = nc32.astype(np.float64)
    J_ref = ot.chisq_all(ts, m32.astype(np.float64), ts.pix, ts.psi, ts.d, nc_r)
    mag, fft, _ = magnitudes(ts, m32.astype(np.float64), nc_r, float(np.finfo(np.float32).eps))
    assert np.all(np.abs(J.cpu().numpy() - J_ref) <= TOL["mixed"] * mag[0] + fft[0])
    nz_ref = on.sample_noise_all(ts, ts.d, t.astype(np.float32).astype(np.float64), ts.gain, nc_r, ts.fknee,
                                 seed, it)
    got = np.stack([o.cpu().numpy() for o in outs])
    assert np.isfinite(got).all()
    assert (np.abs(got - nz_ref) / np.abs(nz_ref)).max() < TOL["mixed"]


@pytest.mark.parametrize("L", ROWC)
def test_compiled_row_lengths_chisq_noise(tmp_path, L):
    """Every compiled row length, as M = 16 x L (rows 0 and 8 of the split
    share one task): the chi^2's Whittle sums and the noise draw's periodogram
    against the oracle."""
    M = 16 * L
    choice = {"mixed": 1, "M": M, "M1": 16, "M2": L, "B": 64, "colreg": 1, "r1": [],
              "r2": _generic_radices(L)}
    ts = synth.make(1, nscan=1, length=("uniform", M, M), keep_truth=True)
    _chisq_noise_case(tmp_path, ts, choice, 41, 3)


def test_self_rows_of_two_segments(tmp_path):
    """An odd column length (27): each segment has one row that holds its own
    mirror modes (k1 = 0), and the compiled kernel pairs such rows of two
    segments in one task (eight segments: four pair tasks).  n_corr, the
    chi^2 and the noise draw against the oracle; the gain draw (mode 2) takes
    those rows on the generic kernel."""
    from paper_2201_03509_amd import ops
    from oracle import gain as og
    M1, L = 27, 2000
    M = M1 * L
    choice = {"mixed": 1, "M": M, "M1": M1, "M2": L, "B": 64, "colreg": 1, "r1": [],
              "r2": _generic_radices(L)}
    ts = synth.make(1, nscan=2, length=("uniform", M, M), keep_truth=True)
    assert ts.nseg == 8
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": [choice], "bin_stride": {}}))
    t = ot.project(ts.maps.astype(np.float32).astype(np.float64), ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    s_in = (t * np.repeat(ts.gain, np.diff(ts.seg_off))).astype(np.float32)
    seed, it = 17, 5
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        out = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        c.sample_ncorr(tod, "mixed", tod.d, torch.from_numpy(s_in).cuda(), seed, it, out)
        g = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
        c.sample_gain(tod, "mixed", tod.d, torch.from_numpy(t.astype(np.float32)).cuda(), seed, it, g)
        c.sync()
    finally:
        c.close()
    ref = ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it)
    got = out.cpu().numpy().astype(np.float64)
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        assert np.linalg.norm(got[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]) < TOL["mixed"], q
    g_ref, _ = og.sample_gain_all(ts, ts.d, t.astype(np.float32).astype(np.float64), seed, it)
    assert np.all(np.abs(g.cpu().numpy() - g_ref) <= TOL["mixed"] * np.abs(g_ref))
    _chisq_noise_case(tmp_path, ts, choice, seed, it)
