"""FFT work batching (`tod_set_fft_batch`) changes where the intermediate
spectra live, not the results: every FFT-based call gives the same output
with small batches (several segments per batch, a batch boundary inside the
set) as with one batch.  Also the masked draw with the column passes forced
onto the LDS tiles (mixed precision), against the oracle.
"""
import json

import numpy as np
import pytest
import torch

import synth
from oracle import gapfill as og
from oracle import tod as ot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    ts = synth.make(1, nscan=3, length=("uniform", 9000, 13000), keep_truth=True)
    mask = synth.plane_mask(ts, ts.pix)
    t = ot.project(ts.maps.astype(np.float32).astype(np.float64), ot.global_pix(ts, ts.pix), ts.psi, 1.0)
    return ts, mask, t


def _calls(ctx, ts, mask, t, prec):
    from paper_2201_03509_amd import ops
    tod = ops.DeviceTod(ts, "cuda:0")
    ft = torch.float32 if prec == "mixed" else torch.float64
    nf = np.float32 if prec == "mixed" else np.float64
    td = torch.from_numpy(t.astype(nf)).cuda()
    s = torch.from_numpy((t * np.repeat(ts.gain, np.diff(ts.seg_off))).astype(nf)).cuda()
    out = {}
    nc = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    ctx.sample_ncorr(tod, prec, tod.d, s, 3, 1, nc)
    ncm = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    ctx.sample_ncorr_masked(tod, prec, tod.d, s, torch.from_numpy(mask).cuda(), 3, 1, ncm,
                            tol=1e-6 if prec == "mixed" else 1e-13)
    g = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
    sg = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
    ctx.sample_gain(tod, prec, tod.d, td, 3, 1, g, sg)
    xi = [torch.empty(ts.nseg, dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.sample_noise(tod, prec, tod.d, td, nc, 3, 1, *xi)
    ctx.sync()
    out["ncorr"] = nc.cpu().numpy().astype(np.float64)
    out["masked"] = ncm.cpu().numpy().astype(np.float64)
    out["gain"] = g.cpu().numpy()
    out["noise"] = np.stack([x.cpu().numpy() for x in xi])
    return out


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batched_equals_unbatched(data, prec):
    from paper_2201_03509_amd import ops
    ts, mask, t = data
    c = ops.Context(0)
    try:
        one = _calls(c, ts, mask, t, prec)
        n_max = int(np.diff(ts.seg_off).max())
        c.set_fft_batch(3 * n_max)  # about three segments per batch
        many = _calls(c, ts, mask, t, prec)
    finally:
        c.close()
    for k in ("ncorr", "masked", "gain"):
        assert np.array_equal(one[k], many[k]), k
    # the periodogram bins are summed with atomics: last bits may differ
    assert np.abs(one["noise"] - many["noise"]).max() <= 1e-12 * np.abs(one["noise"]).max()


def test_masked_draw_on_lds_column_tiles(data, tmp_path):
    """Force every segment's column passes onto the LDS tiles (mixed): the
    whole-vector input and output of those kernels against the oracle."""
    from paper_2201_03509_amd import ops
    ts, mask, t = data
    # splits whose column lengths have no register kernel: (M1, LDS column
    # radices, row radices) per complex length M of this set
    split = {9720: (120, [8, 5, 3], [27, 3]), 10800: (120, [8, 5, 3], [10, 9]),
             12800: (128, [8, 8, 2], [25, 4])}
    Ms = sorted({int(ot.fft_length(n)) // 2 for n in np.diff(ts.seg_off)})
    assert set(Ms) <= set(split)
    choices = [{"mixed": 1, "M": M, "M1": split[M][0], "M2": M // split[M][0], "B": 16, "colreg": 0,
                "r1": split[M][1], "r2": split[M][2]} for M in Ms]
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fft": choices, "bin_stride": {}}))
    s_in = (t * np.repeat(ts.gain, np.diff(ts.seg_off))).astype(np.float32)
    ref, _ = og.cg_ncorr_all(ts, ts.d, s_in.astype(np.float64), mask, 5, 2, tol=1e-14)
    c = ops.Context(0)
    try:
        c.load_tuning(str(path))
        tod = ops.DeviceTod(ts, "cuda:0")
        out = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        c.sample_ncorr_masked(tod, "mixed", tod.d, torch.from_numpy(s_in).cuda(), torch.from_numpy(mask).cuda(),
                              5, 2, out, tol=1e-6)
        c.sync()
        got = out.cpu().numpy().astype(np.float64)
    finally:
        c.close()
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        assert np.linalg.norm(got[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]) < 1e-5
