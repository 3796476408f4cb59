"""Parity at the full 70 GHz-like workload (3600 segments, 9.35e8 samples),
in the launch configuration the benchmark times: autotuned FFT splits and
binning runs, the sweep captured into a hipGraph and replayed.

Outputs the oracle can compute one segment at a time are checked on a seeded
sample of segments: the decoded pointing bit-exact, n_corr within 1e-5 per
segment, and the binned b, A (bin_tod on the sampled segments alone, through
the accept flags) within 1e-12 with exact hits.  Properties that hold at any
size are checked on the whole set: the replayed sweep's n_corr equals the
eager sweep's bit for bit at the same seed and iteration, every sample is
binned once (the hits sum to the sample count), and the sweep's own
accumulators equal bin_tod's on the same inputs.

Generating the set takes a few minutes on a fresh machine; it is kept under
the benchmark's cache directory for later runs.  Progress goes straight to the
terminal so that the long steps are visibly alive.
"""
import os
import time

import numpy as np
import pytest
import torch

import synth
from oracle import huffman as oh
from oracle import tod as ot

pytestmark = pytest.mark.gpu

CACHE = "/tmp/c3cache"
NSAMPLE = 12
SEED_IT = 5


def _say(capsys, msg):
    with capsys.disabled():
        print("[full-size parity] " + msg, flush=True)


def _oracle_segment(ts, maps64, seed, it, q):
    n = int(ts.seg_off[q + 1] - ts.seg_off[q])
    a = int(ts.seg_off[q])
    pix = oh.StreamDecoder(ts.pix_huff).segment(q, n)
    psi = oh.StreamDecoder(ts.psi_huff).segment(q, n)
    gp = pix + ts.band_pix_off[ts.seg_band[q]]
    s = ot.project(maps64, gp, psi, ts.gain[q])
    r = ts.d[a:a + n].astype(np.float64) - s
    fs = ts.band_fsamp[ts.seg_band[q]]
    nc = ot.sample_ncorr_segment(r, fs, ts.sigma0[q], ts.fknee[q], ts.alpha[q], seed, q, it)
    return pix, psi, nc


@pytest.mark.timeout(1200)
def test_lfi70_full_size_sampled(capsys):
    from paper_2201_03509_amd import ops
    t0 = time.perf_counter()
    _say(capsys, "generating (or loading) the set under %s" % CACHE)
    with capsys.disabled():
        ts = synth.make_cached(2, cache_dir=CACHE, tod_streams=True)
    _say(capsys, "%d segments, %d samples (%.0f s)" % (ts.nseg, ts.nsamp, time.perf_counter() - t0))
    assert ts.nseg == 3600 and ts.nsamp > 9e8
    seed = synth.seed32(2)
    maps32 = ts.maps.astype(np.float32)
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        m_dev = torch.from_numpy(maps32).cuda()
        og = ops.new_outputs(tod, "mixed")
        c.decode_pointing(tod, og["pix"], og["psi"])
        c.sync()
        tune = os.path.join("/tmp", "c3tod_tune_test_%d.json" % os.getpid())
        c.autotune(tod, "mixed", og["pix"], cache_path=tune)
        os.remove(tune)
        _say(capsys, "autotuned (%.0f s)" % (time.perf_counter() - t0))
        for it in (SEED_IT - 1, SEED_IT):  # capture, then a replay at the checked iteration
            c.tod_sweep(tod, "mixed", m_dev, seed, it, og["ncorr"], og["acc"], og["pix"], og["psi"],
                        use_graph=True)
        oe = ops.new_outputs(tod, "mixed")
        c.tod_sweep(tod, "mixed", m_dev, seed, SEED_IT, oe["ncorr"], oe["acc"], oe["pix"], oe["psi"])
        c.sync()
        assert torch.equal(og["ncorr"], oe["ncorr"])
        assert torch.equal(og["pix"], oe["pix"]) and torch.equal(og["psi"], oe["psi"])
        acc_sweep = og["acc"].cpu().numpy()
        # the sweep's binning against bin_tod on the same inputs (every segment)
        ab = ops.new_acc(ts.npix_total, "cuda:0")
        c.bin_tod(tod, "mixed", og["pix"], og["psi"], tod.d, og["ncorr"], ab)
        c.sync()
        acc_bin = ab.cpu().numpy()
        del ab
        # bin_tod on the sampled segments alone (accept flags)
        rng = np.random.default_rng(2201)
        sample = np.sort(rng.choice(ts.nseg, size=NSAMPLE, replace=False))
        keep = np.zeros(ts.nseg, dtype=np.uint8)
        keep[sample] = 1
        saved = tod.seg_accept.clone()
        tod.seg_accept.copy_(torch.from_numpy(keep))
        asmp = ops.new_acc(ts.npix_total, "cuda:0")
        c.bin_tod(tod, "mixed", og["pix"], og["psi"], tod.d, og["ncorr"], asmp)
        c.sync()
        tod.seg_accept.copy_(saved)
        acc_smp = asmp.cpu().numpy()
        nc = og["ncorr"].cpu().numpy()
        pix = og["pix"].cpu().numpy()
        psi = og["psi"].cpu().numpy()
    finally:
        c.close()
    _say(capsys, "GPU done (%.0f s); oracle on %d sampled segments" % (time.perf_counter() - t0, NSAMPLE))

    assert acc_sweep[9].sum() == ts.nsamp
    assert np.array_equal(acc_sweep[9], acc_bin[9])
    for rows in (slice(0, 3), slice(3, 9)):
        scale = np.abs(acc_bin[rows]).max()
        assert np.abs(acc_sweep[rows] - acc_bin[rows]).max() <= 1e-12 * scale

    maps64 = maps32.astype(np.float64)
    errs = []
    for q in sample:
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        p_ref, s_ref, nc_ref = _oracle_segment(ts, maps64, seed, SEED_IT, int(q))
        assert np.array_equal(pix[a:b], p_ref) and np.array_equal(psi[a:b].astype(np.int64), s_ref)
        errs.append(np.linalg.norm(nc[a:b] - nc_ref) / np.linalg.norm(nc_ref))
    _say(capsys, "n_corr per segment rel L2: max %.2e" % max(errs))
    assert max(errs) < 1e-5
    # the oracle's binning of the sampled segments (the GPU's n_corr, as the
    # sweep bins it; their pointing was checked above)
    b_ref, A_ref, hits_ref = ot.bin_tod(ts, pix, psi, ts.d, nc, accept=keep)
    assert np.array_equal(acc_smp[9], hits_ref)
    assert np.abs(acc_smp[0:3] - b_ref).max() <= 1e-12 * np.abs(b_ref).max()
    assert np.abs(acc_smp[3:9] - A_ref).max() <= 1e-12 * np.abs(A_ref).max()
    _say(capsys, "done (%.0f s)" % (time.perf_counter() - t0))
