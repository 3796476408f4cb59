#!/usr/bin/env python3
"""Throughput of the TOD sweep (decode -> project -> n_corr draw -> bin) on one GPU.

One *step* is one fused sweep over the whole synthetic TOD set of the chosen
workload (default: the 70 GHz-like set, nside 1024, 12 detectors x 300 scans of
230k-290k samples at 78.8 Hz, i.e. ~9.4e8 samples) with all inputs resident in
HBM.  Prints ONE JSON line on stdout; progress goes to stderr.

The timed region replays the mixed-precision sweep as one captured hipGraph
per step (HIP events on the context stream around it).  The same number of
sweeps then runs eagerly with HIP events around every kernel, so the dominant
kernel's duration is measured live; that eager sweep and the plain-FP64 sweep
are reported beside the headline value.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed
# FP32) x 2.4 GHz.  The kernels here are built without packed FP32
# instructions, so half of it is the ceiling they can reach.
FP32_VALU_PEAK_TFLOPS = 157.3
# families bound by vector-ALU issue rather than by HBM (the counter pass finds
# the row pass filling about 0.82 of the chip's VALU issue slots)
ALU_BOUND = {"fft_row"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(ts, tod, prec, sum_m):
    """Compulsory bytes per sweep of each kernel (summed over its launches):
    every input array the kernel needs read once, every output written once."""
    f = 4 if prec == "mixed" else 8
    ns = ts.nsamp
    dsz = ts.d.dtype.itemsize
    comp = 0
    for hs in (ts.pix_huff, ts.psi_huff):
        comp += hs.words.nbytes + hs.chunk_bit.nbytes + hs.chunk_prev.nbytes + hs.tables.nbytes
    npt = ts.npix_total
    return {
        "decode": comp + ns * (4 + 2),
        "fft_col_fwd": ns * f + 2 * f * sum_m,
        "fft_row": 2 * (2 * f * sum_m),
        "fft_col_inv": 2 * f * sum_m + ns * f,
        "bin": ns * (4 + 2 + dsz + f) + 2 * 80 * npt,
        "project": ns * (4 + 2 + dsz + f) + 3 * f * npt,  # the sweep's residual r = d - g P m
        "solve": 80 * npt + 3 * f * npt + 8 * npt,
        "chisq_time": ns * (4 + 2 + dsz + f) + 3 * f * npt,
    }


def next5(n):
    m = max(1, n)
    while True:
        x = m
        for q in (2, 3, 5):
            while x % q == 0:
                x //= q
        if x == 1:
            return m
        m += 1


# the sources each timed kernel family is compiled from (kernel code and the
# headers it includes); its counter summary is valid while these are unchanged
FAMILY_SOURCES = {
    "decode": ["decode.hip", "common.h"],
    "project": ["pixel.hip", "common.h"],
    "bin": ["pixel.hip", "common.h"],
    "zero": ["pixel.hip", "common.h"],
    "fft_col_fwd": ["fftcol.hip", "fft.hip", "fftdev.h", "fftmode.h", "rng.h", "common.h"],
    "fft_row": ["fft.hip", "rowc.hip", "rowc.h", "fftdev.h", "fftmode.h", "rng.h", "common.h"],
    "fft_col_inv": ["fftcol.hip", "fft.hip", "fftdev.h", "fftmode.h", "rng.h", "common.h"],
}


def source_sha(family):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2201_03509_amd", "csrc")
    for f in sorted(FAMILY_SOURCES[family]):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload):
    """The committed counter summary of a kernel family (HBM bytes per sweep
    over all its launches, VALU issue fraction), if it was taken on the
    current kernel sources; else {}."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    try:
        t = json.load(open(p))
    except ValueError:
        return {}
    e = t.get(workload, {}).get(kernel)
    if not e or kernel not in FAMILY_SOURCES or e.get("source_sha") != source_sha(kernel):
        return {}
    return e


def sweep_counters(workload, ms_step):
    """HBM bytes of one whole sweep by counters (the committed per-family
    FETCH_SIZE + WRITE_SIZE summary summed over every family of the sweep),
    and the rate they make at the timed step; None unless every family's
    counters were taken on its current sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p)).get(workload, {})
    except ValueError:
        return None
    fams = [k for k in t if k in FAMILY_SOURCES]
    if not fams or any(t[k].get("source_sha") != source_sha(k) for k in fams):
        return None
    gb = sum(t[k]["bytes_per_step"] for k in fams) / 1e9
    return {"gb_per_step": round(gb, 2), "families": sorted(fams),
            "gbs_at_step": round(gb / (ms_step / 1e3), 1),
            "frac_of_peak": round(gb / (ms_step / 1e3) / HBM_PEAK_GBS, 4)}


def row_pass_flops(ts, tuned):
    """Algorithmic FP32 flops of the row passes of one sweep.  A segment of
    M = M1 x M2 complex points has M1 rows: each is transformed forward and
    back (5 M2 log2 M2 flops each, the conventional count), and each of its M
    modes takes about 30 flops for the real-spectrum split, the
    constrained-realisation filter and the re-pack.  The Philox and
    Box-Muller work (integer and transcendental) is not counted."""
    import math
    import numpy as np
    m2_of = {int(e["M"]): int(e["M2"]) for e in tuned.get("fft", []) if e.get("mixed") == 1}
    fl = 0.0
    for n in np.diff(ts.seg_off):
        if n <= 0:
            continue
        M = next5(int(n))
        M2 = m2_of.get(M)
        if M2 is None:
            return None
        fl += 10.0 * M * math.log2(M2) + 30.0 * M
    return fl


# ------------------------------------------------------------- CPU baseline
_BASE = {}


def _oracle_segment(q):
    ts, seed, it, maps32 = _BASE["ts"], _BASE["seed"], _BASE["it"], _BASE["maps"]
    import numpy as np
    from oracle import huffman as oh
    from oracle import tod as ot
    n = int(ts.seg_off[q + 1] - ts.seg_off[q])
    tm = [time.perf_counter()]
    pix = oh.StreamDecoder(ts.pix_huff).segment(q, n)
    psi = oh.StreamDecoder(ts.psi_huff).segment(q, n)
    tm.append(time.perf_counter())
    a = ts.seg_off[q]
    gp = pix + ts.band_pix_off[ts.seg_band[q]]
    s = ot.project(maps32, gp, psi, ts.gain[q])
    r = ts.d[a:a + n].astype(np.float64) - s
    tm.append(time.perf_counter())
    fs = ts.band_fsamp[ts.seg_band[q]]
    nc = ot.sample_ncorr_segment(r, fs, ts.sigma0[q], ts.fknee[q], ts.alpha[q], seed, q, it)
    tm.append(time.perf_counter())
    _, c, sn = ot.pointing_rows(gp, psi)
    g = ts.gain[q]
    w = g / ts.sigma0[q] ** 2
    v = ts.d[a:a + n] - nc
    # binned on the segment's own pixels (the accumulation of section 2.4)
    up, inv = np.unique(gp, return_inverse=True)
    b = np.zeros((3, len(up)))
    A = np.zeros((6, len(up)))
    rows = (np.ones(n), c, sn)
    for i in range(3):
        np.add.at(b[i], inv, w * v * rows[i])
    for k, (i, j) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        np.add.at(A[k], inv, g * w * rows[i] * rows[j])
    hits = np.bincount(inv, minlength=len(up))
    tm.append(time.perf_counter())
    steps = dict(zip(("decode", "project", "n_corr", "bin"), np.diff(tm)))
    return q, pix, nc, (up, b, A, hits), steps


MASKED_IT = 7777      # Gibbs iteration number of the masked-draw leg
RCOND_MIN = 1e-3      # conditioning threshold of the map solve in the accuracy report
MASKED_TOL = 1e-6     # its CG tolerance (residual reduction from x0 = M b)


GAIN_IT = 4242        # Gibbs iteration number of the gain-draw leg
NOISE_IT = 4343       # Gibbs iteration number of the noise-parameter leg


def _oracle_next(q):
    """Masked n_corr draw of segment q (processing mask +-10 deg around the
    map frame's equator) by the oracle's CG, and its gain draw, for the
    accuracy reports of those legs."""
    ts, seed, maps32 = _BASE["ts"], _BASE["seed"], _BASE["maps"]
    import numpy as np
    import synth
    from oracle import gapfill as og
    from oracle import huffman as oh
    from oracle import tod as ot
    n = int(ts.seg_off[q + 1] - ts.seg_off[q])
    pix = oh.StreamDecoder(ts.pix_huff).segment(q, n)
    psi = oh.StreamDecoder(ts.psi_huff).segment(q, n)
    a = ts.seg_off[q]
    band = ts.seg_band[q]
    gp = pix + ts.band_pix_off[band]
    s = ot.project(maps32, gp, psi, ts.gain[q])
    r = ts.d[a:a + n].astype(np.float64) - s
    m = synth.plane_mask_pixels(int(ts.band_nside[band]), pix)
    sec = {}
    c0 = time.perf_counter()
    nc, k = og.cg_ncorr_segment(r, m, ts.band_fsamp[band], ts.sigma0[q], ts.fknee[q], ts.alpha[q],
                                seed, q, MASKED_IT, tol=1e-12)
    sec["masked"] = time.perf_counter() - c0
    from oracle import gain as ogain
    from oracle import noise as onoise
    t = ot.project(maps32, gp, psi, 1.0)
    c0 = time.perf_counter()
    g, sg, _, _ = ogain.sample_gain_segment(ts.d[a:a + n], t, ts.band_fsamp[band], ts.sigma0[q], ts.fknee[q],
                                            ts.alpha[q], seed, q, GAIN_IT)
    sec["gain"] = time.perf_counter() - c0
    # noise parameters from the oracle's own n_corr of the sweep's last iteration
    ncs = ot.sample_ncorr_segment(r, ts.band_fsamp[band], ts.sigma0[q], ts.fknee[q], ts.alpha[q], seed, q,
                                  _BASE["it"])
    c0 = time.perf_counter()
    xi = onoise.sample_noise_segment(ts.d[a:a + n], t, ts.gain[q], ncs, ts.band_fsamp[band], ts.fknee[q],
                                     seed, q, NOISE_IT)
    sec["noise"] = time.perf_counter() - c0
    if getattr(ts, "tod_huff", None) is not None:
        c0 = time.perf_counter()
        oh.StreamDecoder(ts.tod_huff).segment(q, n)
        oh.StreamDecoder(ts.flag_huff).segment(q, n)
        sec["streams"] = time.perf_counter() - c0
    # chi^2 and its gain derivative at that same n_corr
    c0 = time.perf_counter()
    rc = r - ncs
    fs = ts.band_fsamp[band]
    J = ot.chisq_segment(rc, ncs, fs, ts.sigma0[q], ts.fknee[q], ts.alpha[q])
    _, dg, _, _, _ = ot.chisq_grad_segment(rc, t, ncs, fs, ts.gain[q], ts.sigma0[q], ts.fknee[q], ts.alpha[q])
    sec["chisq"] = time.perf_counter() - c0
    # sizes of the terms summed into J and dJ/dg, to scale their errors by
    I, P, _ = ot.whittle_parts(ncs, fs, ts.sigma0[q], ts.fknee[q], ts.alpha[q])
    J_terms = float(np.sum(rc * rc) / ts.sigma0[q] ** 2 + np.sum(I / P) + np.sum(np.abs(np.log(P))))
    dg_terms = 2.0 * float(np.sum(np.abs(t * rc))) / ts.sigma0[q] ** 2
    return q, nc, k, g, sg, xi, n, sec, (J, J_terms, dg, dg_terms)


def cpu_baseline(ts, seed, it, maps32, budget_s=15.0, masked_segments=2):
    """The oracle, as it stands, over a bounded sample of the same workload,
    one segment per worker process.  Runs before the GPU is touched (the
    worker processes are forked)."""
    import multiprocessing as mp
    import numpy as np
    workers = max(1, min(16, os.cpu_count() or 1))
    _BASE.update(ts=ts, seed=seed, it=it, maps=maps32)
    t0 = time.perf_counter()
    _oracle_segment(0)
    t1 = time.perf_counter() - t0
    single = int(ts.seg_off[1] - ts.seg_off[0]) / t1   # one process alone on the host
    nseg = int(max(workers, min(ts.nseg, budget_s * workers / max(t1, 1e-3))))
    nseg = min(nseg, ts.nseg)
    log("cpu baseline: %.2fs per segment, sampling %d segments on %d processes" % (t1, nseg, workers))
    ctx = mp.get_context("fork")
    res = []
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        for r in pool.imap_unordered(_oracle_segment, range(nseg)):
            res.append(r)
            if len(res) % workers == 0:
                log("  oracle segments done: %d/%d" % (len(res), nseg))
    wall = time.perf_counter() - t0
    nsamp = int(sum(ts.seg_off[q + 1] - ts.seg_off[q] for q in range(nseg)))
    # masked-draw and gain references (not part of the timed sample)
    mq = [int(q) for q in np.linspace(0, ts.nseg - 1, masked_segments).round()] if masked_segments else []
    with ctx.Pool(max(1, min(workers, len(mq)))) as pool:
        _BASE["next"] = list(pool.imap_unordered(_oracle_next, mq)) if mq else []
    step_s = {k: float(sum(r[4][k] for r in res)) for k in ("decode", "project", "n_corr", "bin")}
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": nsamp / wall, "unit": "TOD samples/s", "cores": workers, "kind": "oracle",
        "sample": "%d of %d segments (%d samples): decode+project+n_corr+bin, FP64 numpy/C, "
                  "one segment per process" % (nseg, ts.nseg, nsamp),
        "cpu_model": model, "host_cpus": os.cpu_count(),
        "single_core_value": single,
        "per_step_core_seconds": {k: round(v, 3) for k, v in step_s.items()},
        "per_step_samples_per_core_second": {k: nsamp / v if v > 0 else None for k, v in step_s.items()},
        "wall_seconds": round(wall, 2),
    }, [r[:4] for r in res]


def oracle_binned(res):
    """The oracle's (pixels, b, A, hits) summed over the sampled segments."""
    import numpy as np
    up = np.unique(np.concatenate([r[3][0] for r in res]))
    b = np.zeros((3, len(up)))
    A = np.zeros((6, len(up)))
    hits = np.zeros(len(up), dtype=np.int64)
    for r in res:
        u, bb, AA, hh = r[3]
        j = np.searchsorted(up, u)
        b[:, j] += bb
        A[:, j] += AA
        hits[j] += hh
    return up, b, A, hits


def compare_maps(res, acc, gpu_map, rcond_min):
    """Binned accumulators and solved maps of the sampled segments, GPU vs
    oracle, on every pixel they touch (maps: where the oracle's solve is
    conditioned)."""
    import numpy as np
    from oracle import tod as ot
    up, b, A, hits = oracle_binned(res)
    ga = acc[:, up]
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
    m_ref, _ = ot.solve_maps(b, A, hits, rcond_min)
    ok = np.isfinite(m_ref[0])
    gm = gpu_map[:, up]
    return {"pixels": int(len(up)), "b_rel_l2": [rel(ga[i], b[i]) for i in range(3)],
            "A_rel_l2": rel(ga[3:9], A), "hits_exact": bool(np.array_equal(ga[9], hits)),
            "conditioned_pixels": int(ok.sum()),
            "map_rel_l2_TQU": [rel(gm[i, ok], m_ref[i, ok]) for i in range(3)],
            "gpu_conditioned_same": bool(np.array_equal(np.isfinite(gm[0]), ok))}


def compare_to_oracle(ts, res, gpu_ncorr, gpu_pix):
    import numpy as np
    errs, exact = [], True
    for q, pix, nc, _ in res:
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        g = gpu_ncorr[a:b].astype(np.float64)
        errs.append(float(np.linalg.norm(g - nc) / np.linalg.norm(nc)))
        exact &= bool(np.array_equal(gpu_pix[a:b], pix))
    return {"ncorr_rel_l2_max": max(errs), "ncorr_rel_l2_median": float(np.median(errs)),
            "decode_bit_exact": exact, "segments": len(res)}


def stream_leg(ctx, ts, tod):
    """Decoding the compressed TOD and flag streams over the whole workload;
    returns the report and the processing mask decoded from the flags."""
    import torch
    import synth
    dev = tod.d.device
    d = torch.empty(ts.nsamp, dtype=torch.float32, device=dev)
    ms_d, _ = timed_call(ctx, lambda: ctx.decode_tod(tod, "mixed", d))
    exact = bool(torch.equal(d, tod.d))
    del d
    mask = torch.empty(ts.nsamp, dtype=torch.uint8, device=dev)
    ms_f, _ = timed_call(ctx, lambda: ctx.decode_flags(tod, synth.FLAG_PLANE, None, mask))

    def comp(h):
        return h.words.nbytes + h.chunk_bit.nbytes + h.chunk_prev.nbytes + h.tables.nbytes

    rep = {"tod": {"ms_per_call": round(ms_d, 3), "samples_per_s": ts.nsamp / (ms_d / 1e3),
                   "compressed_bytes_per_sample": comp(ts.tod_huff) / ts.nsamp,
                   "ratio_vs_32bit": 4.0 * ts.nsamp / comp(ts.tod_huff),
                   "decoded_equals_fp32_tod": exact},
           "flags": {"ms_per_call": round(ms_f, 3), "samples_per_s": ts.nsamp / (ms_f / 1e3),
                     "compressed_bytes_per_sample": comp(ts.flag_huff) / ts.nsamp,
                     "ratio_vs_32bit": 4.0 * ts.nsamp / comp(ts.flag_huff)},
           "cpu_baseline_tod_and_flags": oracle_rate("streams")}
    # compulsory: the compressed stream (words, side index, tables) read once,
    # the FP32 TOD or the mask byte written once
    rep["tod"]["roofline"] = leg_roofline(comp(ts.tod_huff) + 4 * ts.nsamp, ms_d)
    rep["flags"]["roofline"] = leg_roofline(comp(ts.flag_huff) + ts.nsamp, ms_f)
    log("tod stream: %.2f ms, flag stream: %.2f ms" % (ms_d, ms_f))
    return rep, mask


def masked_leg(ctx, ts, tod, out, maps32, seed, gpu_pix, mask):
    """The masked n_corr draw (CG gap filling) over the whole workload with the
    processing mask decoded from the flag stream (+-10 deg around the map
    frame's equator): one warm-up call, one timed call (HIP events around
    every launch), iteration counts and the error against the oracle's CG on
    the sampled segments."""
    import numpy as np
    import torch
    import synth
    dev = tod.d.device
    mask_h = synth.plane_mask(ts, gpu_pix)
    mask_ok = bool(np.array_equal(mask.cpu().numpy(), mask_h))
    s = torch.empty(ts.nsamp, dtype=torch.float32, device=dev)
    ctx.project_sky(tod, "mixed", out["pix"], out["psi"], maps32, s)
    nc = torch.empty(ts.nsamp, dtype=torch.float32, device=dev)
    iters = torch.empty(ts.nseg, dtype=torch.int32, device=dev)
    ctx.sample_ncorr_masked(tod, "mixed", tod.d, s, mask, seed, MASKED_IT, nc, tol=MASKED_TOL, iters=iters)
    ctx.sync()
    ctx.enable_timing(True)
    ctx.kernel_times()
    t0 = time.perf_counter()
    ctx.sample_ncorr_masked(tod, "mixed", tod.d, s, mask, seed, MASKED_IT, nc, tol=MASKED_TOL, iters=iters)
    ctx.sync()
    ms = (time.perf_counter() - t0) * 1e3
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    it_h = iters.cpu().numpy()
    rep = {"ms_per_call": round(ms, 2), "samples_per_s": ts.nsamp / (ms / 1e3),
           "masked_fraction": round(float(1.0 - mask_h.mean()), 4), "tol": MASKED_TOL,
           "mask_from_flag_stream_equals_plane_mask": mask_ok,
           "iterations": {"min": int(np.abs(it_h).min()), "median": float(np.median(np.abs(it_h))),
                          "max": int(np.abs(it_h).max()), "unconverged": int((it_h < 0).sum())},
           "kernels_ms": {k: round(v[0], 2) for k, v in kt.items() if v[1]},
           "launches": {k: v[1] for k, v in kt.items() if v[1]}}
    ref = _BASE.get("next")
    if ref:
        g = nc.cpu().numpy()
        errs = []
        for q, r, k, *_ in ref:
            a, b = ts.seg_off[q], ts.seg_off[q + 1]
            errs.append({"segment": q, "rel_l2": float(np.linalg.norm(g[a:b] - r) / np.linalg.norm(r)),
                         "iterations_gpu": int(it_h[q]), "iterations_oracle": int(k)})
        rep["accuracy_vs_oracle"] = errs
    # compulsory, estimated per segment from its iteration count: whole-vector
    # FFT round trips (x0, one per iteration, the final M S y) move 6 N f bytes
    # each, the F^H W1 transform 3 N f; the right-hand side reads d, s, mask
    # and F^H W1 and writes mu u (N (4 + 4 + 1 + 4 + 4)); the small system
    # moves about 108 B per masked extended position per iteration; the crop
    # reads x0 and M S y and writes n_corr (3 n f)
    n_s = np.diff(ts.seg_off).astype(np.int64)
    N_s = np.array([2 * next5(int(x)) for x in n_s], dtype=np.int64)
    mk = (mask_h == 0).astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(mk)])
    m_s = 2 * (cs[ts.seg_off[1:]] - cs[ts.seg_off[:-1]])
    its = np.abs(it_h).astype(np.int64)
    f = 4
    nbytes = float(np.sum((its + 2) * 6 * N_s * f + 3 * N_s * f + 17 * N_s + 108 * m_s * its + 3 * n_s * f))
    rep["roofline_estimate"] = leg_roofline(nbytes, ms)
    rep["cpu_baseline"] = oracle_rate("masked")
    if rep["cpu_baseline"]:
        rep["cpu_baseline"]["sample"] += "; full-system PCG to tol 1e-12"
    log("masked n_corr: %.1f ms per call, iterations %s" % (ms, rep["iterations"]))
    return rep


def oracle_rate(kind):
    """The oracle timed on the sampled segments of a leg (one process per
    segment): samples/s of one process."""
    ref = _BASE.get("next")
    if not ref or kind not in ref[0][7]:
        return None
    n = sum(r[6] for r in ref)
    sec = sum(r[7][kind] for r in ref)
    return {"value": n / sec, "unit": "TOD samples/s", "cores": 1, "kind": "oracle",
            "sample": "%d segments (%d samples), one process each, rate per process" % (len(ref), n)}


def fft_round_trip_bytes(ns, sum_m, f):
    """Compulsory bytes of one forward + inverse FFT round trip over the set
    from per-sample input to per-sample output (the sweep's column and row
    passes): read the input, write and read the spectrum twice, write the output."""
    return 2 * ns * f + 8 * f * sum_m


def leg_roofline(nbytes, ms):
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "compulsory_gb": round(nbytes / 1e9, 3), "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def unit_template(ctx, ts, tod, out, maps32):
    import torch
    dev = tod.d.device
    t = torch.empty(ts.nsamp, dtype=torch.float32, device=dev)
    ones = torch.ones(ts.nseg, dtype=torch.float64, device=dev)
    ctx.project_sky(tod, "mixed", out["pix"], out["psi"], maps32, t, gain=ones)
    return t


def timed_call(ctx, fn):
    """One warm-up call, one timed call with HIP events around every launch:
    (ms, {kernel: (ms, launches)})."""
    fn()
    ctx.sync()
    ctx.enable_timing(True)
    ctx.kernel_times()
    t0 = time.perf_counter()
    fn()
    ctx.sync()
    ms = (time.perf_counter() - t0) * 1e3
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    return ms, kt


def noise_leg(ctx, ts, tod, out, t, seed):
    """The noise-parameter draw over the whole workload from the sweep's last
    n_corr; error against the oracle (fed its own n_corr of that iteration)
    on the sampled segments."""
    import numpy as np
    import torch
    dev = tod.d.device
    s0, fk, al = (torch.empty(ts.nseg, dtype=torch.float64, device=dev) for _ in range(3))
    ms, kt = timed_call(ctx, lambda: ctx.sample_noise(tod, "mixed", tod.d, t, out["ncorr"], seed, NOISE_IT,
                                                      s0, fk, al))
    xi = np.stack([s0.cpu().numpy(), fk.cpu().numpy(), al.cpu().numpy()])
    truth = np.stack([ts.sigma0, ts.fknee, ts.alpha])
    rep = {"ms_per_call": round(ms, 2), "samples_per_s": ts.nsamp / (ms / 1e3),
           "kernels_ms": {k: round(v[0], 2) for k, v in kt.items() if v[1]},
           "launches": {k: v[1] for k, v in kt.items() if v[1]},
           "draw_vs_generator_median_rel": [float(np.median(np.abs(xi[i] / truth[i] - 1))) for i in range(3)]}
    ref = _BASE.get("next")
    if ref:
        rep["vs_oracle_with_its_own_ncorr"] = [
            {"segment": q, "rel_err": [float(abs(xi[i, q] / x[i] - 1)) for i in range(3)]}
            for q, _, _, _, _, x, *_ in ref]
    # compulsory: forward column pass (n_corr read, spectrum written), row
    # pass (spectrum read), white sums (d, t, n_corr read)
    sum_m = sum(next5(int(x)) for x in np.diff(ts.seg_off))
    rep["roofline"] = leg_roofline(4 * ts.nsamp + 8 * sum_m + 8 * sum_m + 12 * ts.nsamp, ms)
    rep["cpu_baseline"] = oracle_rate("noise")
    log("noise draw: %.1f ms per call" % ms)
    return rep


def chisq_leg(ctx, ts, tod, out, maps32):
    """tod_chisq and tod_chisq_backward over the whole workload at the sweep's
    last n_corr; J and dJ/dg against the oracle (fed its own
    n_corr of that iteration) on the sampled segments."""
    import numpy as np
    import torch
    dev = tod.d.device
    J = torch.empty(ts.nseg, dtype=torch.float64, device=dev)
    ms_f, kt_f = timed_call(ctx, lambda: ctx.tod_chisq(tod, "mixed", out["pix"], out["psi"], tod.d,
                                                       out["ncorr"], maps32, J))
    gm = torch.empty((3, ts.npix_total), dtype=torch.float64, device=dev)
    gg = torch.empty(ts.nseg, dtype=torch.float64, device=dev)
    gs, gf, ga = (torch.empty(ts.ndet, dtype=torch.float64, device=dev) for _ in range(3))
    ms_b, kt_b = timed_call(ctx, lambda: ctx.tod_chisq_backward(tod, "mixed", out["pix"], out["psi"], tod.d,
                                                                out["ncorr"], maps32, 1.0, gm, gg, gs, gf, ga))
    rep = {"forward_ms_per_call": round(ms_f, 2), "backward_ms_per_call": round(ms_b, 2),
           "forward_samples_per_s": ts.nsamp / (ms_f / 1e3), "backward_samples_per_s": ts.nsamp / (ms_b / 1e3),
           "forward_kernels_ms": {k: round(v[0], 2) for k, v in kt_f.items() if v[1]},
           "backward_kernels_ms": {k: round(v[0], 2) for k, v in kt_b.items() if v[1]},
           "grad_maps_finite": bool(torch.isfinite(gm).all().item())}
    ref = _BASE.get("next")
    if ref:
        Jh, gh = J.cpu().numpy(), gg.cpu().numpy()
        acc = []
        for q, *_, chi in ref:
            Jr, J_terms, dgr, dg_terms = chi
            acc.append({"segment": q, "J_err_over_terms": float(abs(Jh[q] - Jr) / J_terms),
                        "dJdg_err_over_terms": float(abs(gh[q] - dgr) / dg_terms)})
        rep["accuracy_vs_oracle"] = acc
    # compulsory: pix, psi, d, n_corr read once per sample; the FP32 map read
    # once; the n_corr spectrum written and read once; backward adds the FP64
    # map gradient written once
    sum_m = sum(next5(int(x)) for x in np.diff(ts.seg_off))
    fwd = 14 * ts.nsamp + 12 * ts.npix_total + 16 * sum_m
    rep["forward_roofline"] = leg_roofline(fwd, ms_f)
    rep["backward_roofline"] = leg_roofline(fwd + 24 * ts.npix_total, ms_b)
    rep["cpu_baseline"] = oracle_rate("chisq")
    log("chisq: forward %.1f ms, backward %.1f ms per call" % (ms_f, ms_b))
    return rep


def gain_leg(ctx, ts, tod, seed, t):
    """The gain draw over the whole workload against the unit-gain sky
    template t; error against the oracle on the sampled segments."""
    import numpy as np
    import torch
    dev = tod.d.device
    g = torch.empty(ts.nseg, dtype=torch.float64, device=dev)
    sg = torch.empty(ts.nseg, dtype=torch.float64, device=dev)
    ms, kt = timed_call(ctx, lambda: ctx.sample_gain(tod, "mixed", tod.d, t, seed, GAIN_IT, g, sg))
    gh, sh = g.cpu().numpy(), sg.cpu().numpy()
    z = (gh - ts.gain) / sh
    rep = {"ms_per_call": round(ms, 2), "samples_per_s": ts.nsamp / (ms / 1e3),
           "kernels_ms": {k: round(v[0], 2) for k, v in kt.items() if v[1]},
           "launches": {k: v[1] for k, v in kt.items() if v[1]},
           "sigma_g": {"min": float(sh.min()), "max": float(sh.max())},
           "draw_minus_true_over_sigma": {"mean": float(z.mean()), "std": float(z.std())}}
    ref = _BASE.get("next")
    if ref:
        rep["accuracy_vs_oracle"] = [{"segment": q, "gain_rel_err": float(abs(gh[q] - gr) / abs(gr)),
                                      "sigma_rel_err": float(abs(sh[q] - sr) / sr)}
                                     for q, _, _, gr, sr, *_ in ref]
    # compulsory: two FFT round trips (t and d filtered), then t, Kt, Kd read
    sum_m = sum(next5(int(x)) for x in np.diff(ts.seg_off))
    rep["roofline"] = leg_roofline(2 * fft_round_trip_bytes(ts.nsamp, sum_m, 4) + 12 * ts.nsamp, ms)
    rep["cpu_baseline"] = oracle_rate("gain")
    log("gain draw: %.1f ms per call" % ms)
    return rep


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--nscan", type=int, default=None, help="fewer scans (quick runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cache-dir", default=None, help="reuse generated inputs saved here")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-masked", action="store_true", help="skip the masked n_corr draw leg")
    ap.add_argument("--no-gain", action="store_true", help="skip the gain draw leg")
    ap.add_argument("--no-noise", action="store_true", help="skip the noise-parameter draw leg")
    ap.add_argument("--no-chisq", action="store_true", help="skip the chi^2 forward/backward leg")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the sweep: no stream, gain, noise or masked-draw legs (profiling runs)")
    ap.add_argument("--fft-batch", type=int, default=None,
                    help="complex elements per FFT batch (0 = all segments at once)")
    ap.add_argument("--bin-stride", type=int, default=None, help="override the binning stride")
    ap.add_argument("--bin-runs", type=int, default=None,
                    help="scans per binning run (0 = chosen per layout)")
    ap.add_argument("--chunk-len", type=int, default=None,
                    help="Huffman side-index spacing of the generated inputs (symbols)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.sweep_only:
        args.no_gain = args.no_noise = args.no_masked = args.no_chisq = True
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2201_03509_amd import ops

    t0 = time.perf_counter()
    ts = synth.make_cached(args.config, cache_dir=args.cache_dir, nscan=args.nscan,
                           chunk_len=args.chunk_len, tod_streams=True)
    log("generated config %d: %d segments, %d samples in %.1fs" %
        (args.config, ts.nseg, ts.nsamp, time.perf_counter() - t0))
    seed = synth.seed32(args.config)
    last_it = args.warmup + args.steps - 1
    maps32_h = ts.maps.astype(np.float32)
    cpu, oracle_res = None, None
    if not args.no_cpu_baseline:
        c0 = time.perf_counter()
        cpu, oracle_res = cpu_baseline(ts, seed, last_it, maps32_h.astype(np.float64))
        log("cpu baseline %.3e samples/s on %d cores (%.1fs)" %
            (cpu["value"], cpu["cores"], time.perf_counter() - c0))
    dev = torch.device("cuda:0")
    ctx = ops.Context(0)
    if args.fft_batch is not None:
        ctx.set_fft_batch(args.fft_batch)
    tod = ops.DeviceTod(ts, dev)
    maps32 = torch.from_numpy(maps32_h).to(dev)
    maps64 = torch.from_numpy(ts.maps).to(dev)
    out = ops.new_outputs(tod, "mixed")
    # plans: autotune FFT splits and the binning stride on the decoded pointing
    ctx.decode_pointing(tod, out["pix"], out["psi"])
    ctx.sync()
    t1 = time.perf_counter()
    tune_path = os.path.join(args.cache_dir or "/tmp", "c3tod_tune_%d.json" % os.getpid())
    ctx.autotune(tod, "mixed", out["pix"], cache_path=tune_path)
    log("autotuned mixed plans in %.1fs" % (time.perf_counter() - t1))
    tuned = json.load(open(tune_path))
    os.remove(tune_path)
    if args.bin_stride:
        for b in range(ts.nband):
            ctx.set_bin_stride(b, args.bin_stride)
    if args.bin_runs is not None:
        ctx.set_bin_runs(args.bin_runs)
    plans = {}
    for e in tuned.get("fft", []):
        if e["mixed"] == 1:
            k = "%dx%d/B%d" % (e["M1"], e["M2"], e["B"])
            plans[k] = plans.get(k, 0) + 1

    def sweeps(prec, maps, o, k, it0, graph=False):
        for i in range(k):
            ctx.tod_sweep(tod, prec, maps, seed, it0 + i, o["ncorr"], o["acc"], o["pix"], o["psi"],
                          use_graph=graph)

    # warm-up: the first sweep captures the sweep's kernels into a hipGraph
    sweeps("mixed", maps32, out, args.warmup, 0, graph=True)
    ctx.sync()
    # timed region: graph-replayed sweeps (one graph launch per sweep, seed
    # and iteration read from device memory), HIP events on the context stream
    st = ctx.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    sweeps("mixed", maps32, out, args.steps, args.warmup, graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    ctx.sync()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = ts.nsamp * args.steps / (ms_total / 1e3)
    log("mixed, graph-replayed: %.3f ms/step, %.3e samples/s" % (ms_step, value))

    # per-kernel durations: the same sweeps eager, HIP events around every kernel
    ctx.enable_timing(True)
    ctx.kernel_times()
    torch.cuda.synchronize()
    e0.record(st)
    sweeps("mixed", maps32, out, args.steps, args.warmup)
    e1.record(st)
    torch.cuda.synchronize()
    ctx.sync()
    ms_eager = e0.elapsed_time(e1) / args.steps
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    log("mixed eager (per-kernel events): %.3f ms/step" % ms_eager)
    # the same sweep with the TOD decoded from its compressed stream in the
    # sweep (tod_sweep_stream); its n_corr must equal the d-reading sweep's
    stream_sweep = None
    if tod.tod_huff is not None:
        dw = torch.empty(ts.nsamp, dtype=torch.float32, device=dev)
        os_ = ops.new_outputs(tod, "mixed")
        ctx.tod_sweep_stream(tod, "mixed", maps32, seed, last_it, os_["ncorr"], os_["acc"], os_["pix"],
                             os_["psi"], dw)
        ctx.sync()
        s0 = time.perf_counter()
        for i in range(args.steps):
            ctx.tod_sweep_stream(tod, "mixed", maps32, seed, args.warmup + i, os_["ncorr"], os_["acc"],
                                 os_["pix"], os_["psi"], dw)
        ctx.sync()
        ms_stream = (time.perf_counter() - s0) * 1e3 / args.steps
        tod_bytes = sum(getattr(ts.tod_huff, k).nbytes for k in ("words", "chunk_bit", "chunk_prev", "tables"))
        stream_sweep = {"ms_per_step": round(ms_stream, 3), "value": ts.nsamp / (ms_stream / 1e3),
                        "tod_compressed_bytes_per_sample": round(tod_bytes / ts.nsamp, 3)}
        log("sweep from the compressed TOD: %.3f ms/step" % ms_stream)
        del dw, os_
    # restore the eager last iteration's n_corr for the accuracy check
    sweeps("mixed", maps32, out, 1, last_it)
    ctx.sync()
    gpu_nc = out["ncorr"].cpu().numpy()
    gpu_pix = out["pix"].cpu().numpy()
    # binning and solve of the oracle's sampled segments alone (accept flags)
    map_report = None
    if oracle_res:
        keep = np.zeros(ts.nseg, dtype=np.uint8)
        keep[[r[0] for r in oracle_res]] = 1
        acc_keep = tod.seg_accept.clone()
        tod.seg_accept.copy_(torch.from_numpy(keep))
        ctx.bin_tod(tod, "mixed", out["pix"], out["psi"], tod.d, out["ncorr"], out["acc"])
        gmap = torch.empty((3, ts.npix_total), dtype=torch.float32, device=dev)
        ctx.solve_maps(out["acc"], RCOND_MIN, gmap)
        ctx.sync()
        tod.seg_accept.copy_(acc_keep)
        map_report = compare_maps(oracle_res, out["acc"].cpu().numpy(), gmap.cpu().numpy().astype(np.float64),
                                  RCOND_MIN)
        del gmap

    sum_m = sum(next5(int(ts.seg_off[q + 1] - ts.seg_off[q])) for q in range(ts.nseg))
    kb = kernel_bytes(ts, tod, "mixed", sum_m)
    # a kernel may run as several launches per sweep (one per column length or
    # occupancy class); its time per sweep is the sum over them
    per = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
               "ms_per_launch": (v[0] / v[1]) if v[1] else None,
               "compulsory_gb_per_step": kb[k] / 1e9 if k in kb else None}
           for k, v in kt.items() if v[1]}
    dom = max(per, key=lambda k: kt[k][0])
    avg_ms = per[dom]["ms_per_step"]
    ach = kb[dom] / (avg_ms / 1e3) / 1e9
    workload = "lfi70" if args.config == 2 and args.nscan is None else "config%d_nscan%s" % (args.config, args.nscan)
    meas = measured_counters(dom, workload)
    traffic = meas.get("bytes_per_step")
    fl = row_pass_flops(ts, tuned) if dom in ALU_BOUND else None
    if fl is not None:
        tfs = fl / (avg_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(tfs, 2), "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfs / FP32_VALU_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": dom,
                "flops_per_step": fl, "valu_issue": meas.get("valu_issue"),
                "hbm_compulsory_gbs": round(ach, 1), "ms_per_step": round(avg_ms, 4),
                "launches_per_step": per[dom]["launches_per_step"]}
    else:
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_step": kb[dom], "ms_per_step": round(avg_ms, 4),
                "launches_per_step": per[dom]["launches_per_step"]}
    # fused-sweep minimum: the compressed pointing (words, side index, tables)
    # decoded twice, d read once, n_corr written once, map + accumulators once
    comp = sum(h.words.nbytes + h.chunk_bit.nbytes + h.chunk_prev.nbytes + h.tables.nbytes
               for h in (ts.pix_huff, ts.psi_huff))
    sweep_alg = 2 * comp + ts.nsamp * (4 + 4) + 84 * ts.npix_total
    log("dominant kernel %s: %.3f ms per sweep, %.0f GB/s compulsory, roofline %s %s %s of %s" % (
        dom, avg_ms, ach, roof["bound"], roof["achieved"], roof["unit"], roof["peak"]))

    plain = None
    if not args.no_plain:
        outp = ops.new_outputs(tod, "fp64")
        ctx.autotune(tod, "fp64", out["pix"])
        sweeps("fp64", maps64, outp, 1, 0)
        ctx.sync()
        p0 = time.perf_counter()
        ksteps = max(1, args.steps // 2)
        sweeps("fp64", maps64, outp, ksteps, 1)
        ctx.sync()
        ms_plain = (time.perf_counter() - p0) * 1e3 / ksteps
        plain = {"value": ts.nsamp / (ms_plain / 1e3), "ms_per_step": round(ms_plain, 3)}
        log("plain fp64: %.3f ms/step" % ms_plain)
        del outp
        torch.cuda.empty_cache()

    gain = noise = None
    if not (args.no_gain and args.no_noise):
        t_unit = unit_template(ctx, ts, tod, out, maps32)
        if not args.no_gain:
            gain = gain_leg(ctx, ts, tod, seed, t_unit)
        if not args.no_noise:
            noise = noise_leg(ctx, ts, tod, out, t_unit, seed)
        del t_unit
        torch.cuda.empty_cache()

    chisq = None
    if not args.no_chisq:
        chisq = chisq_leg(ctx, ts, tod, out, maps32)
        torch.cuda.empty_cache()

    streams = masked = None
    if not args.sweep_only:
        streams, flag_mask = stream_leg(ctx, ts, tod)
        if not args.no_masked:
            masked = masked_leg(ctx, ts, tod, out, maps32, seed, gpu_pix, flag_mask)
        del flag_mask
        torch.cuda.empty_cache()

    copy = None
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        copy = {"bytes": 2 * a.numel() * 4}

    acc_report = compare_to_oracle(ts, oracle_res, gpu_nc, gpu_pix) if oracle_res else None
    if acc_report is not None:
        acc_report["binned_and_maps"] = map_report

    line = {
        "metric": "TOD samples/s (decode+project+n_corr+bin), mixed-FP32 vs FP64 plain, 1 GPU",
        "value": value,
        "unit": "TOD samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "nside": [int(x) for x in ts.band_nside],
                   "segments": ts.nseg, "samples": ts.nsamp,
                   "precision": "FP32 projection/FFT/draws, FP64 pixel accumulation",
                   "fft_padding": "even 5-smooth >= 2n",
                   "huffman_chunk_len": int(ts.pix_huff.chunk_len)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "eager_ms_per_step": round(ms_eager, 3),
        "sweep_from_compressed_tod": stream_sweep,
        "plain_fp64": plain,
        "sweep_algorithmic_gb": round(sweep_alg / 1e9, 3),
        "sweep_algorithmic_frac": round(sweep_alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "sweep_counter_traffic": sweep_counters(workload, ms_step),
        "kernels": per,
        "fft_splits": plans,
        "bin_stride": tuned.get("bin_stride"),
        "accuracy_vs_oracle": acc_report,
        "tod_flag_streams": streams,
        "gain_draw": gain,
        "noise_draw": noise,
        "chisq": chisq,
        "masked_ncorr": masked,
        "copy_probe": copy,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
