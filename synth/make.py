"""Seeded synthetic TOD sets (inputs only: no step of the sampler lives here).

Recipe (each item is a generator choice, fixed so results are reproducible):

* seeds: ``SeedSequence([2201, 3509, config, stream, ...])`` with streams
  sky=0, gain=1, noise params=2, lengths=3, psi=4, white=5, true n_corr=6;
* sky per band: T ~ N(0,100^2), Q,U ~ N(0,10^2) i.i.d. per pixel;
* scan law: spin axis on the ecliptic advancing 1 deg/day, boresight at 85 deg
  from it (plus 0.5 deg per horn step), spinning at 1 rpm; horns hold two
  radiometers with identical pointing; HEALPix RING pixel per sample;
* psi: i.i.d. uniform bin in [0, 4096) per sample and detector; the bin centre
  2*pi*(b+1/2)/4096 is the angle the data were simulated with;
* gain 1 + 0.01 N(0,1) per segment; sigma0 = 1; f_knee, alpha per detector;
* correlated noise: Gaussian with PSD sigma0^2 (f/f_knee)^alpha drawn on a
  periodic grid and truncated to the segment, zero mean; white noise N(0, sigma0^2);
* d = g * (T + Re[(Q - iU) exp(2i psi)]) + n_corr + n_w, quantised to integer
  multiples of TOD_QUANTUM (the ADC step: the paper's TOD are integers) and
  stored FP64 or FP32 (exact: |d / TOD_QUANTUM| < 2^24);
* optional compressed TOD and flag streams (``tod_streams=True``): the
  integer TOD and a flag word per sample (bit 0: processing mask, the pixel
  centre within 10 deg of the map frame's equator; bit 1: isolated glitches,
  probability 1e-4 per sample, stream 7), differenced and Huffman coded per
  scan exactly like the pointing streams.

A *segment* is one (scan, detector) pair; segments are ordered band, scan,
detector, and all per-sample arrays are flat with ``seg_off`` offsets.
"""
import os
import multiprocessing as mp
import numpy as np
import scipy.fft

from . import configs as cfgmod
from . import healpix
from . import huffman_enc as H

NPSI = 4096
TOD_QUANTUM = 0.125        # ADC step of the stored TOD (sigma0 / 8)
FLAG_PLANE = 1             # flag bits
FLAG_GLITCH = 2
OPENING_DEG = 85.0
HORN_STEP_DEG = 0.5
SPIN_PERIOD_S = 60.0
PRECESS_DEG_PER_DAY = 1.0


def _ss(k, *stream):
    return np.random.SeedSequence([2201, 3509, int(k)] + [int(s) for s in stream])


def _rng(k, *stream):
    return np.random.default_rng(_ss(k, *stream))


def scan_pointing(nside, t, horn_offset_deg):
    """HEALPix pixel of the boresight at times t (seconds)."""
    lam = np.deg2rad(PRECESS_DEG_PER_DAY) * t / 86400.0
    ax, ay = np.cos(lam), np.sin(lam)
    ux, uy = np.sin(lam), -np.cos(lam)               # unit a x z
    beta = np.deg2rad(OPENING_DEG + horn_offset_deg)
    om = 2.0 * np.pi * t / SPIN_PERIOD_S
    c, s = np.cos(om), np.sin(om)
    cb, sb = np.cos(beta), np.sin(beta)
    bx = cb * ax + sb * s * ux
    by = cb * ay + sb * s * uy
    bz = sb * c
    theta = np.arccos(np.clip(bz, -1.0, 1.0))
    phi = np.arctan2(by, bx)
    return healpix.ang2pix_ring(nside, theta, phi)


def _lengths(cfg):
    r = _rng(cfg.index, 3)
    if cfg.length[0] == "list":  # ("list", n_0, n_1, ...): given lengths, repeated over the scans
        ns = np.asarray(cfg.length[1:], dtype=np.int64)
        return ns[np.arange(cfg.nscan) % len(ns)]
    kind, a, b = cfg.length
    if kind == "uniform":
        return r.integers(int(a), int(b) + 1, size=cfg.nscan).astype(np.int64)
    u = r.random(cfg.nscan)
    return np.floor(2.0 ** (a + (b - a) * u)).astype(np.int64)


def _band_of_scan(cfg):
    nb = len(cfg.bands)
    return np.arange(cfg.nscan) % nb


def _sky(cfg, b, npix):
    r = _rng(cfg.index, 0, b)
    m = np.empty((3, npix))
    m[0] = r.normal(0.0, 100.0, npix)
    m[1] = r.normal(0.0, 10.0, npix)
    m[2] = r.normal(0.0, 10.0, npix)
    return m


def _corr_noise(rng, n, fsamp, sigma0, fknee, alpha):
    if n == 0:
        return np.zeros(0)
    ngrid = scipy.fft.next_fast_len(2 * n, real=True)
    nk = ngrid // 2 + 1
    f = np.arange(nk) * fsamp / ngrid
    P = np.zeros(nk)
    P[1:] = sigma0 ** 2 * (f[1:] / fknee) ** alpha
    X = (rng.normal(size=nk) + 1j * rng.normal(size=nk)) * np.sqrt(P / 2.0)
    X[0] = 0.0
    if ngrid % 2 == 0:
        X[-1] = rng.normal() * np.sqrt(P[-1])
    x = scipy.fft.irfft(X, n=ngrid) * np.sqrt(ngrid)
    return x[:n]


_G = {}


def _scan_worker(args):
    (k, g_scan, b, n, t0, seg0, det0) = args
    cfg = _G["cfg"]
    band = cfg.bands[b]
    sky = _G["sky"][b]
    gains = _G["gain"]
    sig0, fkn, alp = _G["sigma0"], _G["fknee"], _G["alpha"]
    nd = band.ndet
    nh = max(1, nd // 2)
    t = t0 + np.arange(n) / band.fsamp
    horn_pix = [scan_pointing(band.nside, t, HORN_STEP_DEG * (h - (nh - 1) / 2.0))
                for h in range(nh)]
    pix, psi = [], []
    for j in range(nd):
        pix.append(horn_pix[min(j // 2, nh - 1)])
        psi.append(_rng(k, 4, g_scan, j).integers(0, NPSI, size=n))
    out = {"streams": {}}
    for name, vals in (("pix", pix), ("psi", psi)):
        diffs = [H.difference(v) for v in vals]
        blob, lookup = H.build_table(np.concatenate(diffs))
        segs = []
        for j in range(nd):
            words, pos = H.encode_values(diffs[j], lookup)
            cb, cp = H.chunk_index(vals[j], pos, cfg.chunk_len)
            segs.append((words, cb, cp))
        out["streams"][name] = (blob, segs)
    dd, di = [], []
    for j in range(nd):
        seg = seg0 + j
        det = det0 + j
        ang = 2.0 * np.pi * (psi[j] + 0.5) / NPSI
        p = pix[j]
        sig = sky[0, p] + np.real((sky[1, p] - 1j * sky[2, p]) * np.exp(2j * ang))
        nc = _corr_noise(_rng(k, 6, g_scan, j), n, band.fsamp, sig0[det], fkn[det], alp[det])
        nw = _rng(k, 5, g_scan, j).normal(0.0, sig0[det], size=n)
        x = np.rint((gains[seg] * sig + nc + nw) / TOD_QUANTUM).astype(np.int64)
        di.append(x)
        dd.append(x * TOD_QUANTUM)
    out["d"] = dd
    if _G["tod_streams"]:
        horn_flag = [FLAG_PLANE * (1 - plane_mask_pixels(band.nside, hp)).astype(np.int64) for hp in horn_pix]
        flags = []
        for j in range(nd):
            fl = horn_flag[min(j // 2, nh - 1)].copy()
            fl |= FLAG_GLITCH * (_rng(k, 7, g_scan, j).random(n) < 1e-4)
            flags.append(fl)
        for name, vals in (("tod", di), ("flag", flags)):
            diffs = [H.difference(v) for v in vals]
            blob, lookup = H.build_table(np.concatenate(diffs))
            segs = []
            for j in range(nd):
                words, pos = H.encode_values(diffs[j], lookup)
                cb, cp = H.chunk_index(vals[j], pos, cfg.chunk_len)
                segs.append((words, cb, cp))
            out["streams"][name] = (blob, segs)
    if _G["keep_truth"]:
        out["pix"] = [p.astype(np.int32) for p in pix]
        out["psi"] = [p.astype(np.uint16) for p in psi]
    return out


class HuffStream:
    """Concatenated Huffman stream of one kind over all segments."""

    def __init__(self, chunk_len):
        self.chunk_len = int(chunk_len)
        self.words = None          # uint32 [nwords]
        self.seg_word_off = None   # int64 [nseg+1]
        self.seg_table = None      # int32 [nseg]
        self.tables = None         # uint32 [sum of blobs]
        self.table_off = None      # int64 [ntable+1]
        self.chunk_bit = None      # uint32 [nchunk]
        self.chunk_prev = None     # int32 [nchunk]
        self.seg_chunk_off = None  # int64 [nseg+1]

    @property
    def nbytes(self):
        return int(self.words.nbytes + self.chunk_bit.nbytes + self.chunk_prev.nbytes)


class TodSet:
    """A synthetic TOD set; every array is a numpy array on the host."""


def make(k, nscan=None, length=None, workers=None, keep_truth=False, bands=None, chunk_len=None,
         tod_streams=False):
    cfg = cfgmod.get(k).scaled(nscan=nscan, length=length, bands=bands, chunk_len=chunk_len)
    kk = cfg.index
    nb = len(cfg.bands)
    lengths = _lengths(cfg)
    band_of = _band_of_scan(cfg)
    npix = [healpix.npix_of(b.nside) for b in cfg.bands]
    pix_off = np.concatenate([[0], np.cumsum(npix)]).astype(np.int64)
    det_off = np.concatenate([[0], np.cumsum([b.ndet for b in cfg.bands])]).astype(np.int64)
    ndet_tot = int(det_off[-1])

    # segment table: band-major, then scan, then detector
    scan_order = []
    for b in range(nb):
        scan_order += [s for s in range(cfg.nscan) if band_of[s] == b]
    seg_scan, seg_det, seg_band, seg_len = [], [], [], []
    jobs = []
    t_band = [0.0] * nb
    seg = 0
    for s in scan_order:
        b = int(band_of[s])
        n = int(lengths[s])
        jobs.append((kk, s, b, n, t_band[b], seg, int(det_off[b])))
        t_band[b] += n / cfg.bands[b].fsamp
        for j in range(cfg.bands[b].ndet):
            seg_scan.append(s)
            seg_det.append(int(det_off[b]) + j)
            seg_band.append(b)
            seg_len.append(n)
            seg += 1
    nseg = seg
    seg_off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(seg_len, out=seg_off[1:])

    rg = _rng(kk, 1)
    gain = 1.0 + 0.01 * rg.normal(size=nseg)
    rn = _rng(kk, 2)
    sigma0_det = np.ones(ndet_tot)
    if cfg.fknee_fixed > 0:
        fknee_det = np.full(ndet_tot, cfg.fknee_fixed)
        alpha_det = np.full(ndet_tot, cfg.alpha_fixed)
    else:
        fknee_det = rn.uniform(*cfg.fknee_range, size=ndet_tot)
        alpha_det = rn.uniform(*cfg.alpha_range, size=ndet_tot)

    sky = [_sky(cfg, b, npix[b]) for b in range(nb)]
    _G.clear()
    _G.update(cfg=cfg, sky=sky, gain=gain, sigma0=sigma0_det, fknee=fknee_det,
              alpha=alpha_det, keep_truth=keep_truth, tod_streams=tod_streams)
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if len(jobs) > 8 else 1
    import sys
    import time
    t0 = time.time()
    verbose = len(jobs) >= 100
    if workers > 1:
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            res = []
            for r in pool.imap(_scan_worker, jobs, chunksize=1):
                res.append(r)
                if verbose and len(res) % 25 == 0:
                    print("  generated %d/%d scans (%.0fs)" % (len(res), len(jobs), time.time() - t0),
                          file=sys.stderr, flush=True)
    else:
        res = [_scan_worker(j) for j in jobs]
    _G.clear()

    ts = TodSet()
    ts.cfg = cfg
    ts.config = kk
    ts.nseg = nseg
    ts.nband = nb
    ts.ndet = ndet_tot
    ts.nsamp = int(seg_off[-1])
    ts.seg_off = seg_off
    ts.seg_scan = np.array(seg_scan, dtype=np.int32)
    ts.seg_det = np.array(seg_det, dtype=np.int32)
    ts.seg_band = np.array(seg_band, dtype=np.int32)
    ts.seg_accept = np.ones(nseg, dtype=np.uint8)
    ts.band_nside = np.array([b.nside for b in cfg.bands], dtype=np.int32)
    ts.band_npix = np.array(npix, dtype=np.int64)
    ts.band_pix_off = pix_off[:-1].copy()
    ts.npix_total = int(pix_off[-1])
    ts.band_fsamp = np.array([b.fsamp for b in cfg.bands], dtype=np.float64)
    ts.gain = gain
    ts.sigma0 = sigma0_det[ts.seg_det]
    ts.fknee = fknee_det[ts.seg_det]
    ts.alpha = alpha_det[ts.seg_det]
    ts.maps = np.concatenate(sky, axis=1)        # [3][npix_total] FP64 truth
    dt = np.float64 if cfg.tod_f64 else np.float32
    ts.d = np.concatenate([np.concatenate(r["d"]) for r in res]).astype(dt)
    ts.tod_quantum = TOD_QUANTUM
    for name in ("pix", "psi") + (("tod", "flag") if tod_streams else ()):
        hs = HuffStream(cfg.chunk_len)
        blobs, words, cbits, cprevs = [], [], [], []
        seg_table, wlen, clen = [], [], []
        for ti, r in enumerate(res):
            blob, segs = r["streams"][name]
            blobs.append(blob)
            for (w, cb, cp) in segs:
                words.append(w)
                cbits.append(cb)
                cprevs.append(cp)
                seg_table.append(ti)
                wlen.append(len(w))
                clen.append(len(cb))
        hs.words = np.concatenate(words).astype(np.uint32)
        hs.seg_word_off = np.concatenate([[0], np.cumsum(wlen)]).astype(np.int64)
        hs.seg_table = np.array(seg_table, dtype=np.int32)
        hs.tables = np.concatenate(blobs).astype(np.uint32)
        hs.table_off = np.concatenate([[0], np.cumsum([len(b) for b in blobs])]).astype(np.int64)
        hs.chunk_bit = np.concatenate(cbits).astype(np.uint32)
        hs.chunk_prev = np.concatenate(cprevs).astype(np.int32)
        hs.seg_chunk_off = np.concatenate([[0], np.cumsum(clen)]).astype(np.int64)
        setattr(ts, name + "_huff", hs)
    if keep_truth:
        ts.pix = np.concatenate([np.concatenate(r["pix"]) for r in res])
        ts.psi = np.concatenate([np.concatenate(r["psi"]) for r in res])
    return ts


def seed32(k):
    """Sampler seed of a configuration."""
    return (0x22013509 ^ int(k)) & 0xFFFFFFFF


_SCALARS = ("config", "nseg", "nband", "ndet", "nsamp", "npix_total")


def save(ts, path):
    """Write a TOD set as .npy files plus a small JSON of scalars."""
    import json
    os.makedirs(path, exist_ok=True)
    meta = {k: int(getattr(ts, k)) for k in _SCALARS}
    meta["cfg"] = [ts.cfg.index, ts.cfg.nscan, list(ts.cfg.length)]
    meta["chunk_len"] = ts.pix_huff.chunk_len
    meta["tod_quantum"] = ts.tod_quantum
    names = [n for n in ("pix_huff", "psi_huff", "tod_huff", "flag_huff") if hasattr(ts, n)]
    meta["streams"] = names
    for k, v in vars(ts).items():
        if isinstance(v, np.ndarray):
            np.save(os.path.join(path, k + ".npy"), v)
    for name in names:
        for k, v in vars(getattr(ts, name)).items():
            if isinstance(v, np.ndarray):
                np.save(os.path.join(path, name + "." + k + ".npy"), v)
    with open(os.path.join(path, "meta.json"), "w") as f:
        json.dump(meta, f)


def load(path):
    import json
    meta = json.load(open(os.path.join(path, "meta.json")))
    ts = TodSet()
    for k in _SCALARS:
        setattr(ts, k, meta[k])
    idx, nscan, length = meta["cfg"]
    ts.cfg = cfgmod.get(idx).scaled(nscan=nscan, length=length, chunk_len=meta["chunk_len"])
    ts.tod_quantum = meta["tod_quantum"]
    hs = {n: HuffStream(meta["chunk_len"]) for n in meta["streams"]}
    for f in sorted(os.listdir(path)):
        if not f.endswith(".npy"):
            continue
        arr = np.load(os.path.join(path, f))
        key = f[:-4]
        if "." in key:
            a, b = key.split(".", 1)
            setattr(hs[a], b, arr)
        else:
            setattr(ts, key, arr)
    for n, h in hs.items():
        setattr(ts, n, h)
    return ts


def make_cached(k, cache_dir=None, **kw):
    """make(), reusing a copy saved under cache_dir when one exists."""
    if not cache_dir:
        return make(k, **kw)
    tag = "c%d_n%s_l%s_q" % (k, kw.get("nscan"), "_".join(map(str, kw.get("length") or [])))
    if kw.get("chunk_len"):
        tag += "_c%d" % kw["chunk_len"]
    if kw.get("tod_streams"):
        tag += "_t"
    path = os.path.join(cache_dir, tag)
    if os.path.exists(os.path.join(path, "meta.json")):
        return load(path)
    ts = make(k, **kw)
    save(ts, path)
    return ts


def plane_mask(ts, pix, half_width_deg=10.0):
    """Processing mask (uint8, 1 = usable) that removes every sample whose
    pixel centre lies within half_width_deg of the map frame's equator: a
    stand-in for a Galactic-plane mask, crossed twice per spin period in long
    contiguous gaps."""
    out = np.ones(ts.nsamp, dtype=np.uint8)
    table = {}  # per nside: the mask of every pixel centre
    for q in range(ts.nseg):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        if b == a:
            continue
        nside = int(ts.band_nside[ts.seg_band[q]])
        if nside not in table:
            table[nside] = plane_mask_pixels(nside, np.arange(12 * nside * nside), half_width_deg)
        out[a:b] = table[nside][np.asarray(pix[a:b], dtype=np.int64)]
    return out


def plane_mask_pixels(nside, pix, half_width_deg=10.0):
    """The same mask for a list of RING pixels of one nside."""
    theta, _ = healpix.pix2ang_ring(nside, np.asarray(pix, dtype=np.int64))
    return (np.abs(np.cos(theta)) >= np.sin(np.radians(half_width_deg))).astype(np.uint8)
