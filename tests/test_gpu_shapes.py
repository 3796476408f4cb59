"""Parity at the workloads' real segment shapes, through the C-ABI.

* 70 GHz-like shape: nside 1024, 12 detectors, two scans of 230k-290k
  samples at 78.8 Hz (24 segments).  The FFT splits are autotuned, as in the
  benchmark, so the column lengths M1 in 50..100 and the compiled row
  lengths (2430..4096 on the full set) run here: decode bit-exact, n_corr of the
  fused sweep (eager and graph-replayed) and of sample_ncorr within 1e-5 per
  segment, b and A of the sweep's binning within 1e-12 of the oracle's.
* 30 GHz-like shape at full length (the differentiation workload): nside
  512, 4 detectors, two scans of 100k-130k samples.  chi^2 per segment, the
  adjoint per pixel and per detector against the oracle's analytic
  gradients, and FP64 central differences (h = 1e-6) through the autograd
  wrapper for the gain, sigma0, f_knee, alpha and four random map directions.

Error bounds for sums of terms of both signs (J, dJ/dg, the noise-parameter
and map gradients) are relative to the sum of the terms' magnitudes, the
scale the rounding of any summation order is proportional to.  The Whittle
terms of J and the noise-parameter gradients add the transform's own error:
a stable FFT of length N leaves each unitary mode E_k an absolute error of
about delta = 4 eps log2(N) rms(e) (eps of the transform's type), so
I_k / P_k = |E_k|^2 / P_k moves by up to (2 sqrt(I_k) delta + delta^2) / P_k.
On the FP32 path that dominates at high frequencies, where a red spectrum
leaves |E_k| far below rms(e).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import huffman as oh
from oracle import tod as ot
from chisq_bounds import magnitudes as _magnitudes

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}


def seg_errs(ts, got, ref):
    out = []
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        out.append(np.linalg.norm(got[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]))
    return np.asarray(out)


@pytest.fixture(scope="module")
def lfi70():
    ts = synth.make(2, nscan=2, keep_truth=True)
    pix, psi = oh.decode_pointing(ts)
    assert np.array_equal(pix, ts.pix) and np.array_equal(psi, ts.psi)
    return ts


def test_lfi70_shape_autotuned(lfi70, tmp_path):
    from paper_2201_03509_amd import ops
    import json
    ts = lfi70
    seed = synth.seed32(2)
    m32 = ts.maps.astype(np.float32)
    c = ops.Context(0)
    try:
        tod = ops.DeviceTod(ts, "cuda:0")
        out = ops.new_outputs(tod, "mixed")
        c.decode_pointing(tod, out["pix"], out["psi"])
        c.sync()
        assert np.array_equal(out["pix"].cpu().numpy(), ts.pix)
        assert np.array_equal(out["psi"].cpu().numpy().astype(np.int64), ts.psi)
        path = tmp_path / "tune.json"
        c.autotune(tod, "mixed", out["pix"], cache_path=str(path))
        plans = [e for e in json.loads(path.read_text())["fft"] if e["mixed"] == 1]
        print("autotuned splits:", sorted({(e["M1"], e["M2"]) for e in plans}))
        assert all(e["colreg"] == 1 and 50 <= e["M1"] <= 100 for e in plans)
        maps = torch.from_numpy(m32).cuda()
        c.set_bin_runs(2)  # binning walks both scans of a detector pair per run
        c.tod_sweep(tod, "mixed", maps, seed, 4, out["ncorr"], out["acc"], out["pix"], out["psi"])
        c.sync()
        nc_e = out["ncorr"].cpu().numpy().astype(np.float64)
        acc = out["acc"].cpu().numpy()
        og_ = ops.new_outputs(tod, "mixed")
        for it in (3, 4):   # capture, then replay with the iteration of the eager sweep
            c.tod_sweep(tod, "mixed", maps, seed, it, og_["ncorr"], og_["acc"], og_["pix"], og_["psi"],
                        use_graph=True)
        c.sync()
        assert np.array_equal(og_["ncorr"].cpu().numpy().astype(np.float64), nc_e)
        # the standalone draw on the same residual inputs (d and s in FP32)
        s = ot.project_all(ts, m32.astype(np.float64), ts.pix, ts.psi)
        s32 = s.astype(np.float32)
        nc_s = torch.empty(ts.nsamp, dtype=torch.float32, device="cuda")
        c.sample_ncorr(tod, "mixed", tod.d, torch.from_numpy(s32).cuda(), seed, 9, nc_s)
        c.sync()
        nc_s = nc_s.cpu().numpy().astype(np.float64)
    finally:
        c.close()
    ref = ot.sample_ncorr_all(ts, ts.d, s, seed, 4)
    e = seg_errs(ts, nc_e, ref)
    print("sweep n_corr per segment rel L2: max %.2e median %.2e" % (e.max(), np.median(e)))
    assert e.max() < TOL["mixed"]
    ref_s = ot.sample_ncorr_all(ts, ts.d, s32.astype(np.float64), seed, 9)
    e = seg_errs(ts, nc_s, ref_s)
    print("sample_ncorr per segment rel L2: max %.2e" % e.max())
    assert e.max() < TOL["mixed"]
    b, A, hits = ot.bin_tod(ts, ts.pix, ts.psi, ts.d, nc_e)
    assert np.array_equal(acc[9], hits)
    assert np.abs(acc[0:3] - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(acc[3:9] - A).max() <= 1e-12 * np.abs(A).max()


@pytest.fixture(scope="module")
def lfi30():
    from paper_2201_03509_amd import ops
    ts = synth.make(1, nscan=2, keep_truth=True)
    rng = np.random.default_rng(30)
    ts.gain = 1.0 + 0.05 * rng.normal(size=ts.nseg)
    sig_det = rng.uniform(0.8, 1.5, ts.ndet)
    ts.sigma0 = sig_det[ts.seg_det]
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, 5, 0)
    maps = ts.maps + rng.normal(size=ts.maps.shape) * 0.5
    c = ops.Context(0)
    tod = ops.DeviceTod(ts, "cuda:0")
    yield ts, c, tod, nc, maps, sig_det
    c.close()


def _inputs(ts, prec, nc, maps):
    ft = np.float32 if prec == "mixed" else np.float64
    nc_h, m_h = nc.astype(ft), maps.astype(ft)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return (dev(ts.pix.astype(np.int32)), dev(ts.psi.astype(np.uint16)), dev(nc_h), dev(m_h),
            nc_h.astype(np.float64), m_h.astype(np.float64))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_lfi30_shape_chisq_and_adjoint(lfi30, prec):
    ts, c, tod, nc, maps, _ = lfi30
    pix, psi, ncd, md, nc_r, m_r = _inputs(ts, prec, nc, maps)
    J = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
    c.tod_chisq(tod, prec, pix, psi, tod.d, ncd, md, J)
    out = [torch.empty((3, ts.npix_total), dtype=torch.float64, device="cuda"),
           torch.empty(ts.nseg, dtype=torch.float64, device="cuda")] + \
          [torch.empty(ts.ndet, dtype=torch.float64, device="cuda") for _ in range(3)]
    c.tod_chisq_backward(tod, prec, pix, psi, tod.d, ncd, md, 1.0, *out)
    c.sync()
    J_ref = ot.chisq_all(ts, m_r, ts.pix, ts.psi, ts.d, nc_r)
    gm, gg, gs, gf, ga = ot.chisq_grad_all(ts, m_r, ts.pix, ts.psi, ts.d, nc_r)
    eps = float(np.finfo(np.float32 if prec == "mixed" else np.float64).eps)
    mag, fft, gmag = _magnitudes(ts, m_r, nc_r, eps)
    tol = TOL[prec]
    dJ = np.abs(J.cpu().numpy() - J_ref)
    print("J: max error / bound %.3f" % (dJ / (tol * mag[0] + fft[0])).max())
    assert np.all(dJ <= tol * mag[0] + fft[0])
    assert np.all(np.abs(out[1].cpu().numpy() - gg) <= tol * mag[1])
    # the map gradient pixel by pixel: both sides sum the same FP64 terms
    # (the mixed path's FP32 maps and n_corr enter both exactly), in any order
    g = out[0].cpu().numpy()
    hit = gmag > 0
    assert np.all(g[~hit] == 0.0)
    assert np.all(np.abs(g[hit] - gm[hit]) <= 1e-12 * gmag[hit])
    det = ts.seg_det
    for got, ref, k in zip(out[2:], (gs, gf, ga), (2, 3, 4)):
        r_det = np.bincount(det, weights=ref, minlength=ts.ndet)
        bound = np.bincount(det, weights=tol * mag[k] + fft[k], minlength=ts.ndet)
        err = np.abs(got.cpu().numpy() - r_det)
        print("noise gradient %d: max error / bound %.3f" % (k, (err / bound).max()))
        assert np.all(err <= bound), (k, got.cpu().numpy(), r_det)


def test_lfi30_shape_finite_differences(lfi30):
    """FP64 central differences (h = 1e-6) of the GPU objective vs the
    adjoint reached through TodChisq.backward (incoming gradient read on the
    device)."""
    from paper_2201_03509_amd.autograd import tod_chisq
    ts, c, tod, nc, maps, sig_det = lfi30
    pix, psi, ncd, md, nc_r, m_r = _inputs(ts, "fp64", nc, maps)
    dev = "cuda"
    first = [int(np.argmax(ts.seg_det == d)) for d in range(ts.ndet)]
    m = md.clone().requires_grad_(True)
    g = torch.from_numpy(ts.gain.copy()).to(dev).requires_grad_(True)
    s = torch.from_numpy(sig_det.copy()).to(dev).requires_grad_(True)
    f = torch.from_numpy(ts.fknee[first].copy()).to(dev).requires_grad_(True)
    a = torch.from_numpy(ts.alpha[first].copy()).to(dev).requires_grad_(True)
    J = tod_chisq(m, g, s, f, a, c, tod, "fp64", pix, psi, ncd)
    (3.0 * J).backward()     # a non-unit incoming gradient

    def Jat(**kw):
        args = dict(m=md, g=g.detach(), s=s.detach(), f=f.detach(), a=a.detach())
        args.update(kw)
        with torch.no_grad():
            return 3.0 * float(tod_chisq(args["m"], args["g"], args["s"], args["f"], args["a"], c, tod,
                                         "fp64", pix, psi, ncd))

    h = 1e-6
    for name, t, grad in (("g", g, g.grad), ("s", s, s.grad), ("f", f, f.grad), ("a", a, a.grad)):
        for i in sorted({0, t.numel() - 1}):
            tp, tm = t.detach().clone(), t.detach().clone()
            tp[i] += h
            tm[i] -= h
            fd = (Jat(**{name: tp}) - Jat(**{name: tm})) / (2 * h)
            assert abs(fd - float(grad[i])) <= 1e-5 * max(1.0, abs(fd)), (name, i, fd, float(grad[i]))
    rng = np.random.default_rng(3)
    for _ in range(4):
        v = torch.from_numpy(rng.normal(size=md.shape)).to(dev)
        fd = (Jat(m=md + h * v) - Jat(m=md - h * v)) / (2 * h)
        an = float((m.grad * v).sum())
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd)), (fd, an)
