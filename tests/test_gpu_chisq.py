"""chi^2 forward and hand-written adjoint on the GPU vs the oracle, plus
finite-difference checks of the torch.autograd wrapper in FP64."""
import numpy as np
import pytest
import torch

import synth
from oracle import tod as ot
from chisq_bounds import magnitudes

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}


@pytest.fixture(scope="module")
def setup():
    from paper_2201_03509_amd import ops
    ts = synth.make(1, nscan=2, length=("uniform", 6000, 9000), keep_truth=True)
    rng = np.random.default_rng(8)
    ts.gain = 1.0 + 0.05 * rng.normal(size=ts.nseg)
    sig_det = rng.uniform(0.8, 1.5, ts.ndet)
    ts.sigma0 = sig_det[ts.seg_det]
    c = ops.Context(0)
    tod = ops.DeviceTod(ts, "cuda:0")
    # n_corr: the oracle's mean-only draw on this data (any fixed n_corr would do)
    s = ot.project_all(ts, ts.maps, ts.pix, ts.psi)
    nc = ot.sample_ncorr_all(ts, ts.d, s, 5, 0, mean_only=True)
    maps = ts.maps + rng.normal(size=ts.maps.shape) * 0.5
    yield ts, c, tod, nc, maps, sig_det
    c.close()


def _dev(ts, prec, nc, maps):
    ft = np.float32 if prec == "mixed" else np.float64
    nc_h = nc.astype(ft)
    m_h = maps.astype(ft)
    pix = torch.from_numpy(ts.pix.astype(np.int32)).cuda()
    psi = torch.from_numpy(ts.psi.astype(np.uint16)).cuda()
    return pix, psi, torch.from_numpy(nc_h).cuda(), torch.from_numpy(m_h).cuda(), \
        nc_h.astype(np.float64), m_h.astype(np.float64)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_chisq_forward(setup, prec):
    ts, c, tod, nc, maps, _ = setup
    pix, psi, ncd, md, nc_r, m_r = _dev(ts, prec, nc, maps)
    ref = ot.chisq_all(ts, m_r, ts.pix, ts.psi, ts.d, nc_r)
    out = torch.empty(ts.nseg, dtype=torch.float64, device="cuda")
    c.tod_chisq(tod, prec, pix, psi, tod.d, ncd, md, out)
    c.sync()
    got = out.cpu().numpy()
    eps = float(np.finfo(np.float32 if prec == "mixed" else np.float64).eps)
    mag, fft, _ = magnitudes(ts, m_r, nc_r, eps)
    assert np.all(np.abs(got - ref) <= TOL[prec] * mag[0] + fft[0])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_chisq_backward(setup, prec):
    ts, c, tod, nc, maps, _ = setup
    pix, psi, ncd, md, nc_r, m_r = _dev(ts, prec, nc, maps)
    gm, gg, gs, gf, ga = ot.chisq_grad_all(ts, m_r, ts.pix, ts.psi, ts.d, nc_r)
    det_sum = lambda x: np.bincount(ts.seg_det, weights=x, minlength=ts.ndet)
    out = [torch.empty((3, ts.npix_total), dtype=torch.float64, device="cuda"),
           torch.empty(ts.nseg, dtype=torch.float64, device="cuda")] + \
          [torch.empty(ts.ndet, dtype=torch.float64, device="cuda") for _ in range(3)]
    c.tod_chisq_backward(tod, prec, pix, psi, tod.d, ncd, md, 2.0, *out)
    c.sync()
    g = [o.cpu().numpy() for o in out]
    # bounds relative to the summed terms' magnitudes (pixel by pixel for the
    # map gradient), plus the transforms' rounding in the Whittle sums
    eps = float(np.finfo(np.float32 if prec == "mixed" else np.float64).eps)
    mag, fft, gmag = magnitudes(ts, m_r, nc_r, eps)
    tol = TOL[prec]
    hit = gmag > 0
    assert np.all(g[0][~hit] == 0.0)
    assert np.all(np.abs(g[0][hit] - 2 * gm[hit]) <= 2e-12 * gmag[hit])
    assert np.all(np.abs(g[1] - 2 * gg) <= 2 * tol * mag[1])
    for got, ref, k in zip(g[2:], (gs, gf, ga), (2, 3, 4)):
        bound = 2 * det_sum(tol * mag[k] + fft[k])
        assert np.all(np.abs(got - 2 * det_sum(ref)) <= bound), k


def test_autograd_fd_fp64(setup):
    """FP64 central differences (h = 1e-6) of the GPU objective vs its adjoint."""
    from paper_2201_03509_amd.autograd import tod_chisq
    ts, c, tod, nc, maps, sig_det = setup
    pix, psi, ncd, md, nc_r, m_r = _dev(ts, "fp64", nc, maps)
    dev = "cuda"
    fk_det = np.asarray([ts.fknee[np.argmax(ts.seg_det == d)] for d in range(ts.ndet)])
    al_det = np.asarray([ts.alpha[np.argmax(ts.seg_det == d)] for d in range(ts.ndet)])
    m = md.clone().requires_grad_(True)
    g = torch.from_numpy(ts.gain.copy()).to(dev).requires_grad_(True)
    s = torch.from_numpy(sig_det.copy()).to(dev).requires_grad_(True)
    f = torch.from_numpy(fk_det).to(dev).requires_grad_(True)
    a = torch.from_numpy(al_det).to(dev).requires_grad_(True)
    J = tod_chisq(m, g, s, f, a, c, tod, "fp64", pix, psi, ncd)
    J.backward()

    def Jat(**kw):
        args = dict(m=md, g=g.detach(), s=s.detach(), f=f.detach(), a=a.detach())
        args.update(kw)
        with torch.no_grad():
            return float(tod_chisq(args["m"], args["g"], args["s"], args["f"], args["a"], c, tod,
                                   "fp64", pix, psi, ncd))

    h = 1e-6
    for name, t, grad in (("g", g, g.grad), ("s", s, s.grad), ("f", f, f.grad), ("a", a, a.grad)):
        for i in [0, t.numel() - 1]:
            tp = t.detach().clone()
            tm = t.detach().clone()
            tp[i] += h
            tm[i] -= h
            fd = (Jat(**{name: tp}) - Jat(**{name: tm})) / (2 * h)
            assert abs(fd - float(grad[i])) <= 1e-5 * max(1.0, abs(fd)), (name, i, fd, float(grad[i]))
    # random directions in map space
    rng = np.random.default_rng(2)
    for _ in range(4):
        v = torch.from_numpy(rng.normal(size=md.shape)).to(dev)
        fd = (Jat(m=md + h * v) - Jat(m=md - h * v)) / (2 * h)
        an = float((m.grad * v).sum())
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd)), (fd, an)
