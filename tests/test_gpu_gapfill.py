"""Masked correlated-noise draw (CG gap filling) on the GPU vs the oracle,
through the C-ABI.

The reference is the plain definition of the draw: x = A^-1 b with
A = F^H diag(1/P) F + diag(mu)/sigma0^2 solved on the whole extended vector
by the oracle's full-system preconditioned CG (`cg_ncorr_segment`, run to a
relative residual of 1e-14), and, for segments short enough to build A as a
dense matrix (n <= 64), `numpy.linalg.solve` of the dense system.  The GPU
solves the same system in its gap-space (Woodbury) form, CG on the masked
positions only; the oracle's restatement of that form (`gap_cg`) is used
here only for a labelled self-consistency check of the iteration counts.

Inputs: the small synthetic sets of the parity suite with a processing mask
that removes a band of +-10 degrees around the map frame's equator (about 11%
of the samples, in long gaps crossed twice per spin period).

Tolerances.  The FP64 path is asked for a relative gap residual of 1e-15 and
held to the spec FP64 bar (1e-12 relative per segment): the gap-space
system is well conditioned (its eigenvalues lie in (0, sigma0^2) and are
bounded away from 0 by the prior at the gap's lowest frequency), so its
solution error stays near its residual.  The mixed path applies M with FP32
transforms while the small system's vectors and every sum stay FP64; it is
asked for 1e-6 and held to the FP32 bar (1e-5 relative per segment).  x0's
drawn term F^H(W2 P^-1/2), large at high frequencies, is added per mode and
never rounded to FP32 in the time domain.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import gapfill as og
from oracle import tod as ot

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-12}
CG_TOL = {"mixed": 1e-6, "fp64": 1e-15}
ORACLE_TOL = 1e-14

_CASES = {
    "tiny": (0, None, None),
    "lfi30_small": (1, 3, ("uniform", 9000, 13000)),
    "mixed_small": (4, 6, ("loguniform2", 11.0, 14.0)),
}
_CACHE = {}


def dataset(name):
    if name not in _CACHE:
        k, ns, ln = _CASES[name]
        ts = synth.make(k, nscan=ns, length=ln, keep_truth=True)
        mask = synth.plane_mask(ts, ts.pix)
        _CACHE[name] = (ts, mask)
    return _CACHE[name]


@pytest.fixture(scope="module")
def ctx():
    from paper_2201_03509_amd import ops
    c = ops.Context(0)
    yield c
    c.close()


def _signal(ts, prec):
    m = ts.maps.astype(np.float32) if prec == "mixed" else ts.maps
    s = ot.project_all(ts, m.astype(np.float64), ts.pix, ts.psi)
    return s.astype(np.float32 if prec == "mixed" else np.float64)


def _gpu(ctx, ts, prec, d, s_in, mask, seed, it, mean_only=False, tol=None, max_iter=500):
    from paper_2201_03509_amd import ops
    tod = ops.DeviceTod(ts, "cuda:0")
    ft = torch.float32 if prec == "mixed" else torch.float64
    out = torch.empty(ts.nsamp, dtype=ft, device="cuda")
    iters = torch.empty(ts.nseg, dtype=torch.int32, device="cuda")
    d_dev = tod.d if d is None else torch.from_numpy(d).cuda()
    ctx.sample_ncorr_masked(tod, prec, d_dev, torch.from_numpy(s_in).cuda(),
                            torch.from_numpy(mask.astype(np.uint8)).cuda(), seed, it, out,
                            mean_only=mean_only, tol=CG_TOL[prec] if tol is None else tol,
                            max_iter=max_iter, iters=iters)
    ctx.sync()
    return out.cpu().numpy().astype(np.float64), iters.cpu().numpy()


def seg_rel(ts, got, ref):
    errs = []
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        nr = np.linalg.norm(ref[a:b])
        if b > a:
            errs.append(np.linalg.norm(got[a:b] - ref[a:b]) / max(nr, 1e-300))
    return max(errs)


@pytest.mark.parametrize("mean_only", [False, True])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["tiny", "lfi30_small", "mixed_small"])
def test_masked_draw(ctx, name, prec, mean_only):
    ts, mask = dataset(name)
    s_in = _signal(ts, prec)
    seed, it = synth.seed32(ts.config), 5
    # the plain definition: the full extended system, preconditioned CG
    ref, _ = og.cg_ncorr_all(ts, ts.d, s_in.astype(np.float64), mask, seed, it, mean_only=mean_only,
                             tol=ORACLE_TOL)
    got, iters = _gpu(ctx, ts, prec, None, s_in, mask, seed, it, mean_only)
    err = seg_rel(ts, got, ref)
    print("%s %s mean_only=%s: max segment rel L2 %.3e, iterations %d..%d" % (
        name, prec, mean_only, err, iters.min(), iters.max()))
    assert err < TOL[prec]
    assert (iters > 0).all()  # every segment converged


def test_masked_iterations_self_consistent(ctx):
    """Self-consistency, not parity: the GPU's gap-space CG and the oracle's
    restatement of it (same recurrence, same stopping rule) take the same
    number of iterations, up to rounding, on the FP64 path."""
    ts, mask = dataset("lfi30_small")
    s_in = _signal(ts, "fp64")
    seed, it = synth.seed32(ts.config), 5
    _, ref_it = og.cg_ncorr_all_gap(ts, ts.d, s_in, mask, seed, it, tol=1e-13)
    _, iters = _gpu(ctx, ts, "fp64", None, s_in, mask, seed, it, tol=1e-13)
    for q, k in ref_it.items():
        assert abs(int(iters[q]) - k) <= 1


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_masked_draw_dense_solve(ctx, prec):
    """Segments of 5..64 samples: A and b built as dense matrices from the DFT
    matrix, x = numpy.linalg.solve(A, b), against the GPU draw."""
    ts = synth.make(1, nscan=4, length=("uniform", 5, 64), keep_truth=True)
    rng = np.random.default_rng(21)
    mask = np.ones(ts.nsamp, dtype=np.uint8)
    for q in range(ts.nseg):  # one masked run per segment, never the whole segment
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        i0 = a + 1 + int(rng.integers(0, b - a - 1))
        mask[i0:min(b, i0 + int(rng.integers(1, 20)))] = 0
    s_in = _signal(ts, prec)
    seed, it = 77, 3
    got, iters = _gpu(ctx, ts, prec, None, s_in, mask, seed, it)
    errs = []
    for q in range(ts.nseg):
        a, b = int(ts.seg_off[q]), int(ts.seg_off[q + 1])
        band = int(ts.seg_band[q])
        A, rhs = og.dense_system(ts.d[a:b] - s_in[a:b].astype(np.float64), mask[a:b],
                                 float(ts.band_fsamp[band]), float(ts.sigma0[q]), float(ts.fknee[q]),
                                 float(ts.alpha[q]), seed, q, it)
        ref = np.linalg.solve(A, rhs)[:b - a]
        errs.append(np.linalg.norm(got[a:b] - ref) / np.linalg.norm(ref))
    print("dense-solve check: max segment rel L2 %.3e" % max(errs))
    assert max(errs) < TOL[prec]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_unmasked_is_the_fourier_draw(ctx, prec):
    """With nothing masked A^-1 = M: x = M b is the unmasked constrained
    realisation (the same Philox modes), with no CG iteration."""
    ts, _ = dataset("lfi30_small")
    s_in = _signal(ts, prec)
    seed, it = synth.seed32(ts.config), 8
    ones = np.ones(ts.nsamp, dtype=np.uint8)
    got, iters = _gpu(ctx, ts, prec, None, s_in, ones, seed, it)
    ref = ot.sample_ncorr_all(ts, ts.d, s_in.astype(np.float64), seed, it)
    assert seg_rel(ts, got, ref) < TOL[prec]
    assert (iters == 0).all()


def test_masked_samples_do_not_matter(ctx):
    ts, mask = dataset("lfi30_small")
    s_in = _signal(ts, "fp64")
    seed, it = 17, 2
    d2 = ts.d.astype(np.float64).copy()
    bad = mask == 0
    d2[bad] += np.random.default_rng(4).normal(size=int(bad.sum())) * 1e3
    a, _ = _gpu(ctx, ts, "fp64", ts.d.astype(np.float64), s_in, mask, seed, it)
    b, _ = _gpu(ctx, ts, "fp64", d2, s_in, mask, seed, it)
    assert seg_rel(ts, b, a) < TOL["fp64"]


def test_max_iter_stops_with_the_oracle_iterate(ctx):
    """max_iter = 3: the GPU returns the third CG iterate, flagged unconverged,
    equal to the oracle's third iterate."""
    ts, mask = dataset("tiny")
    s_in = _signal(ts, "fp64")
    seed, it = 3, 1
    ref, _ = og.cg_ncorr_all_gap(ts, ts.d, s_in, mask, seed, it, tol=0.0, maxiter=3)
    got, iters = _gpu(ctx, ts, "fp64", None, s_in, mask, seed, it, tol=0.0, max_iter=3)
    assert (iters == -3).all()
    assert seg_rel(ts, got, ref) < TOL["fp64"]


def test_fully_masked_segment(ctx):
    """A segment with every sample masked: the draw is the prior's, b = F^H W2 P^-1/2
    plus the observed pad."""
    ts, mask = dataset("tiny")
    mask = mask.copy()
    a, b = int(ts.seg_off[2]), int(ts.seg_off[3])
    mask[a:b] = 0
    s_in = _signal(ts, "fp64")
    seed, it = 9, 4
    full, _ = og.cg_ncorr_all(ts, ts.d, s_in, mask, seed, it, tol=ORACLE_TOL)
    got, iters = _gpu(ctx, ts, "fp64", None, s_in, mask, seed, it)
    assert (iters > 0).all()
    assert seg_rel(ts, got, full) < TOL["fp64"]
