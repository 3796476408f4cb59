"""Host-side argument checks of the draw and stream entry points: each bad
argument is reported as InvalidArgument before any device work is queued,
and the context stays usable afterwards."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_2201_03509_amd import ops
    ts = synth.make(0, tod_streams=True, keep_truth=True)
    c = ops.Context(0)
    tod = ops.DeviceTod(ts, "cuda:0")
    yield c, ts, tod
    c.close()


def test_bad_arguments_rejected(env):
    from paper_2201_03509_amd import ops
    c, ts, tod = env
    n, k = ts.nsamp, ts.nseg
    s = torch.zeros(n, dtype=torch.float64, device="cuda")
    m = torch.ones(n, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty(k, dtype=torch.float64, device="cuda")
    bad = [
        lambda: c.sample_ncorr_masked(tod, "fp64", tod.d, s, m, 1, 1, out, tol=-1.0),
        lambda: c.sample_ncorr_masked(tod, "fp64", tod.d, s, m, 1, 1, out, max_iter=0),
        lambda: c.sample_ncorr_masked(tod, "fp64", tod.d, s, None, 1, 1, out),
        lambda: c.sample_gain(tod, "fp64", tod.d, s, 1, 1, None),
        lambda: c.sample_noise(tod, "fp64", tod.d, s, s, 1, 1, g, None, g),
        lambda: c.decode_tod(tod, "fp64", out, quantum=0.0),
        lambda: c.decode_flags(tod, 1, None, None),
    ]
    for f in bad:
        with pytest.raises(ops.InvalidArgument):
            f()
    c.sync()
    # still usable
    c.decode_tod(tod, "fp64", out)
    c.sync()
    assert np.array_equal(out.cpu().numpy(), ts.d.astype(np.float64))
