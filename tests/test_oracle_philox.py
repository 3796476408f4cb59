"""Pin the oracle's Philox4x32-10 and Box-Muller normals."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_philox_matches_rocrand_host():
    """rocRAND ships its own Philox4x32-10; its host path must agree word for word."""
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "ph")
    subprocess.check_call(["hipcc", "-O1", "--offload-arch=gfx950", "-o", exe,
                           os.path.join(HERE, "philox_rocrand_host.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(7)
    v = rng.integers(0, 2 ** 32, size=(500, 6), dtype=np.uint64)
    v[0] = 0
    v[1] = 2 ** 32 - 1
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in v) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()])
    mine = np.stack(philox.philox4x32_10(*v.T), axis=1).astype(np.int64)
    shutil.rmtree(d)
    assert np.array_equal(mine, ref)


def test_normals_distribution():
    z0, z1, z2, z3 = philox.mode_normals(0x22013509, 3, 0, np.arange(200000))
    z = np.concatenate([z0, z1, z2, z3])
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 5 / np.sqrt(len(z0))


def test_counter_mapping_distinct_streams():
    a = philox.mode_words(1, 0, 0, np.arange(8))
    b = philox.mode_words(1, 1, 0, np.arange(8))
    c = philox.mode_words(1, 0, 1, np.arange(8))
    d = philox.mode_words(1 + (1 << 32), 0, 0, np.arange(8))
    for x in (b, c, d):
        assert not np.array_equal(a[0], x[0])
