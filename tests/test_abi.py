"""The C-ABI library loads and exports every function include/c3tod.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "c3tod.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tod_status|const char \*|uint32_t)\s*([a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_header_declares_hot_path():
    names = _declared()
    for n in ["decode_pointing", "project_sky", "sample_ncorr", "bin_tod", "tod_chisq",
              "tod_chisq_backward", "solve_maps", "tod_sweep", "tod_ctx_create"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2201_03509_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libc3tod.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing
    assert sorted(_lib.EXPORTS) == _declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2201_03509_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()


def test_struct_layouts():
    from paper_2201_03509_amd import _lib
    assert ctypes.sizeof(_lib.tod_band) == 32
    assert ctypes.sizeof(_lib.tod_layout) == 4 * 4 + 8 * 2 + 8 * 8
    assert ctypes.sizeof(_lib.tod_huff) == 8 * 8 + 4 * 2 + 8 * 2


def test_accumulator_layout_is_pixel_major():
    """The binned accumulators are [npix][10] in memory (one record of ten per
    pixel); the binding hands them out as a (10, npix) view and refuses any
    other layout before a call."""
    import torch
    from paper_2201_03509_amd import ops
    acc = ops.new_acc(7, "cpu")
    assert acc.shape == (10, 7) and acc.stride() == (1, 10)
    acc.zero_()
    acc[3, 5] = 1.0  # component 3 of pixel 5 is word 5 * 10 + 3 of the buffer
    flat = torch.as_strided(acc, (70,), (1,))
    assert flat[53].item() == 1.0 and flat.sum().item() == 1.0
    assert ops._acc(acc).value == acc.data_ptr()
    for bad in (torch.zeros((10, 7), dtype=torch.float64),      # component-major
                torch.zeros((7, 10), dtype=torch.float64),      # pixel-major but not the view
                ops.new_acc(7, "cpu").float()):                 # wrong type
        with pytest.raises(ValueError):
            ops._acc(bad)
