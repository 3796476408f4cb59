"""Workload shapes: synthetic Planck-LFI-shaped scans (the LFI data are absent).

Five configurations; shapes come from the paper's LFI bands (nside 512/512/1024
and n_psi = 4096, section 4.1; pointing periods as scans, section 2.4).

* ``tiny``      nside 16, 1 detector, 8 scans x 4096 samples at 32.5 Hz, FP64 TOD.
* ``lfi30``     nside 512, 4 detectors, 200 scans, n ~ U{100000..130000}, 32.5 Hz.
* ``lfi70``     nside 1024, 12 detectors, 300 scans, n ~ U{230000..290000}, 78.8 Hz.
* ``grad``      the ``lfi30`` data, used for the chi^2 forward/adjoint checks.
* ``mixed``     1000 scans, n = floor(2^(14+5u)); three bands nside 256/512/1024 at
                32.5/46.5/78.8 Hz with 4/6/12 detectors, scans dealt round-robin.
"""
from dataclasses import dataclass, field, replace
from typing import List, Tuple


@dataclass(frozen=True)
class Band:
    nside: int
    fsamp: float
    ndet: int


@dataclass(frozen=True)
class Config:
    index: int
    name: str
    bands: Tuple[Band, ...]
    nscan: int
    length: Tuple                          # ("uniform", lo, hi), ("loguniform2", e0, e1) or ("list", n0, n1, ...)
    tod_f64: bool
    fknee_fixed: float = 0.0               # >0: every detector uses it
    alpha_fixed: float = 0.0
    fknee_range: Tuple[float, float] = (0.05, 0.3)
    alpha_range: Tuple[float, float] = (-1.8, -1.0)
    chunk_len: int = 32                    # Huffman side-index spacing (symbols): the
                                           # densest the format allows; neighbouring
                                           # chunks then share cache lines in the decoder

    def scaled(self, nscan=None, length=None, bands=None, chunk_len=None):
        kw = {}
        if chunk_len is not None:
            kw["chunk_len"] = int(chunk_len)
        if nscan is not None:
            kw["nscan"] = int(nscan)
        if length is not None:
            kw["length"] = tuple(length)
        if bands is not None:
            kw["bands"] = tuple(bands)
        return replace(self, **kw)


CONFIGS = {
    0: Config(0, "tiny", (Band(16, 32.5, 1),), 8, ("uniform", 4096, 4096), True,
              fknee_fixed=0.1, alpha_fixed=-1.5),
    1: Config(1, "lfi30", (Band(512, 32.5, 4),), 200, ("uniform", 100000, 130000), False),
    2: Config(2, "lfi70", (Band(1024, 78.8, 12),), 300, ("uniform", 230000, 290000), False),
    3: Config(3, "grad", (Band(512, 32.5, 4),), 200, ("uniform", 100000, 130000), False),
    4: Config(4, "mixed", (Band(256, 32.5, 4), Band(512, 46.5, 6), Band(1024, 78.8, 12)),
              1000, ("loguniform2", 14.0, 19.0), False),
}


def get(k):
    return CONFIGS[int(k)]
