"""The oracle: a slow, plain FP64 CPU reference of the TOD step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package;
the product path (``paper_2201_03509_amd``) never does, and shares no code,
header, table or constant with it.

Modules:
  huffman  -- tree-walk decode of the differenced Huffman pointing (section 4.1)
  philox   -- Philox4x32-10 and Box-Muller draws (randomness of the n_corr step)
  tod      -- projection, n_corr constrained realisation (Eq. 4, section 4.2),
              binning and per-pixel solve (section 2.4), chi^2 and gradients
"""
from . import huffman, philox, tod  # noqa: F401
