"""Seeded synthetic input generators (inputs only; no step of the method)."""
from .make import make, seed32, TodSet, HuffStream, save, load, make_cached, plane_mask, plane_mask_pixels  # noqa: F401
from .make import TOD_QUANTUM, FLAG_PLANE, FLAG_GLITCH  # noqa: F401
from . import configs, healpix, huffman_enc  # noqa: F401
