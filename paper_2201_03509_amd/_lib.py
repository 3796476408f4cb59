"""ctypes view of the c3tod C-ABI (include/c3tod.h).  Marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libc3tod.so")

TOD_OK, TOD_EINVAL, TOD_ENOMEM, TOD_EHIP, TOD_ECORRUPT, TOD_ENOTSUP = range(6)
TOD_PLAIN_FP64, TOD_MIXED = 0, 1
TOD_F32, TOD_F64 = 0, 1

STATUS_NAMES = {0: "TOD_OK", 1: "TOD_EINVAL", 2: "TOD_ENOMEM", 3: "TOD_EHIP",
                4: "TOD_ECORRUPT", 5: "TOD_ENOTSUP"}

# every entry point the header declares
EXPORTS = [
    "tod_ctx_create", "tod_ctx_destroy", "tod_sync", "tod_clear_error", "tod_last_error",
    "tod_device_error_bits", "decode_pointing", "decode_tod", "decode_flags", "project_sky", "sample_ncorr", "sample_ncorr_masked", "sample_gain", "sample_noise",
    "bin_tod",
    "solve_maps", "tod_chisq", "tod_chisq_backward", "tod_sweep", "tod_autotune",
    "tod_load_tuning", "tod_set_bin_stride", "tod_set_fft_batch", "tod_enable_timing",
    "tod_kernel_times", "tod_plan", "decode_pointing_noalloc", "tod_set_bin_runs",
    "tod_sweep_stream",
]


class tod_band(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int32), ("npsi", ctypes.c_int32), ("npix", ctypes.c_int64),
                ("pix_off", ctypes.c_int64), ("fsamp", ctypes.c_double)]


class tod_layout(ctypes.Structure):
    _fields_ = [("nseg", ctypes.c_int32), ("nband", ctypes.c_int32), ("ndet", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("nsamp", ctypes.c_int64),
                ("npix_total", ctypes.c_int64),
                ("seg_off", ctypes.c_void_p), ("seg_band", ctypes.c_void_p),
                ("seg_det", ctypes.c_void_p), ("seg_accept", ctypes.c_void_p),
                ("h_seg_off", ctypes.c_void_p), ("h_seg_band", ctypes.c_void_p),
                ("bands", ctypes.POINTER(tod_band)), ("h_seg_det", ctypes.c_void_p)]


class tod_huff(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("seg_word_off", ctypes.c_void_p),
                ("seg_table", ctypes.c_void_p), ("tables", ctypes.c_void_p),
                ("table_off", ctypes.c_void_p), ("chunk_bit", ctypes.c_void_p),
                ("chunk_prev", ctypes.c_void_p), ("seg_chunk_off", ctypes.c_void_p),
                ("chunk_len", ctypes.c_int32), ("ntable", ctypes.c_int32),
                ("nwords", ctypes.c_int64), ("nchunk", ctypes.c_int64)]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load libc3tod.so; raises LibraryMissing when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing("libc3tod.so not built: run __graft_entry__.build() "
                             "or python paper_2201_03509_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    LP, HP = ctypes.POINTER(tod_layout), ctypes.POINTER(tod_huff)
    sig = {
        "tod_ctx_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, P],
        "tod_ctx_destroy": [P],
        "tod_sync": [P],
        "tod_clear_error": [P],
        "tod_last_error": [P],
        "tod_device_error_bits": [P],
        "decode_pointing": [P, LP, HP, HP, P, P],
        "decode_pointing_noalloc": [P, LP, HP, HP, P, P],
        "project_sky": [P, LP, ctypes.c_int, P, P, P, P, P],
        "sample_ncorr": [P, LP, ctypes.c_int, P, ctypes.c_int, P, P, P, P, U64, U64,
                         ctypes.c_int, P],
        "sample_ncorr_masked": [P, LP, ctypes.c_int, P, ctypes.c_int, P, P, P, P, P, U64, U64,
                                ctypes.c_int, D, ctypes.c_int, P, P],
        "sample_gain": [P, LP, ctypes.c_int, P, ctypes.c_int, P, P, P, P, U64, U64, ctypes.c_int, P, P],
        "decode_tod": [P, LP, ctypes.c_int, HP, D, P],
        "decode_flags": [P, LP, HP, ctypes.c_uint32, P, P],
        "sample_noise": [P, LP, ctypes.c_int, P, ctypes.c_int, P, P, P, P, U64, U64, ctypes.c_int, P, P, P],
        "bin_tod": [P, LP, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int],
        "solve_maps": [P, I64, P, D, P, ctypes.c_int, P],
        "tod_chisq": [P, LP, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P, P, P],
        "tod_chisq_backward": [P, LP, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P, P,
                               D, P, P, P, P, P, P],
        "tod_sweep": [P, LP, ctypes.c_int, HP, HP, P, ctypes.c_int, P, P, P, P, P, U64, U64,
                      P, P, P, P, ctypes.c_int],
        "tod_sweep_stream": [P, LP, ctypes.c_int, HP, HP, HP, D, P, P, P, P, P, P, U64, U64,
                             P, P, P, P, ctypes.c_int],
        "tod_autotune": [P, LP, ctypes.c_int, P, ctypes.c_char_p],
        "tod_load_tuning": [P, ctypes.c_char_p],
        "tod_plan": [P, LP, ctypes.c_int, ctypes.c_char_p],
        "tod_set_bin_stride": [P, I32, I32],
        "tod_set_bin_runs": [P, I32],
        "tod_set_fft_batch": [P, I64],
        "tod_enable_timing": [P, ctypes.c_int],
        "tod_kernel_times": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.tod_last_error.restype = ctypes.c_char_p
    lib.tod_device_error_bits.restype = ctypes.c_uint32
    _lib = lib
    return lib
