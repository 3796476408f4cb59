"""Python binding of the c3tod C-ABI: the same entry points, taking torch tensors.

Every step of the TOD path runs in the HIP kernels of libc3tod.so; this module
only turns tensors into device pointers and status codes into exceptions.
PyTorch provides device memory and the stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L


class C3todError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (L.STATUS_NAMES.get(status, status), msg))
        self.status = status


class InvalidArgument(C3todError):
    pass


class CorruptStream(C3todError):
    pass


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _acc(acc):
    """Pointer of binned accumulators: a (10, npix) FP64 view of a pixel-major
    [npix][10] device buffer, as new_acc returns."""
    if (acc.dtype != torch.float64 or acc.dim() != 2 or acc.shape[0] != 10
            or acc.stride() != (1, 10)):
        raise ValueError("acc must be the (10, npix) view of a pixel-major [npix][10] FP64 buffer "
                         "(ops.new_acc)")
    return ctypes.c_void_p(acc.data_ptr())


def new_acc(npix_total, device):
    """Binned accumulators for npix_total pixels: stored pixel-major, [npix][10]
    (one record of ten per pixel), returned as a (10, npix) view so that
    acc[j] is component j of every pixel."""
    return torch.empty((npix_total, 10), dtype=torch.float64, device=device).t()


def _prec(prec):
    if prec in ("mixed", L.TOD_MIXED):
        return L.TOD_MIXED
    if prec in ("fp64", "plain", L.TOD_PLAIN_FP64):
        return L.TOD_PLAIN_FP64
    raise ValueError("precision must be 'mixed' or 'fp64'")


def _dt(t):
    if t.dtype == torch.float32:
        return L.TOD_F32
    if t.dtype == torch.float64:
        return L.TOD_F64
    raise ValueError("TOD must be float32 or float64")


class DeviceTod:
    """A TOD set resident on the GPU plus the C structs that describe it.

    ``src`` is any object with the numpy arrays of a TOD set (segment table,
    bands, Huffman streams, d, per-segment gain and noise parameters)."""

    def __init__(self, src, device="cuda"):
        dev = torch.device(device)
        self.device = dev
        to = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a if dt is None else a.astype(dt))).to(dev)
        self.nseg = int(src.nseg)
        self.nband = int(src.nband)
        self.ndet = int(src.ndet)
        self.nsamp = int(src.nsamp)
        self.npix_total = int(src.npix_total)
        self.h_seg_off = np.ascontiguousarray(src.seg_off, dtype=np.int64)
        self.h_seg_band = np.ascontiguousarray(src.seg_band, dtype=np.int32)
        self.seg_off = to(self.h_seg_off)
        self.seg_band = to(self.h_seg_band)
        self.seg_det = to(src.seg_det, np.int32)
        self.seg_accept = to(src.seg_accept, np.uint8)
        self.seg_det_h = np.ascontiguousarray(src.seg_det, dtype=np.int32)
        bands = (L.tod_band * self.nband)()
        for b in range(self.nband):
            bands[b].nside = int(src.band_nside[b])
            bands[b].npsi = 4096
            bands[b].npix = int(src.band_npix[b])
            bands[b].pix_off = int(src.band_pix_off[b])
            bands[b].fsamp = float(src.band_fsamp[b])
        self._bands = bands
        lay = L.tod_layout()
        lay.nseg, lay.nband, lay.ndet = self.nseg, self.nband, self.ndet
        lay.nsamp, lay.npix_total = self.nsamp, self.npix_total
        lay.seg_off = self.seg_off.data_ptr()
        lay.seg_band = self.seg_band.data_ptr()
        lay.seg_det = self.seg_det.data_ptr()
        lay.seg_accept = self.seg_accept.data_ptr()
        lay.h_seg_off = self.h_seg_off.ctypes.data
        lay.h_seg_band = self.h_seg_band.ctypes.data
        lay.bands = bands
        lay.h_seg_det = self.seg_det_h.ctypes.data
        self.layout = lay
        self.d = to(src.d)
        self.gain = to(src.gain, np.float64)
        self.sigma0 = to(src.sigma0, np.float64)
        self.fknee = to(src.fknee, np.float64)
        self.alpha = to(src.alpha, np.float64)
        self.pix_huff, self._pt = self._huff(src.pix_huff, to)
        self.psi_huff, self._qt = self._huff(src.psi_huff, to)
        # compressed TOD and flag streams, when the set carries them
        self.tod_huff = self.flag_huff = None
        if getattr(src, "tod_huff", None) is not None:
            self.tod_huff, self._tt = self._huff(src.tod_huff, to)
            self.tod_quantum = float(src.tod_quantum)
        if getattr(src, "flag_huff", None) is not None:
            self.flag_huff, self._ft = self._huff(src.flag_huff, to)

    def refresh_accept(self):
        self.layout.seg_accept = self.seg_accept.data_ptr()

    @staticmethod
    def _huff(hs, to):
        t = {
            "words": to(hs.words, np.uint32),
            "seg_word_off": to(hs.seg_word_off, np.int64),
            "seg_table": to(hs.seg_table, np.int32),
            "tables": to(hs.tables, np.uint32),
            "table_off": to(hs.table_off, np.int64),
            "chunk_bit": to(hs.chunk_bit, np.uint32),
            "chunk_prev": to(hs.chunk_prev, np.int32),
            "seg_chunk_off": to(hs.seg_chunk_off, np.int64),
        }
        h = L.tod_huff()
        for k, v in t.items():
            setattr(h, k, v.data_ptr())
        h.chunk_len = int(hs.chunk_len)
        h.ntable = int(len(hs.table_off) - 1)
        h.nwords = int(len(hs.words))
        h.nchunk = int(len(hs.chunk_bit))
        return h, t


class Context:
    """One c3tod context on one device and stream."""

    def __init__(self, device=0, stream=None):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise C3todError(L.TOD_EHIP, "no HIP device available")
        torch.cuda.set_device(device)
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = st
        h = ctypes.c_void_p()
        self._chk(self.lib.tod_ctx_create(ctypes.byref(h), int(device),
                                          ctypes.c_void_p(st.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tod_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st == L.TOD_OK:
            return
        msg = ""
        if getattr(self, "h", None):
            m = self.lib.tod_last_error(self.h)
            msg = m.decode() if m else ""
        if st == L.TOD_EINVAL:
            raise InvalidArgument(st, msg)
        if st == L.TOD_ECORRUPT:
            raise CorruptStream(st, msg)
        raise C3todError(st, msg)

    # --------------------------------------------------------------- entry points
    def sync(self):
        self._chk(self.lib.tod_sync(self.h))

    def clear_error(self):
        self._chk(self.lib.tod_clear_error(self.h))

    def device_error_bits(self):
        return int(self.lib.tod_device_error_bits(self.h))

    def decode_pointing(self, tod, pix_out, psi_out, pix_huff=None, psi_huff=None):
        self._chk(self.lib.decode_pointing(self.h, ctypes.byref(tod.layout),
                                           ctypes.byref(pix_huff or tod.pix_huff),
                                           ctypes.byref(psi_huff or tod.psi_huff),
                                           _ptr(pix_out), _ptr(psi_out)))

    def decode_pointing_noalloc(self, tod, pix_out, psi_out, pix_huff=None, psi_huff=None):
        self._chk(self.lib.decode_pointing_noalloc(self.h, ctypes.byref(tod.layout),
                                                   ctypes.byref(pix_huff or tod.pix_huff),
                                                   ctypes.byref(psi_huff or tod.psi_huff),
                                                   _ptr(pix_out), _ptr(psi_out)))

    def decode_tod(self, tod, prec, d_out, quantum=None, tod_huff=None):
        self._chk(self.lib.decode_tod(self.h, ctypes.byref(tod.layout), _prec(prec),
                                      ctypes.byref(tod_huff or tod.tod_huff),
                                      float(tod.tod_quantum if quantum is None else quantum), _ptr(d_out)))

    def decode_flags(self, tod, flag_mask, flags_out=None, mask_out=None, flag_huff=None):
        self._chk(self.lib.decode_flags(self.h, ctypes.byref(tod.layout), ctypes.byref(flag_huff or tod.flag_huff),
                                        ctypes.c_uint32(int(flag_mask)), _ptr(flags_out), _ptr(mask_out)))

    def project_sky(self, tod, prec, pix, psi, maps, s_out, gain=None):
        self._chk(self.lib.project_sky(self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(pix),
                                       _ptr(psi), _ptr(maps), _ptr(tod.gain if gain is None else gain),
                                       _ptr(s_out)))

    def sample_ncorr(self, tod, prec, d, s, seed, it, out, mean_only=False, sigma0=None,
                     fknee=None, alpha=None):
        self._chk(self.lib.sample_ncorr(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(d), _dt(d), _ptr(s),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _ptr(tod.fknee if fknee is None else fknee),
            _ptr(tod.alpha if alpha is None else alpha), ctypes.c_uint64(int(seed)),
            ctypes.c_uint64(int(it)), int(bool(mean_only)), _ptr(out)))

    def sample_ncorr_masked(self, tod, prec, d, s, mask, seed, it, out, mean_only=False, tol=1e-6,
                            max_iter=500, iters=None, sigma0=None, fknee=None, alpha=None):
        self._chk(self.lib.sample_ncorr_masked(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(d), _dt(d), _ptr(s), _ptr(mask),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _ptr(tod.fknee if fknee is None else fknee),
            _ptr(tod.alpha if alpha is None else alpha), ctypes.c_uint64(int(seed)),
            ctypes.c_uint64(int(it)), int(bool(mean_only)), float(tol), int(max_iter), _ptr(out),
            _ptr(iters)))

    def sample_gain(self, tod, prec, d, t, seed, it, gain_out, sigma_out=None, mean_only=False,
                    sigma0=None, fknee=None, alpha=None):
        self._chk(self.lib.sample_gain(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(d), _dt(d), _ptr(t),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _ptr(tod.fknee if fknee is None else fknee),
            _ptr(tod.alpha if alpha is None else alpha), ctypes.c_uint64(int(seed)),
            ctypes.c_uint64(int(it)), int(bool(mean_only)), _ptr(gain_out), _ptr(sigma_out)))

    def sample_noise(self, tod, prec, d, t, ncorr, seed, it, sigma0_out, fknee_out, alpha_out,
                     mean_only=False, gain=None, fknee=None):
        self._chk(self.lib.sample_noise(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(d), _dt(d), _ptr(t),
            _ptr(tod.gain if gain is None else gain), _ptr(ncorr),
            _ptr(tod.fknee if fknee is None else fknee), ctypes.c_uint64(int(seed)),
            ctypes.c_uint64(int(it)), int(bool(mean_only)), _ptr(sigma0_out), _ptr(fknee_out),
            _ptr(alpha_out)))

    def bin_tod(self, tod, prec, pix, psi, d, ncorr, acc, accumulate=False, gain=None, sigma0=None):
        self._chk(self.lib.bin_tod(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(pix), _ptr(psi), _ptr(d), _dt(d),
            _ptr(ncorr), _ptr(tod.gain if gain is None else gain),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _acc(acc), int(bool(accumulate))))

    def solve_maps(self, acc, rcond_min, map_out, rcond_out=None):
        a = _acc(acc)
        npix = acc.shape[1]
        self._chk(self.lib.solve_maps(self.h, int(npix), a, float(rcond_min), _ptr(map_out),
                                      _dt(map_out), _ptr(rcond_out)))

    def tod_chisq(self, tod, prec, pix, psi, d, ncorr, maps, chisq_seg, gain=None, sigma0=None,
                  fknee=None, alpha=None):
        self._chk(self.lib.tod_chisq(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(pix), _ptr(psi), _ptr(d), _dt(d),
            _ptr(ncorr), _ptr(maps), _ptr(tod.gain if gain is None else gain),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _ptr(tod.fknee if fknee is None else fknee),
            _ptr(tod.alpha if alpha is None else alpha), _ptr(chisq_seg)))

    def tod_chisq_backward(self, tod, prec, pix, psi, d, ncorr, maps, grad_scale, grad_maps=None,
                           grad_gain=None, grad_sigma0=None, grad_fknee=None, grad_alpha=None,
                           gain=None, sigma0=None, fknee=None, alpha=None):
        """grad_scale: a number, or a one-element FP64 device tensor read by the kernels."""
        if torch.is_tensor(grad_scale):
            if grad_scale.dtype != torch.float64 or grad_scale.numel() != 1 or not grad_scale.is_cuda:
                raise ValueError("a tensor grad_scale must be one FP64 value on the device")
            gs_host, gs_dev = 1.0, _ptr(grad_scale)
        else:
            gs_host, gs_dev = float(grad_scale), None
        self._chk(self.lib.tod_chisq_backward(
            self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(pix), _ptr(psi), _ptr(d), _dt(d),
            _ptr(ncorr), _ptr(maps), _ptr(tod.gain if gain is None else gain),
            _ptr(tod.sigma0 if sigma0 is None else sigma0), _ptr(tod.fknee if fknee is None else fknee),
            _ptr(tod.alpha if alpha is None else alpha), gs_host, gs_dev, _ptr(grad_maps),
            _ptr(grad_gain), _ptr(grad_sigma0), _ptr(grad_fknee), _ptr(grad_alpha)))

    def tod_sweep(self, tod, prec, maps, seed, it, ncorr_out, acc, pix_work, psi_work,
                  use_graph=False, pix_huff=None, psi_huff=None):
        self._chk(self.lib.tod_sweep(
            self.h, ctypes.byref(tod.layout), _prec(prec), ctypes.byref(pix_huff or tod.pix_huff),
            ctypes.byref(psi_huff or tod.psi_huff), _ptr(tod.d), _dt(tod.d), _ptr(maps), _ptr(tod.gain),
            _ptr(tod.sigma0), _ptr(tod.fknee), _ptr(tod.alpha), ctypes.c_uint64(int(seed)),
            ctypes.c_uint64(int(it)), _ptr(ncorr_out), _acc(acc), _ptr(pix_work), _ptr(psi_work),
            int(bool(use_graph))))

    def tod_sweep_stream(self, tod, prec, maps, seed, it, ncorr_out, acc, pix_work, psi_work, d_work,
                         use_graph=False):
        """The fused sweep with the TOD decoded from tod.tod_huff into d_work."""
        self._chk(self.lib.tod_sweep_stream(
            self.h, ctypes.byref(tod.layout), _prec(prec), ctypes.byref(tod.pix_huff),
            ctypes.byref(tod.psi_huff), ctypes.byref(tod.tod_huff), float(tod.tod_quantum), _ptr(d_work),
            _ptr(maps), _ptr(tod.gain), _ptr(tod.sigma0), _ptr(tod.fknee), _ptr(tod.alpha),
            ctypes.c_uint64(int(seed)), ctypes.c_uint64(int(it)), _ptr(ncorr_out), _acc(acc), _ptr(pix_work),
            _ptr(psi_work), int(bool(use_graph))))

    def autotune(self, tod, prec, pix=None, cache_path=None):
        self._chk(self.lib.tod_autotune(self.h, ctypes.byref(tod.layout), _prec(prec), _ptr(pix),
                                        cache_path.encode() if cache_path else None))

    def plan(self, tod, prec, tune_cache=None):
        self._chk(self.lib.tod_plan(self.h, ctypes.byref(tod.layout), _prec(prec),
                                    tune_cache.encode() if tune_cache else None))

    def load_tuning(self, path):
        self._chk(self.lib.tod_load_tuning(self.h, path.encode()))

    def set_bin_stride(self, band, stride):
        self._chk(self.lib.tod_set_bin_stride(self.h, int(band), int(stride)))

    def set_bin_runs(self, scans):
        self._chk(self.lib.tod_set_bin_runs(self.h, int(scans)))

    def set_fft_batch(self, complex_elems):
        self._chk(self.lib.tod_set_fft_batch(self.h, int(complex_elems)))

    def enable_timing(self, on=True):
        self._chk(self.lib.tod_enable_timing(self.h, int(bool(on))))

    KERNELS = ["decode", "project", "fft_col_fwd", "fft_row", "fft_col_inv", "bin", "solve",
               "chisq_time", "cg_vector", "gain", "noise"]

    def kernel_times(self):
        """{kernel: (total_ms, launches)} since the previous read."""
        t = (ctypes.c_double * len(self.KERNELS))()
        n = (ctypes.c_int32 * len(self.KERNELS))()
        self._chk(self.lib.tod_kernel_times(self.h, t, n))
        return {k: (t[i], n[i]) for i, k in enumerate(self.KERNELS)}


def new_outputs(tod, prec):
    """Allocate the per-sample and per-pixel outputs of one sweep."""
    dev = tod.device
    ft = torch.float32 if _prec(prec) == L.TOD_MIXED else torch.float64
    return {
        "pix": torch.empty(tod.nsamp, dtype=torch.int32, device=dev),
        "psi": torch.empty(tod.nsamp, dtype=torch.uint16, device=dev),
        "ncorr": torch.empty(tod.nsamp, dtype=ft, device=dev),
        "acc": new_acc(tod.npix_total, dev),
    }
