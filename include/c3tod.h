/*
 * c3tod -- time-ordered-data (TOD) step of a Commander3-style Gibbs sampler
 * (Galloway et al., "BeyondPlanck III. Commander3", arXiv:2201.03509) on one
 * AMD Instinct MI355X (gfx950).
 *
 * Data model (Eq. 1, reduced to one pixelised sky and no beam):
 *     d_t = g P_t m + n_corr,t + n_w,t,
 *     P_t m = T[p_t] + Q[p_t] cos 2psi_t + U[p_t] sin 2psi_t,
 * where p_t is a HEALPix pixel and psi_t the centre 2 pi (b_t + 1/2)/n_psi of
 * a quantised polarisation-angle bin b_t (section 4.1, n_psi = 4096).
 *
 * Conventions shared by every call
 * --------------------------------
 * Segment: one (scan, detector) pair -- the paper's comm_detscan (Listing of
 *   the TOD classes, section 3.3) -- with n_s samples.  All per-sample arrays
 *   are flat: segment s occupies [seg_off[s], seg_off[s+1]).
 * Band: one frequency channel with its own nside, sampling rate and map.
 *   The maps of all bands are concatenated along the pixel axis: band b's
 *   pixel p is global pixel pix_off[b] + p; npix_total = sum of npix.
 * Maps: [3][npix_total] (T block, Q block, U block), FP32 for TOD_MIXED,
 *   FP64 for TOD_PLAIN_FP64.
 * Binned accumulators: [npix_total][10] FP64, pixel-major (one record of ten
 *   per pixel, in the same pixel order as the maps):
 *   { b_T, b_Q, b_U, A_TT, A_TQ, A_TU, A_QQ, A_QU, A_UU, hits }.
 * Pointers: "device" = HIP device memory on the context's device; "host" =
 *   ordinary host memory.  The caller owns every buffer it passes; the
 *   context owns its scratch (FFT workspace, plans, task lists, graphs).
 * Streams: every call is asynchronous on the context's stream; one context
 *   serves one stream and one host thread at a time.
 * Errors: host-detectable problems return a status before any device work
 *   is queued.  Device-detected problems (corrupt Huffman stream, decoded
 *   value out of range, noise parameters outside their domain, non-finite
 *   data) raise a sticky device error word that tod_sync() returns as
 *   TOD_ECORRUPT; it stays set until tod_clear_error().
 *   tod_last_error() describes the last failure.
 * Precision: TOD_MIXED runs projection, residuals, FFTs and draws in FP32
 *   and keeps per-pixel accumulation and the 3x3 solve in FP64, as it keeps
 *   every per-segment sum and scalar recurrence of the gain, noise and masked
 *   draws; TOD_PLAIN_FP64 runs everything in FP64 (the TOD d may still be
 *   FP32).
 *
 * Entry points by Gibbs step: decode_pointing, decode_tod, decode_flags
 * (compressed data, section 4.1); project_sky (Eq. 1); sample_gain (Eq. 3);
 * sample_ncorr and sample_ncorr_masked (Eq. 4); sample_noise (Eq. 5);
 * bin_tod and solve_maps (binning, section 2.4); tod_chisq and
 * tod_chisq_backward (the likelihood and its adjoint); tod_sweep (decode,
 * projection, n_corr draw and binning fused for one Gibbs iteration).
 */
#ifndef C3TOD_H
#define C3TOD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tod_ctx_s *tod_ctx;

typedef enum {
    TOD_OK = 0,
    TOD_EINVAL = 1,     /* bad argument, detected on the host before any launch */
    TOD_ENOMEM = 2,     /* device allocation of context scratch failed */
    TOD_EHIP = 3,       /* a HIP runtime call failed */
    TOD_ECORRUPT = 4,   /* sticky device error: corrupt stream / value out of range */
    TOD_ENOTSUP = 5     /* unsupported size (e.g. FFT length beyond the plan limits) */
} tod_status;

typedef enum { TOD_PLAIN_FP64 = 0, TOD_MIXED = 1 } tod_prec;
typedef enum { TOD_F32 = 0, TOD_F64 = 1 } tod_dtype;

/* One frequency band (host struct).  npsi must be 4096 (section 4.1). */
typedef struct {
    int32_t nside;
    int32_t npsi;
    int64_t npix;       /* 12 nside^2 */
    int64_t pix_off;    /* first global pixel of this band */
    double fsamp;       /* sampling rate, Hz */
} tod_band;

/* Segment table (the paper's comm_tod -> comm_scan -> comm_detscan tree,
 * flattened).  Device arrays are read by kernels; host mirrors are read when
 * planning work, so they must hold the same values. */
typedef struct {
    int32_t nseg;                /* number of (scan, detector) segments */
    int32_t nband;               /* number of bands */
    int32_t ndet;                /* number of detectors (per-detector gradients) */
    int32_t reserved;
    int64_t nsamp;               /* seg_off[nseg] */
    int64_t npix_total;          /* sum of band npix */
    const int64_t *seg_off;      /* device [nseg+1], non-decreasing, seg_off[0] = 0 */
    const int32_t *seg_band;     /* device [nseg], in [0, nband) */
    const int32_t *seg_det;      /* device [nseg], in [0, ndet) */
    const uint8_t *seg_accept;   /* device [nseg], the paper's `accept`: 0 = leave out
                                    of binning and chi^2; may be NULL (all accepted) */
    const int64_t *h_seg_off;    /* host mirror [nseg+1] */
    const int32_t *h_seg_band;   /* host mirror [nseg] */
    const tod_band *bands;       /* host [nband] */
    const int32_t *h_seg_det;    /* host mirror [nseg] of seg_det; may be NULL.  With it the
                                    binning chains a detector's segments, taken in index order
                                    as consecutive in time, over several scans (see
                                    tod_set_bin_runs); without it each segment (or pair of
                                    equal neighbours) is binned alone */
} tod_layout;

/* One Huffman-coded, sample-differenced pointing stream kind (section 4.1):
 * the pixel stream or the psi-bin stream.  All arrays are device arrays.
 * Table blob t (uint32 words, at tables[table_off[t]]):
 *   [nsym, maxlen, count[1..32], sym[0..nsym)]
 * with sym the int32 difference values in canonical code order (codes of one
 * length consecutive, first code of length L = (first(L-1) + count(L-1)) << 1).
 * Segment s's bitstream is MSB-first in words[seg_word_off[s] .. seg_word_off[s+1]),
 * zero padded.  Its first symbol is the absolute first value (d(-1) = 0).
 * Side index: chunk c of segment s (symbols [c*chunk_len, (c+1)*chunk_len))
 * starts at bit chunk_bit[seg_chunk_off[s] + c] of the segment stream and the
 * undifferenced value before it is chunk_prev[...] (0 for c = 0). */
typedef struct {
    const uint32_t *words;
    const int64_t *seg_word_off;     /* [nseg+1] */
    const int32_t *seg_table;        /* [nseg] table id of each segment */
    const uint32_t *tables;
    const int64_t *table_off;        /* [ntable+1] */
    const uint32_t *chunk_bit;       /* [nchunk] */
    const int32_t *chunk_prev;       /* [nchunk] */
    const int64_t *seg_chunk_off;    /* [nseg+1], seg_chunk_off[s+1]-seg_chunk_off[s] = ceil(n_s/chunk_len) */
    int32_t chunk_len;               /* 32 .. 4096, multiple of 32 */
    int32_t ntable;
    int64_t nwords;
    int64_t nchunk;
} tod_huff;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The stream must outlive the ctx. */
tod_status tod_ctx_create(tod_ctx *ctx, int device, void *hip_stream);
/* Free the context and its scratch (synchronises its stream first). */
tod_status tod_ctx_destroy(tod_ctx ctx);
/* Wait for the stream; return TOD_ECORRUPT if the sticky device error is set. */
tod_status tod_sync(tod_ctx ctx);
/* Clear the sticky device error word. */
tod_status tod_clear_error(tod_ctx ctx);
/* Text of the last failure on this context ("" if none).  Owned by the ctx. */
const char *tod_last_error(tod_ctx ctx);
/* Device error word bits (after tod_sync): 1 = invalid code, 2 = chunk
 * boundary mismatch, 4 = pixel out of range, 8 = psi bin out of range,
 * 16 = a non-empty segment's sigma0 is not finite and > 0, 32 = its f_knee is
 * not finite and > 0, 64 = its alpha is not finite and < 0 (the PSD
 * P(f) = sigma0^2 (f/f_knee)^alpha of Eq. 4 needs all three; every call that
 * reads them checks them on the device, and its kernels still run, giving
 * inf/NaN outputs), 128 = non-finite data: a residual d - g P m (tod_sweep)
 * or a binned d - n_corr (bin_tod, tod_sweep) at an in-range pixel. */
uint32_t tod_device_error_bits(tod_ctx ctx);

/* ------------------------------------------------------------- hot path */

/* Huffman decode + undifferencing of the pixel and psi streams (section 4.1;
 * decompression row of the resource table).  Output: pix_out[nsamp] int32
 * band-local HEALPix RING pixel, psi_out[nsamp] uint16 bin in [0, npsi).
 * Bit-exact.  Corruption is reported through the sticky error word. */
tod_status decode_pointing(tod_ctx ctx, const tod_layout *lay,
                           const tod_huff *pix, const tod_huff *psi,
                           int32_t *pix_out, uint16_t *psi_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * decode_pointing with its device scratch -- the canonical decoding tables of
 * both streams (4528 bytes per table blob) and the decode work list (16 bytes
 * per block of up to 512 chunks, built on the device) -- in one static array
 * of 16 MiB per device instead of context-owned buffers.  It calls no
 * hipMalloc/hipFree and builds no plan.  Same arguments, outputs and error
 * reporting as decode_pointing; TOD_ENOTSUP (before any launch) when the
 * tables and work list exceed the 16 MiB (the 70 GHz-like set of 600 table
 * blobs and 9.35e8 samples needs 3.5 MiB).  Every call on a device shares
 * that device's array and rewrites what it uses: calls on one stream are
 * ordered, calls that overlap on one device (other streams or contexts) race. */
tod_status decode_pointing_noalloc(tod_ctx ctx, const tod_layout *lay,
                                   const tod_huff *pix, const tod_huff *psi,
                                   int32_t *pix_out, uint16_t *psi_out);

/* Compressed TOD and flag streams (section 4.1: TOD and flags are integers
 * by nature (ADC output), differenced sample by sample and Huffman coded like
 * the pointing; Table 1 lists their compression).  Same stream format, side
 * index and error reporting as decode_pointing; one stream per call.
 * decode_tod: d_out[t] = quantum * x_t (x_t the undifferenced integer), device
 * [nsamp] FP32 (mixed) or FP64 (plain).
 * decode_flags: flags_out[t] = x_t (device [nsamp] uint32, may be NULL) and
 * mask_out[t] = (x_t & flag_mask) == 0 (device [nsamp] uint8, may be NULL):
 * the mask input of sample_ncorr_masked.  At least one output. */
tod_status decode_tod(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                      const tod_huff *tod, double quantum, void *d_out);
tod_status decode_flags(tod_ctx ctx, const tod_layout *lay, const tod_huff *flags,
                        uint32_t flag_mask, uint32_t *flags_out, uint8_t *mask_out);

/* Projection s = g P m (Eq. 1; pointing matrix as pixel + psi streams,
 * section 2.1).  pix/psi: device [nsamp] as produced by decode_pointing.
 * maps: device [3][npix_total] FP32 (mixed) or FP64 (plain).  gain: device
 * [nseg] FP64.  s_out: device [nsamp] FP32 (mixed) or FP64 (plain); NaN where
 * pix is out of range for the segment's band.  Samples are visited in strided
 * tiles of the band's revisit period: a band with no period set
 * (tod_set_bin_stride) or tuned (tod_autotune) has it probed from pix on the
 * first call, which waits for the stream.  Workspace: npix_total records of
 * four values, held by the context. */
tod_status project_sky(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                       const int32_t *pix, const uint16_t *psi,
                       const void *maps, const double *gain, void *s_out);

/* Correlated-noise draw n_corr <- P(n_corr | d, g, xi_n, sky) (Eq. 4) as a
 * Fourier-domain constrained realisation on the mirrored segment (section 4.2):
 *   r = d - s;  e = [r, reverse(r), r_0 ...] of length N = smallest even
 *   5-smooth >= 2n;  R = FFT(e)/sqrt(N);  with P_k = sigma0^2 (f_k/f_knee)^alpha,
 *   f_k = k fsamp/N, 1/P_0 = 0:
 *   nhat_k = (R_k/sigma0^2 + W1_k/sigma0 + W2_k P_k^-1/2) / (1/sigma0^2 + 1/P_k);
 *   n_corr = first n samples of the unitary inverse FFT of nhat.
 * W1, W2: unit complex normals (real at k = 0 and N/2) from Philox4x32-10 with
 *   key = (seed & 0xffffffff, segment), counter = (k, iter lo, iter hi, seed hi),
 *   u = (x + 1/2) 2^-32 and Box-Muller on (u0,u1), (u2,u3).  mean_only != 0
 *   sets W = 0 (the Wiener-filter mean).
 * d: device [nsamp] of d_dtype; s: device [nsamp] (FP32 mixed / FP64 plain);
 * sigma0, fknee, alpha: device [nseg] FP64 with sigma0 > 0, fknee > 0,
 * alpha < 0 (device memory, so checked on the device: error bits 16/32/64).
 * ncorr_out: device [nsamp] (FP32 mixed / FP64 plain). */
tod_status sample_ncorr(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                        const void *d, tod_dtype d_dtype, const void *s,
                        const double *sigma0, const double *fknee, const double *alpha,
                        uint64_t seed, uint64_t iter, int mean_only, void *ncorr_out);

/* Gain draw g <- P(g | d, xi_n, sky) per segment (Eq. 3: the gain step comes
 * before n_corr and does not condition on it, so the correlated noise joins
 * the white noise in N; section 4.2 counts its FFTs with the n_corr step).
 * With the sky template t = P m at unit gain and K x = first n samples of
 * F^H diag(h) F ext(x) on sample_ncorr's extension, h_k = 1/(sigma0^2 + P_k),
 * h_0 = 0:
 *   A = t . K t,  B = t . K d  (FP64 sums),  g = B/A + eta/sqrt(A),
 * eta the Box-Muller z0 of the segment's Philox stream (key as sample_ncorr)
 * at counter (2^32-1, iter lo, iter hi, seed hi); mean_only != 0: eta = 0.
 * Flat prior, no smoothing across scans.
 * t: device [nsamp] (FP32 mixed / FP64 plain), e.g. project_sky with unit
 * gains; d: device [nsamp] of d_dtype; sigma0/fknee/alpha: device [nseg] FP64.
 * gain_out: device [nseg] FP64 (NaN where A <= 0, e.g. empty segments);
 * sigma_out: device [nseg] FP64, 1/sqrt(A) (may be NULL).
 * Workspace: two [nsamp] vectors of the precision's type, held by the
 * context. */
tod_status sample_gain(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                       const void *d, tod_dtype d_dtype, const void *t,
                       const double *sigma0, const double *fknee, const double *alpha,
                       uint64_t seed, uint64_t iter, int mean_only,
                       double *gain_out, double *sigma_out);

/* Noise-parameter draw xi_n <- P(xi_n | d, g, n_corr, sky) per segment (Eq. 5:
 * after n_corr; only low-volume spectrum data are involved, section 5):
 * 1. sigma0^2 = S / X, S = sum (d - g t - n_corr)^2 (FP64), X the chi^2_n
 *    variate n (1 - 2/(9n) + z0 sqrt(2/(9n)))^3 (prior flat in ln sigma0);
 * 2. I_k = |FFT(e(n_corr))_k|^2 / N, k = 1..N/2, on sample_ncorr's extension,
 *    summed into log-frequency bins b(k) (k < 8: b = k - 1; else with
 *    e = floor(log2 k): b = 7 + 8 (e - 3) + (k >> (e - 3)) - 8), J_b, count
 *    c_b, f_b = (f_samp/N) exp(mean ln k); binned Whittle likelihood
 *    ln L = -sum_b (J_b / P_b + c_b ln P_b), P_b = sigma0^2 (f_b / f_knee)^alpha;
 * 3. alpha = alpha_hat + z1 / sqrt(H): the maximiser of ln L in alpha at the
 *    input f_knee and the new sigma0 (ln L is concave in alpha), H = -d2 lnL;
 * 4. f_knee = u^(1/alpha), u = G sigma0^2 / sum_b J_b f_b^-alpha,
 *    G = K (1 - 1/(9K) + z2 / (3 sqrt K))^3, K = N/2 (prior flat in ln f_knee).
 * z0..z2: Box-Muller normals of the segment's Philox stream (key as
 * sample_ncorr) at counter (2^32-2, iter lo, iter hi, seed hi); mean_only != 0
 * sets them to 0.  The periodogram's FFT runs in the precision's type, all
 * sums and the sampler in FP64.
 * t: device [nsamp] sky template at unit gain (FP32 mixed / FP64 plain);
 * gain: device [nseg] FP64; ncorr: device [nsamp] (FP32 mixed / FP64 plain);
 * fknee_in: device [nseg] FP64 (the current f_knee, conditioned on by the
 * alpha step).  Outputs: device [nseg] FP64 each (may alias fknee_in); NaN for
 * empty segments.  The bin sums use FP64 atomics: their last bits may vary
 * from call to call. */
tod_status sample_noise(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                        const void *d, tod_dtype d_dtype, const void *t,
                        const double *gain, const void *ncorr, const double *fknee_in,
                        uint64_t seed, uint64_t iter, int mean_only,
                        double *sigma0_out, double *fknee_out, double *alpha_out);

/* Correlated-noise draw with a processing mask (gap filling: the constrained
 * realisation needs FFTs inside a CG solver where scans cross masked sky,
 * section 5 and the correlated-noise row of Table 2).  On the extension and
 * spectrum of sample_ncorr, with mu = [m, reverse(m), 1 ...] the extended mask
 * and F the unitary DFT, each segment's draw is x[0:n], x = A^-1 b:
 *   A = F^H diag(1/P) F + diag(mu)/sigma0^2,
 *   b = mu (e/sigma0^2 + F^H W1/sigma0) + F^H (W2 P^-1/2)   (W as sample_ncorr).
 * Solver: with M = F^H diag(1/(1/sigma0^2 + 1/P)) F and S the masked extended
 * positions, x = x0 + M S y, x0 = M b, (sigma0^2 I - S^T M S) y = S^T x0
 * (Woodbury), by CG from y = 0 on the masked positions only; it stops when
 * the residual (b - A x, which lives on the masked positions) has fallen to
 * tol times its value at x0, or after max_iter iterations.  With nothing
 * masked x = x0 is sample_ncorr's draw and no iteration runs.
 * mask: device [nsamp] uint8, nonzero = sample used (decode_flags writes
 * one).  Transforms and full-length vectors use the precision's type; the
 * masked-position vectors, every sum and the recurrences are FP64; x0's
 * drawn term is added per Fourier mode.  tol 1e-6 reaches the FP32 floor
 * (about 1e-6 relative).
 * iters_out: device [nseg] int32 (may be NULL): iterations per segment,
 * negated where max_iter stopped it first (0: nothing masked).
 * Workspace (context): four sweep-wide vectors of the extended length in
 * the precision's type, and per masked extended position an index and three
 * FP64 values. */
tod_status sample_ncorr_masked(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                               const void *d, tod_dtype d_dtype, const void *s,
                               const uint8_t *mask,
                               const double *sigma0, const double *fknee, const double *alpha,
                               uint64_t seed, uint64_t iter, int mean_only,
                               double tol, int max_iter,
                               void *ncorr_out, int32_t *iters_out);

/* Binning into per-pixel P^T N^-1 d and P^T N^-1 P (section 2.4: co-added on
 * the fly during the TOD loop; binning row of the resource table): with
 * w = g/sigma0^2, v = d - n_corr, (c, s) = (cos 2psi, sin 2psi):
 *   b_p += w v (1, c, s),  A_p += g w (1, c, s)^T (1, c, s),  hits_p += 1.
 * acc: device [npix_total][10] FP64 (pixel-major).  accumulate = 0 zeroes acc first.
 * ncorr may be NULL (v = d).  Segments with accept = 0 are skipped. */
tod_status bin_tod(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                   const int32_t *pix, const uint16_t *psi,
                   const void *d, tod_dtype d_dtype, const void *ncorr,
                   const double *gain, const double *sigma0,
                   double *acc, int accumulate);

/* Per-pixel map solve m_p = A_p^-1 b_p in FP64 with the condition number
 * rcond_p = lambda_min / lambda_max of A_p; pixels with hits < 3 or
 * rcond < rcond_min get NaN.  acc: device [npix][10]; map_out: device
 * [3][npix] of map_dtype; rcond_out: device [npix] FP64 (may be NULL). */
tod_status solve_maps(tod_ctx ctx, int64_t npix, const double *acc, double rcond_min,
                      void *map_out, tod_dtype map_dtype, double *rcond_out);

/* chi^2 per segment (the likelihood evaluation of the TOD step):
 *   J_s = sum_t r_t^2/sigma0^2 + sum_{k=1}^{N/2} (I_k/P_k + ln P_k),
 *   r = d - g P m - n_corr,  I_k = |FFT(e(n_corr))_k|^2 / N on the same
 *   mirrored extension and N as sample_ncorr.
 * pix, psi: device [nsamp]; d: device [nsamp] of d_dtype; ncorr: device
 * [nsamp] (FP32 mixed / FP64 plain, required); maps: device [3][npix_total]
 * of the precision's type; gain, sigma0, fknee, alpha: device [nseg] FP64.
 * chisq_seg: device [nseg] FP64 (0 for rejected segments).  Samples whose
 * pixel is out of range for their band are left out of the time-domain sum.
 * The time-domain terms walk strided tiles of the band's revisit period
 * (probed from pix on the first call when not set or tuned, which waits for
 * the stream).  Workspace: npix_total records of four values, held by the
 * context. */
tod_status tod_chisq(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                     const int32_t *pix, const uint16_t *psi,
                     const void *d, tod_dtype d_dtype, const void *ncorr,
                     const void *maps, const double *gain,
                     const double *sigma0, const double *fknee, const double *alpha,
                     double *chisq_seg);

/* Adjoint of tod_chisq, scaled by dL/dJ = grad_scale * (*grad_scale_dev)
 * (grad_scale_dev: device FP64 scalar, may be NULL = 1; read by the kernels,
 * so an autograd caller passes its incoming gradient without a host sync):
 *   dJ/dm = -2 P^T (g r / sigma0^2)                       -> grad_maps [3][npix_total] FP64
 *   dJ/dg_s = -2 sum_t (P m)_t r_t / sigma0^2             -> grad_gain [nseg]
 *   dJ/dsigma0 = -2 sum r^2/sigma0^3 + sum_k (2/sigma0)(1 - I_k/P_k)
 *   dJ/df_knee = sum_k (1 - I_k/P_k)(-alpha/f_knee)
 *   dJ/dalpha  = sum_k (1 - I_k/P_k) ln(f_k/f_knee)
 * the last three summed over each detector's segments -> [ndet] arrays.
 * All outputs are device FP64 and are overwritten.  Any of them may be NULL. */
tod_status tod_chisq_backward(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                              const int32_t *pix, const uint16_t *psi,
                              const void *d, tod_dtype d_dtype, const void *ncorr,
                              const void *maps, const double *gain,
                              const double *sigma0, const double *fknee, const double *alpha,
                              double grad_scale, const double *grad_scale_dev,
                              double *grad_maps, double *grad_gain,
                              double *grad_sigma0, double *grad_fknee, double *grad_alpha);

/* One fused TOD sweep: decode -> project -> n_corr draw -> binning (the
 * decompress / project / correlated-noise / bin rows of the TOD loop).
 * Writes ncorr_out [nsamp] (FP32 mixed / FP64 plain), zeroes and fills acc
 * [npix_total][10].  pix_work/psi_work: device [nsamp] scratch that receives
 * the decoded pointing.  use_graph != 0 captures the sweep's kernels into a
 * hipGraph on the first call with a given set of arguments and replays it
 * afterwards (seed and iter are read from device memory, so they may change
 * between replays). */
tod_status tod_sweep(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                     const tod_huff *pix, const tod_huff *psi,
                     const void *d, tod_dtype d_dtype, const void *maps,
                     const double *gain, const double *sigma0,
                     const double *fknee, const double *alpha,
                     uint64_t seed, uint64_t iter,
                     void *ncorr_out, double *acc,
                     int32_t *pix_work, uint16_t *psi_work, int use_graph);

/* tod_sweep with the TOD taken from its Huffman-compressed stream (section
 * 4.1: TOD samples are integers, differenced and coded like the pointing;
 * Table 1): the sweep decodes it right after the pointing into d_work as
 * quantum * x (device [nsamp], FP32 mixed / FP64 plain; bit-exact, as
 * decode_tod), and the residual and the binning read it there.  Other
 * arguments, outputs and graph capture as tod_sweep. */
tod_status tod_sweep_stream(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                            const tod_huff *pix, const tod_huff *psi,
                            const tod_huff *tod, double quantum, void *d_work,
                            const void *maps, const double *gain, const double *sigma0,
                            const double *fknee, const double *alpha,
                            uint64_t seed, uint64_t iter,
                            void *ncorr_out, double *acc,
                            int32_t *pix_work, uint16_t *psi_work, int use_graph);

/* --------------------------------------------------------- planning/tuning */

/* Plan a layout ahead of its first call (the measured-cost-table step of
 * section 4.2, done once per data set): load FFT choices and binning strides
 * from tune_cache when it is given (a file written by tod_autotune; missing
 * file: defaults), then build the layout's FFT plans, task lists and twiddle
 * tables and size the FFT workspace in the context.  Later calls with the same
 * layout and precision reuse them.  Every entry point plans on first use
 * anyway; this call moves that host work and its allocations up front. */
tod_status tod_plan(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const char *tune_cache);

/* Measure candidate FFT splits for every FFT length the layout needs (section
 * 4.2's measured cost table, here per length: the split M = M1 x M2, the
 * column kernel -- whole columns in registers for a compiled M1, or LDS
 * tiles -- and the radix order) and the binning stride, keep the fastest in
 * the context, and (if cache_path != NULL) write them to a JSON cache file.
 * Needs the decoded pointing (pix) for the binning probe; may be NULL to skip
 * it. */
tod_status tod_autotune(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                        const int32_t *pix, const char *cache_path);
/* Load plans from a JSON cache written by tod_autotune (missing file: OK;
 * unreadable file: TOD_EINVAL).  A cached split is used only where the
 * kernels can run it (its factors multiply out, its column kernel exists,
 * every radix has a compiled stage); otherwise the default split is used. */
tod_status tod_load_tuning(tod_ctx ctx, const char *cache_path);
/* Binning stride (samples between revisits of a pixel) per band; 0 = let the
 * library choose, at most 2^26.  Correct for any value; only speed depends on
 * it.  A stride longer than a segment acts as the segment's length. */
tod_status tod_set_bin_stride(tod_ctx ctx, int32_t band, int32_t stride);

/* Binning runs: the binning kernel gives each lane one phase of the revisit
 * period (the spin phase, counted from the start of a detector's first segment)
 * and walks it through `scans` consecutive scans of one detector pair before
 * flushing its per-pixel sums, so the nearly coinciding rings of consecutive
 * scans share the flushes (section 2.4: binned on the fly, synchronised once).
 * Needs h_seg_det in the layout.  scans = 0: chosen per layout (as many as keep
 * about 4096 blocks), 1..16: fixed.  Correct for any value. */
tod_status tod_set_bin_runs(tod_ctx ctx, int32_t scans);

/* FFT work batching: the column/row passes run batch by batch over groups of
 * segments whose complex workspace totals at most complex_elems (0 = all
 * segments in one batch).  Smaller batches keep the intermediate spectrum in
 * the device's last-level cache between passes; results do not depend on it. */
tod_status tod_set_fft_batch(tod_ctx ctx, int64_t complex_elems);

/* Per-kernel timing.  While enabled, every launch the context makes outside
 * graph capture is bracketed by HIP events on the context stream (the sweep
 * then runs eagerly).  tod_kernel_times synchronises the stream, returns the
 * summed milliseconds and launch counts since the previous read and resets
 * them.  Kernel ids (arrays of 11): 0 decode, 1 projection, 2 FFT forward
 * column pass, 3 FFT row pass (filter + draw, Whittle sums, the masked and
 * gain draws' Fourier-diagonal filters, or periodogram bins), 4 FFT inverse
 * column pass, 5 binning, 6 per-pixel solve, 7 chi^2 time-domain terms, 8 the
 * masked draw's CG vector updates and reductions, 9 the gain draw's sums and
 * draw, 10 the noise-parameter draw's sums and sampler. */
tod_status tod_enable_timing(tod_ctx ctx, int enable);
tod_status tod_kernel_times(tod_ctx ctx, double *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* C3TOD_H */
