// Internal declarations shared by the c3tod kernels and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/c3tod.h"

#define C3_NT 256            // threads per block of every kernel but the two below
#define C3_DEC_NT 512        // threads per block of the decoders: one side-index chunk each
#define C3_ROW_NT_F32 512    // threads per block of the FFT row pass (two blocks per CU)
#define C3_ROW_NT_F64 1024
#define C3_COL_NT 64         // threads (= columns) per block of the register column passes
#define C3_LDS_MAX 163840    // LDS bytes one workgroup may hold on gfx950

// radices of the row-pass stages: 5-smooth, and small enough that a stage's
// butterflies per thread fit the register budget of two row blocks per CU
#define C3_ROW_RADICES_F32(X) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(20) X(24) X(25) X(27)
#define C3_ROW_RADICES_F64(X) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10)

// column lengths M1 with register column kernels (5-smooth, 16..100; FP32 only)
#define C3_COLREG_LIST(X) \
    X(16) X(18) X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(50) X(54) X(60) X(64) X(72) X(75) X(80) X(81) \
        X(90) X(96) X(100)

// sticky device error bits
#define C3_ERR_CODE 1u       // bit pattern matches no code
#define C3_ERR_CHUNK 2u      // chunk end does not meet the next chunk's start
#define C3_ERR_PIX 4u        // decoded pixel outside [0, npix)
#define C3_ERR_PSI 8u        // decoded psi bin outside [0, npsi)
#define C3_ERR_SIGMA0 16u    // a non-empty segment's sigma0 is not finite and > 0
#define C3_ERR_FKNEE 32u     // a non-empty segment's f_knee is not finite and > 0
#define C3_ERR_ALPHA 64u     // a non-empty segment's alpha is not finite and < 0
#define C3_ERR_NONFINITE 128u  // a residual d - g P m or a binned d - n_corr is not finite

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// Per-segment record built on the host for every kernel that walks segments.
struct SegInfo {
    int64_t samp_off;    // first sample
    int64_t scr_off;     // first complex element of the FFT workspace (ncorr/chisq)
    int32_t n;           // samples
    int32_t plan;        // FFT plan index (-1: none)
    int32_t band;
    int32_t det;
    int32_t accept;
    int32_t pad;
    int64_t ext_off;     // first complex element of the segment's whole extended vector
                         // (N = 2M reals) in sweep-wide vectors (masked n_corr solver)
};

// FFT plan of one complex length M = M1 * M2 (the real length is N = 2M).
#define C3_MAXRAD 16
struct FftPlan {
    int32_t M, M1, M2, B;        // B: columns per column-pass tile
    int32_t nr1, nr2;            // radix counts of the M1 and M2 sub-transforms
    int32_t colreg;              // 1: column passes keep a whole column in registers (M1 fixed
                                 //    at compile time); 0: LDS column tiles of B columns
    int32_t pad;
    int8_t r1[C3_MAXRAD];
    int8_t r2[C3_MAXRAD];
    int64_t tw1;                 // offset of w_M1^m (m < M1) in the twiddle pool
    int64_t tw2;                 // offset of w_M2^m (m < M2)
    int64_t twlo;                // w_N^m, m < 1024           (N = 2M)
    int64_t twhi;                // w_N^(1024 h), h < N/1024 + 1
    int64_t twr;                 // compiled row length M2 (rowc.h): its stage twiddles, -1 if none
    int64_t twh;                 //   and w_(2 M2)^j, j < M2 (the mode loop's twiddle), -1 if none
};

// Column-pass work item: columns [c0, c0 + tile) of one segment's transform,
// with the segment's offsets and sizes, so that a block can issue its column
// loads as soon as it has read its task.
struct ColTask {
    int64_t samp_off;    // first sample
    int64_t scr_off;     // first complex element of the FFT workspace
    int64_t ext_off;     // first complex element of the whole extended vector
    int32_t seg, c0;
    int32_t n;           // samples
    int32_t M2;          // row length of the split
    int32_t pad[2];
};

// Row-pass work item: rows k1 and M1 - k1 of one segment's transform, with
// the workspace offsets (complex elements) of both rows, so that a block can
// issue its row loads as soon as it has read its task.
struct RowTask {
    int64_t off_a;       // row k1
    int64_t off_b;       // row (M1 - k1) mod M1
    int32_t seg, k1;
    int32_t pad[2];
};

// Context-side view of the layout kept on the device.
struct BandDev {
    int64_t npix;
    int64_t pix_off;
    double fsamp;
    int32_t npsi;
    int32_t nside;
};

#define C3_MAXBAND 16
#define C3_XI_NBIN 231       // periodogram bins of modes k = 1 .. 2^31 - 1 (noise-parameter draw)

struct LayoutDev {
    const int64_t *seg_off;
    const int32_t *seg_band;
    const int32_t *seg_det;
    const uint8_t *seg_accept;
    int32_t nseg, nband, ndet, pad;
    int64_t nsamp, npix_total;
    BandDev band[C3_MAXBAND];
};

// Device-side Huffman stream (copy of tod_huff, by value into kernels).
struct HuffDev {
    const uint32_t *words;
    const int64_t *seg_word_off;
    const int32_t *seg_table;
    const uint32_t *tables;
    const int64_t *table_off;
    const uint32_t *chunk_bit;
    const int32_t *chunk_prev;
    const int64_t *seg_chunk_off;
    int32_t chunk_len;
    int32_t ntable;
};

// Canonical decoding table of one Huffman table blob, built on the device per
// decode call (section 4.1 codes; canonical form of the encoder's lengths).
#define C3_KLUT 12
struct alignas(16) DecTab {
    unsigned long long lim[34];  // left-justified limits (first_L + count_L) << (32 - L)
    int32_t delta[34];           // off_L - first_L: symbol index = code + delta[L]
    int32_t minlen, maxlen;
    int32_t nsym;                // symbols with a code (sum of the counts)
    int32_t ok;                  // 0: the table blob is not a valid prefix code
    uint8_t lut[1 << C3_KLUT];   // code length shared by every code with this 12-bit
                                 // prefix; 64 | the shortest if it holds several
                                 // lengths; 0 if no code starts it
    int32_t pad[2];
};

// Decode work item: one block decodes up to C3_NT consecutive chunks of one segment.
struct DecodeTask {
    int32_t seg;
    int32_t chunk0;   // first chunk (segment-local)
    int32_t nchunk;   // chunks in this task (<= C3_DEC_NT)
    int32_t pad;
};

// ------------------------------------------------------------ launchers
// Implemented in the .hip files; all return hipError_t of the launch.
namespace c3 {

// Static device scratch of decode_pointing_noalloc (bytes per device), laid
// out as ntable DecTab records then the DecodeTask list
#define C3_NOALLOC_BYTES (16u << 20)
#define C3_MAX_DEVICES 64
inline int64_t noalloc_task_offset(int64_t ntable) {
    return (ntable * (int64_t)sizeof(DecTab) + 255) / 256 * 256;
}
// address of this device's static scratch (the current device); looked up
// once per device with hipGetSymbolAddress
hipError_t noalloc_scratch(void **ptr);
// decode_pointing's kernels with the tables and a device-built work list of
// ntask entries in the static scratch at scratch_ptr
hipError_t launch_decode_noalloc(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                                 void *scratch_ptr, int ntask, int32_t *pix_out, uint16_t *psi_out,
                                 uint32_t *err);

// tabs: workspace of hp.ntable + hs.ntable DecTab records (pixel tables first)
hipError_t launch_decode(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                         DecTab *tabs, const DecodeTask *tasks, int ntask, int32_t *pix_out,
                         uint16_t *psi_out, uint32_t *err);

// one integer stream (TOD or flags): kind 0 writes FP32 quantum * x, 1 FP64
// quantum * x, 2 the uint32 flag words (out may be NULL) and, if mask_out, the
// byte (x & flag_mask) == 0; tabs: workspace of h.ntable DecTab records
hipError_t launch_decode_stream(hipStream_t st, const LayoutDev &L, const HuffDev &h, DecTab *tabs,
                                const DecodeTask *tasks, int ntask, int kind, double quantum,
                                uint32_t flag_mask, void *out, uint8_t *mask_out, uint32_t *err);

// r = d - g P m on strided tiles (the sweep's residual, input of the n_corr FFTs),
// or s = g P m when d is NULL; maps4: workspace of npix_total records of 4
// values (T, Q, U, 0), filled from the [3][npix] maps first
// trig: the cos/sin 2psi table of the precision's type; err: sticky word that
// receives C3_ERR_NONFINITE where d - s is not finite at an in-range pixel
// (may be NULL)
hipError_t launch_resid_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                              int ntile, const int32_t *pix, const uint16_t *psi, const void *d,
                              int d_f64, const void *maps, void *maps4, const double *gain,
                              const void *trig, void *r_out, uint32_t *err);
// per non-empty segment: sigma0 > 0, f_knee > 0, alpha < 0, all finite (any
// pointer may be NULL: not checked); failures set C3_ERR_SIGMA0 / _FKNEE /
// _ALPHA in the sticky word.  The kernels that use them still run.
hipError_t launch_check_params(hipStream_t st, const LayoutDev &L, const double *sigma0,
                               const double *fknee, const double *alpha, uint32_t *err);

// FFT-based passes (modes: see launch_fft_pass)
struct FftArgs {
    const SegInfo *segs;
    const FftPlan *plans;
    const void *twpool;         // cx<T> pool
    void *work;                 // cx<T> workspace
    const ColTask *col_tasks;
    int ncol_tasks;
    const RowTask *row_tasks;
    int nrow_tasks;
    const void *in_a;           // pass-1 input: r = in_a - in_b (in_b may be NULL)
    int in_a_f64;
    const void *in_b;
    int in_b_f64;
    void *out;                  // pass-3 output
    const double *sigma0, *fknee, *alpha;
    const double *fsamp_band;   // [nband]
    const uint64_t *seed_iter;  // device {seed, iter}
    int mean_only;
    int mode;
    double *whittle;            // mode 1: per-segment sums [nseg][4]
    int col_lds, row_lds;       // dynamic LDS bytes of the column and row passes
    int full_io;                // 1: pass 1 reads, pass 3 writes whole extended vectors
                                //    (N reals per segment at real offset 2 ext_off of
                                //    in_a / out) instead of the mirrored segment / its crop
    int which;                  // mode 2: filter 0: 1/P, 1: 1/(1/sigma0^2 + 1/P),
                                //         2: 1/(sigma0^2 + P), 3: as 1 plus the drawn
                                //         term (1/(1/sigma0^2 + 1/P)) W2 sqrt(1/P);
                                // mode 3: 0 spectrum W1, 1 spectrum W2 sqrt(1/P)
    const int32_t *active;      // per segment, 0: skip (NULL: every segment runs)
    double *bins;               // mode 4: periodogram bins [nseg][C3_XI_NBIN], added to
};
// pass 0: forward column FFTs; 1: row pass (mode 0 n_corr draw, 1 Whittle sums,
// 2 Fourier-diagonal filter, 3 inverse transform of a drawn spectrum: no
// forward transform, no input, 4 periodogram summed into log-frequency bins:
// no inverse transform); 2: inverse column FFTs.  m1reg > 0 selects the
// register column kernels for that column length (passes 0 and 2); 0 the LDS
// column tiles.
hipError_t launch_fft_pass(hipStream_t st, int prec_mixed, const FftArgs &a, int pass, int m1reg);
// register column kernels (fftcol.hip); returns hipErrorInvalidValue for a
// column length without a compiled kernel
hipError_t launch_fft_col_reg(hipStream_t st, int prec_mixed, const FftArgs &a, int pass, int m1);
bool fft_col_reg_supported(int prec_mixed, int m1);
// row kernels compiled per row length (rowc.hip): FP32, modes 0, 1, 2 and 4, the
// two-row tasks (0 < k1 < M1/2) of plans whose M2 is compiled
bool rowc_supported(int prec_mixed, int L, int mode);
hipError_t launch_rowc(hipStream_t st, const FftArgs &a, int L);
hipError_t rowc_init_attributes();
// raise the dynamic LDS limit of the FFT kernels (once per process)
hipError_t fft_init_attributes();

// tiles and runs: the binning runs (get_bin_runs); err receives C3_ERR_NONFINITE
hipError_t launch_bin_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                            int ntile, const int2 *runs, const int32_t *pix, const uint16_t *psi,
                            const void *d, int d_f64, const void *ncorr, const double *gain,
                            const double *sigma0, const void *trig64, double *acc, uint32_t *err);
hipError_t launch_zero(hipStream_t st, void *p, int64_t bytes);
hipError_t launch_solve(hipStream_t st, int64_t npix, const double *acc, double rcond_min,
                        void *map_out, int map_f64, double *rcond_out);
hipError_t launch_repeat_probe(hipStream_t st, const int32_t *pix, int64_t off, int n, int maxlag,
                               unsigned long long *counts);

// chi^2 time-domain part on strided tiles: per segment sum r^2/sigma0^2 (-> seg_sums[4s]),
// sum (Pm) r (-> [4s+1]), sum r^2 (-> [4s+2]); with grad_maps4 != NULL also the map adjoint,
// added to grad_maps4: npix_total records (T, Q, U, unused) of FP64, zeroed by the caller.
// maps4: workspace of npix_total records (T, Q, U, 0), filled from the [3][npix] maps first.
hipError_t launch_chisq_time_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                                   int ntile, const int32_t *pix, const uint16_t *psi,
                                   const void *d, int d_f64, const void *ncorr, const void *maps,
                                   void *maps4, const double *gain, const double *sigma0,
                                   const void *trig64, double *seg_sums, double *grad_maps4,
                                   double grad_scale, const double *gscale_dev);
// grad_maps [3][npt] from the records of grad_maps4
hipError_t launch_gmap_out(hipStream_t st, int64_t npt, const double *grad_maps4, double *grad_maps);
hipError_t launch_chisq_finish(hipStream_t st, const LayoutDev &L, const double *seg_time,
                               const double *seg_whittle, const double *gain, const double *sigma0,
                               const double *fknee, const double *alpha, double grad_scale,
                               const double *gscale_dev, double *chisq_seg, double *grad_gain, double *grad_sigma0,
                               double *grad_fknee, double *grad_alpha);
hipError_t launch_set_u64(hipStream_t st, uint64_t *p, uint64_t a, uint64_t b);

// ---- masked n_corr draw (gapfill.hip): per-segment CG state and vector passes
#define C3_CG_TILE 4096      // entries per elementwise tile (extended reals or gap entries)
struct CgState {
    double bb;       // rho_0 . rho_0: the stopping rule's reference
    double alpha, beta;
    double rr;       // rho . rho of the current residual
    int32_t iters;   // CG iterations done
    int32_t converged;
};
enum CgStep { CG_RZ0 = 0, CG_ALPHA, CG_RES };
enum CgOp {
    CG_OP_INIT = 0,     // mu u -> res (b without its F^H W2 term)     (extended tiles)
    CG_OP_GAP_COUNT,    // masked positions per extended tile -> cnt  (extended tiles)
    CG_OP_GAP_FILL,     // their global extended indices -> gap_idx   (extended tiles)
    CG_OP_GAP_START,    // y = 0, rho = p = x0[gap], partial rho.rho  (gap tiles)
    CG_OP_GAP_SCATTER,  // fin[gap] = scatter_src                     (gap tiles)
    CG_OP_GAP_PQ,       // partial p.q, q = sigma0^2 p - fout[gap]    (gap tiles)
    CG_OP_GAP_UPDATE,   // y += alpha p, rho -= alpha q, partial rho.rho (gap tiles)
    CG_OP_GAP_DIR,      // p = rho + beta p, fin[gap] = p             (gap tiles)
    CG_OP_CROP          // out = (x0 + fout)[0:n]                     (sample tiles)
};
struct CgVecArgs {
    const int4 *tiles;          // extended tiles (seg, first real, length, 0), gap tiles
    int ntile;                  // (seg, first entry low 31 bits, length, high bits) or
                                // sample tiles, by operation
    const SegInfo *segs;
    const int32_t *act;         // per segment: still iterating
    const CgState *cs;
    const void *d;              // INIT: residual d - s and the mask (per sample)
    int d_f64;
    const void *s;
    int s_f64;                  // must match the precision (FP64 s for the plain path)
    const uint8_t *mask;        // 1: sample used, 0: masked
    const double *sigma0;
    const void *w1;             // INIT: F^H W1
    int have_draw;              // INIT: 0 for the mean only (w1 not read)
    void *x;                    // full vectors, transform type: x0 = M b
    void *res;                  //   mu u = mu (e / sigma0^2 + F^H W1 / sigma0)
    void *fin;                  //   FFT input: zero but at the masked positions
    const void *fout;           //   FFT output
    int32_t *cnt;               // masked positions per extended tile
    const int64_t *gap_base;    // their first entry in gap_idx
    int64_t *gap_idx;           // global extended index of every masked position
    double *y, *rho, *p;        // small system (FP64)
    const double *scatter_src;  // GAP_SCATTER source
    const int32_t *has_gap;     // CROP: segment has masked samples
    double *part;               // per-tile partial sums
    void *out;                  // CROP: n_corr per sample
};
hipError_t launch_cg_vec(hipStream_t st, int mixed, int op, const CgVecArgs &a);
// zero n elements of a vector of the transform type (a fill kernel)
hipError_t launch_cg_zero(hipStream_t st, int mixed, void *v, int64_t n);
// step: see CgStep; the CG_RES step counts still-active segments into *nactive
// (zeroed by the CG_ALPHA step of the same iteration)
hipError_t launch_cg_finish(hipStream_t st, int nseg, const int2 *seg_tiles, const double *part, CgState *cs,
                            int32_t *act, int step, double tol2, int max_iter, int32_t *nactive);
// iterations per segment (negative: stopped at max_iter before the tolerance)
hipError_t launch_cg_iters(hipStream_t st, int nseg, const CgState *cs, int32_t *out);

// ---- gain draw (gain.hip): per sample tile the partial sums t . K t and
// t . K d (kt, kd: the filtered template and data, first n samples of each
// segment); then per segment g = B/A + eta/sqrt(A)
hipError_t launch_gain_dots(hipStream_t st, int mixed, const int4 *tiles, int ntile, const int64_t *seg_off,
                            const void *t, const void *kt, const void *kd, double2 *part);
// ---- noise-parameter draw (noise.hip): per sample tile the partial sum of
// (d - g t - n_corr)^2; then per segment (one wave) sigma0, alpha, f_knee from
// it and the periodogram bins of the row pass (mode 4)
hipError_t launch_xi_white(hipStream_t st, int mixed, const int4 *tiles, int ntile, const int64_t *seg_off,
                           const void *d, int d_f64, const void *t, const double *gain, const void *nc,
                           double *part);
hipError_t launch_xi_sample(hipStream_t st, int nseg, const SegInfo *segs, const FftPlan *plans,
                            const int32_t *seg_band, const double *fsamp_band, const int2 *seg_tiles,
                            const double *part, const double *bins, const double *fknee_in,
                            const uint64_t *seed_iter, int mean_only, double *sigma0_out, double *fknee_out,
                            double *alpha_out);
hipError_t launch_gain_finish(hipStream_t st, int nseg, const int2 *seg_tiles, const double2 *part,
                              const uint64_t *seed_iter, int mean_only, double *gain_out, double *sigma_out);

}  // namespace c3
