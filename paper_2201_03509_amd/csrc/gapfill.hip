// Masked correlated-noise draw: the constrained realisation of n_corr when a
// processing mask removes samples (gap filling, section 5 and the correlated
// noise row of Table 2), solved by conjugate gradients on the same mirrored,
// 5-smooth padded extension as the unmasked Fourier draw.
//
// Per segment, with F the unitary DFT, 1/P_k the inverse prior spectrum
// (1/P_0 = 0), mu the extended mask ([m, reverse(m), 1 ...]) and e the
// extended residual d - s:
//     A = F^H diag(1/P) F + diag(mu) / sigma0^2,
//     b = mu (e / sigma0^2 + F^H W1 / sigma0) + F^H (W2 sqrt(1/P)).
// With M = F^H diag(1 / (1/sigma0^2 + 1/P)) F and S the selection of the
// masked extended positions, A = M^-1 - S S^T / sigma0^2, so (Woodbury)
//     x = x0 + M S y,  x0 = M b,  (sigma0^2 I - S^T M S) y = S^T x0,
// and the full residual is b - A x = S rho / sigma0^2 with rho the small
// system's residual.  CG runs on the masked positions only: one
// Fourier-diagonal product (FFT passes, row mode 2) per iteration, the
// vector work on about a tenth of the samples.  It stops when
// ||rho|| <= tol ||rho_0||: the full residual has fallen by tol from x0.
// x0 = M (mu u) + M F^H (W2 sqrt(1/P)), u = e / sigma0^2 + F^H W1 / sigma0,
// is one FFT round trip: the drawn term, large at high frequencies, is added
// per mode and never rounded in the time domain.
//
// Full vectors are sweep-wide (segment s owns reals [2 ext_off, 2 ext_off + N)
// of each) in the transform's type.  The small system's vectors (y, rho, p)
// are FP64, one entry per masked extended position, listed per segment in
// gap_idx (global extended indices, ascending).  Elementwise kernels walk
// tiles of one segment; a tile writes one partial sum, and one wave per
// segment adds its tiles' partials in a fixed order (reproducible, no atomics
// on the sums).
#include "common.h"

namespace {
using namespace c3;

// position of extended index t in the segment: the mirror of the extension;
// -1 in the pad (mask 1, value r_0)
__device__ __forceinline__ int64_t mirror(int64_t t, int n) {
    return t < n ? t : (t < 2 * (int64_t)n ? 2 * (int64_t)n - 1 - t : -1);
}

__device__ __forceinline__ bool masked_at(const uint8_t *mask, int64_t s0, int n, int64_t t) {
    const int64_t u = mirror(t, n);
    return u >= 0 && mask[s0 + u] == 0;
}

// block sum of v (C3_NT threads) -> part[blockIdx.x] by thread 0
__device__ __forceinline__ void block_sum(double v, double *part) {
    __shared__ double red[C3_NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
#pragma unroll
        for (int i = 0; i < C3_NT / 64; ++i) s += red[i];
        part[blockIdx.x] = s;
    }
}

// first entry of a gap tile: (x = seg, y = low 31 bits, z = length, w = high bits)
__device__ __forceinline__ int64_t gap_first(int4 tl) { return ((int64_t)tl.w << 31) | (uint32_t)tl.y; }

// mu u = mu (e / s0^2 + w1 / s0) -> res.  Extended reals in pairs: N and
// every tile length are even.  d of type TD, s of the precision's type T and
// the presence of the drawn term are compile-time, so a pair's loads issue
// together.
template <typename T, typename TD, bool DRAW>
__global__ __launch_bounds__(C3_NT) void k_cg_init(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                   const TD *__restrict__ d, const T *__restrict__ s,
                                                   const uint8_t *__restrict__ mask, const T *__restrict__ w1,
                                                   const double *__restrict__ sigma0, T *__restrict__ res) {
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    const double s0 = sigma0[tl.x], is2 = 1.0 / (s0 * s0), is1 = 1.0 / s0;
    const int64_t base = 2 * sg.ext_off + tl.y;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        cx<T> w = {0, 0};
        if constexpr (DRAW) w = *(const cx<T> *)(w1 + base + i);
        int64_t u[2], j[2];
        TD dv[2];
        T sv[2];
        uint8_t mk[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            u[h] = mirror(tl.y + i + h, sg.n);
            j[h] = sg.samp_off + (u[h] < 0 ? 0 : u[h]);
            dv[h] = d[j[h]];
            sv[h] = s[j[h]];
            mk[h] = mask[j[h]];
        }
        double b[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double e = (double)dv[h] - (double)sv[h];
            const double m = u[h] < 0 ? 1.0 : (double)(mk[h] != 0);
            b[h] = m * (e * is2 + (double)(h ? w.y : w.x) * is1);
        }
        *(cx<T> *)(res + base + i) = cx<T>{(T)b[0], (T)b[1]};
    }
}

// masked positions per extended tile (the tile's share of the gap list)
__global__ __launch_bounds__(C3_NT) void k_gap_count(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                     const uint8_t *__restrict__ mask, int32_t *__restrict__ cnt) {
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    int c = 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) c += masked_at(mask, sg.samp_off, sg.n, tl.y + i) ? 1 : 0;
    __shared__ int red[C3_NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int i = 0; i < C3_NT / 64; ++i) t += red[i];
        cnt[blockIdx.x] = t;
    }
}

// the tile's masked positions, ascending, from gap_idx[base[tile]]: each
// thread takes C3_CG_TILE / C3_NT consecutive positions, a block scan places them
__global__ __launch_bounds__(C3_NT) void k_gap_fill(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                    const uint8_t *__restrict__ mask, const int64_t *__restrict__ base,
                                                    int64_t *__restrict__ gap_idx) {
    constexpr int PER = C3_CG_TILE / C3_NT;
    static_assert(PER <= 32, "one bit per position in a 32-bit word");
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    const int t0 = threadIdx.x * PER;
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (t0 + k < tl.z && masked_at(mask, sg.samp_off, sg.n, tl.y + t0 + k)) bits |= 1u << k;
    const int c = __builtin_popcount(bits);
    __shared__ int scan[C3_NT];
    scan[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < C3_NT; o <<= 1) {  // inclusive Hillis-Steele scan
        const int v = threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t w = base[blockIdx.x] + scan[threadIdx.x] - c;
    const int64_t g0 = 2 * sg.ext_off + tl.y + t0;
    while (bits) {
        const int k = __builtin_ctz(bits);
        bits &= bits - 1;
        gap_idx[w++] = g0 + k;
    }
}

// rho = p = x0 at the masked positions, y = 0; partial sums of rho^2
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gap_start(const int4 *__restrict__ gtiles, const int64_t *__restrict__ gap_idx,
                                                     const T *__restrict__ x0, double *__restrict__ y,
                                                     double *__restrict__ rho, double *__restrict__ p,
                                                     double *__restrict__ part) {
    const int4 tl = gtiles[blockIdx.x];
    const int64_t j0 = gap_first(tl);
    double acc = 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t j = j0 + i;
        const double v = (double)x0[gap_idx[j]];
        y[j] = 0.0;
        rho[j] = v;
        p[j] = v;
        acc += v * v;
    }
    block_sum(acc, part);
}

// fin at the masked positions = src (the rest of fin stays zero)
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gap_scatter(const int4 *__restrict__ gtiles, const int32_t *__restrict__ act,
                                                       const int64_t *__restrict__ gap_idx, const double *__restrict__ src,
                                                       T *__restrict__ fin) {
    const int4 tl = gtiles[blockIdx.x];
    if (act && !act[tl.x]) return;
    const int64_t j0 = gap_first(tl);
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) fin[gap_idx[j0 + i]] = (T)src[j0 + i];
}

// q = sigma0^2 p - (M S p) at the masked positions; partial sums of p . q
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gap_pq(const int4 *__restrict__ gtiles, const int32_t *__restrict__ act,
                                                  const int64_t *__restrict__ gap_idx, const double *__restrict__ sigma0,
                                                  const double *__restrict__ p, const T *__restrict__ fout,
                                                  double *__restrict__ part) {
    const int4 tl = gtiles[blockIdx.x];
    if (!act[tl.x]) return;
    const double s2 = sigma0[tl.x] * sigma0[tl.x];
    const int64_t j0 = gap_first(tl);
    double acc = 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t j = j0 + i;
        const double pv = p[j];
        acc += pv * (s2 * pv - (double)fout[gap_idx[j]]);
    }
    block_sum(acc, part);
}

// y += alpha p; rho -= alpha q; partial sums of rho^2
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gap_update(const int4 *__restrict__ gtiles, const int32_t *__restrict__ act,
                                                      const CgState *__restrict__ cs, const int64_t *__restrict__ gap_idx,
                                                      const double *__restrict__ sigma0, const double *__restrict__ p,
                                                      const T *__restrict__ fout, double *__restrict__ y,
                                                      double *__restrict__ rho, double *__restrict__ part) {
    const int4 tl = gtiles[blockIdx.x];
    if (!act[tl.x]) return;
    const double s2 = sigma0[tl.x] * sigma0[tl.x];
    const double al = cs[tl.x].alpha;
    const int64_t j0 = gap_first(tl);
    double acc = 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t j = j0 + i;
        const double pv = p[j];
        const double q = s2 * pv - (double)fout[gap_idx[j]];
        y[j] += al * pv;
        const double r = rho[j] - al * q;
        rho[j] = r;
        acc += r * r;
    }
    block_sum(acc, part);
}

// p = rho + beta p, scattered into fin for the next product
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gap_dir(const int4 *__restrict__ gtiles, const int32_t *__restrict__ act,
                                                   const CgState *__restrict__ cs, const int64_t *__restrict__ gap_idx,
                                                   const double *__restrict__ rho, double *__restrict__ p,
                                                   T *__restrict__ fin) {
    const int4 tl = gtiles[blockIdx.x];
    if (!act[tl.x]) return;
    const double be = cs[tl.x].beta;
    const int64_t j0 = gap_first(tl);
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t j = j0 + i;
        const double v = rho[j] + be * p[j];
        p[j] = v;
        fin[gap_idx[j]] = (T)v;
    }
}

// one wave per segment: add the segment's tile partials in order, then step
// the scalar recurrence (see CgStep)
__global__ __launch_bounds__(C3_NT) void k_cg_finish(int nseg, const int2 *__restrict__ seg_tiles,
                                                     const double *__restrict__ part, CgState *__restrict__ cs,
                                                     int32_t *__restrict__ act, int step, double tol2, int max_iter,
                                                     int32_t *__restrict__ nactive) {
    const int seg = blockIdx.x * (C3_NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (step == CG_ALPHA && blockIdx.x == 0 && threadIdx.x == 0) *nactive = 0;  // counted by CG_RES
    if (seg >= nseg) return;
    if (step != CG_RZ0 && !act[seg]) return;
    const int2 tr = seg_tiles[seg];
    double v = 0;
    for (int i = lane; i < tr.y; i += 64) v += part[tr.x + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane != 0) return;
    CgState c = cs[seg];
    switch (step) {
    case CG_RZ0:  // v = rho . rho at y = 0 (gap tiles; none: nothing masked)
        c.alpha = c.beta = 0;
        c.rr = c.bb = v;
        c.iters = 0;
        c.converged = (tr.y == 0 || v == 0.0) ? 1 : 0;  // x0 is the solution
        act[seg] = c.converged ? 0 : 1;
        break;
    case CG_ALPHA:  // v = p . q
        c.alpha = v > 0.0 ? c.rr / v : 0.0;
        if (!(v > 0.0)) act[seg] = 0;  // breakdown: the small system is positive definite
        break;
    case CG_RES:  // v = rho . rho after the update
        c.iters += 1;
        if (v <= tol2 * c.bb) {
            c.converged = 1;
            act[seg] = 0;
        } else if (c.iters >= max_iter) {
            act[seg] = 0;
        } else {
            c.beta = c.rr != 0.0 ? v / c.rr : 0.0;
            atomicAdd(nactive, 1);
        }
        c.rr = v;
        break;
    }
    cs[seg] = c;
}

// n_corr = (x0 + M S y)[0:n]: fout holds M S y where the segment has masked
// samples (has_gap), else is not read
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_crop(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                   const int32_t *__restrict__ has_gap, const T *__restrict__ x0,
                                                   const T *__restrict__ fout, T *__restrict__ out) {
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    const int64_t base = 2 * sg.ext_off;
    const bool g = has_gap[tl.x] != 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t t = tl.y + i;
        out[sg.samp_off + t] = g ? (T)((double)x0[base + t] + (double)fout[base + t]) : x0[base + t];
    }
}

__global__ __launch_bounds__(C3_NT) void k_cg_iters(int nseg, const CgState *__restrict__ cs,
                                                    int32_t *__restrict__ out) {
    const int s = blockIdx.x * C3_NT + threadIdx.x;
    if (s < nseg) out[s] = cs[s].converged ? cs[s].iters : -cs[s].iters;
}

template <typename T>
__global__ __launch_bounds__(C3_NT) void k_fill_zero(T *__restrict__ v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * C3_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * C3_NT) v[i] = (T)0;
}

// s is of the precision's type (the entry point passes it so)
template <typename T, typename TD>
void launch_cg_init(hipStream_t st, dim3 g, dim3 b, const c3::CgVecArgs &a) {
    if (a.have_draw)
        hipLaunchKernelGGL((k_cg_init<T, TD, true>), g, b, 0, st, a.tiles, a.segs, (const TD *)a.d, (const T *)a.s,
                           a.mask, (const T *)a.w1, a.sigma0, (T *)a.res);
    else
        hipLaunchKernelGGL((k_cg_init<T, TD, false>), g, b, 0, st, a.tiles, a.segs, (const TD *)a.d,
                           (const T *)a.s, a.mask, (const T *)a.w1, a.sigma0, (T *)a.res);
}

}  // namespace

namespace c3 {

hipError_t launch_cg_vec(hipStream_t st, int mixed, int op, const CgVecArgs &a) {
    if (a.ntile <= 0) return hipSuccess;
    if (op == CG_OP_INIT && a.s_f64 != (mixed ? 0 : 1)) return hipErrorInvalidValue;  // s: the precision's type
    const dim3 g((unsigned)a.ntile), b(C3_NT);
#define C3_CG_OPS(T)                                                                                          \
    switch (op) {                                                                                             \
    case CG_OP_INIT:                                                                                          \
        if (a.d_f64)                                                                                          \
            launch_cg_init<T, double>(st, g, b, a);                                                           \
        else                                                                                                  \
            launch_cg_init<T, float>(st, g, b, a);                                                            \
        break;                                                                                                \
    case CG_OP_GAP_COUNT:                                                                                     \
        hipLaunchKernelGGL(k_gap_count, g, b, 0, st, a.tiles, a.segs, a.mask, a.cnt);                         \
        break;                                                                                                \
    case CG_OP_GAP_FILL:                                                                                      \
        hipLaunchKernelGGL(k_gap_fill, g, b, 0, st, a.tiles, a.segs, a.mask, a.gap_base, a.gap_idx);          \
        break;                                                                                                \
    case CG_OP_GAP_START:                                                                                     \
        hipLaunchKernelGGL(k_gap_start<T>, g, b, 0, st, a.tiles, a.gap_idx, (const T *)a.x, a.y, a.rho, a.p,  \
                           a.part);                                                                           \
        break;                                                                                                \
    case CG_OP_GAP_SCATTER:                                                                                   \
        hipLaunchKernelGGL(k_gap_scatter<T>, g, b, 0, st, a.tiles, a.act, a.gap_idx, a.scatter_src,           \
                           (T *)a.fin);                                                                       \
        break;                                                                                                \
    case CG_OP_GAP_PQ:                                                                                        \
        hipLaunchKernelGGL(k_gap_pq<T>, g, b, 0, st, a.tiles, a.act, a.gap_idx, a.sigma0, a.p,                \
                           (const T *)a.fout, a.part);                                                        \
        break;                                                                                                \
    case CG_OP_GAP_UPDATE:                                                                                    \
        hipLaunchKernelGGL(k_gap_update<T>, g, b, 0, st, a.tiles, a.act, a.cs, a.gap_idx, a.sigma0, a.p,      \
                           (const T *)a.fout, a.y, a.rho, a.part);                                            \
        break;                                                                                                \
    case CG_OP_GAP_DIR:                                                                                       \
        hipLaunchKernelGGL(k_gap_dir<T>, g, b, 0, st, a.tiles, a.act, a.cs, a.gap_idx, a.rho, a.p,            \
                           (T *)a.fin);                                                                       \
        break;                                                                                                \
    case CG_OP_CROP:                                                                                          \
        hipLaunchKernelGGL(k_cg_crop<T>, g, b, 0, st, a.tiles, a.segs, a.has_gap, (const T *)a.x,             \
                           (const T *)a.fout, (T *)a.out);                                                    \
        break;                                                                                                \
    default:                                                                                                  \
        return hipErrorInvalidValue;                                                                          \
    }
    if (mixed) {
        C3_CG_OPS(float)
    } else {
        C3_CG_OPS(double)
    }
#undef C3_CG_OPS
    return hipGetLastError();
}

hipError_t launch_cg_zero(hipStream_t st, int mixed, void *v, int64_t n) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + C3_NT - 1) / C3_NT;
    if (nb > 65536) nb = 65536;
    if (mixed)
        hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)nb), dim3(C3_NT), 0, st, (float *)v, n);
    else
        hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)nb), dim3(C3_NT), 0, st, (double *)v, n);
    return hipGetLastError();
}

hipError_t launch_cg_finish(hipStream_t st, int nseg, const int2 *seg_tiles, const double *part, CgState *cs,
                            int32_t *act, int step, double tol2, int max_iter, int32_t *nactive) {
    if (nseg <= 0) return hipSuccess;
    const int per = C3_NT / 64;
    hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)((nseg + per - 1) / per)), dim3(C3_NT), 0, st, nseg, seg_tiles,
                       part, cs, act, step, tol2, max_iter, nactive);
    return hipGetLastError();
}

hipError_t launch_cg_iters(hipStream_t st, int nseg, const CgState *cs, int32_t *out) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_iters, dim3((unsigned)((nseg + C3_NT - 1) / C3_NT)), dim3(C3_NT), 0, st, nseg, cs,
                       out);
    return hipGetLastError();
}

}  // namespace c3
