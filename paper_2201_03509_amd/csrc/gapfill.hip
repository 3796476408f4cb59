// Masked correlated-noise draw: the constrained realisation of n_corr when a
// processing mask removes samples (gap filling, section 5 and the correlated
// noise row of Table 2), solved by preconditioned conjugate gradients on the
// same mirrored, 5-smooth padded extension as the unmasked Fourier draw.
//
// Per segment, with F the unitary DFT, 1/P_k the inverse prior spectrum
// (1/P_0 = 0), mu the extended mask ([m, reverse(m), 1 ...]) and e the
// extended residual d - s:
//     A = F^H diag(1/P) F + diag(mu) / sigma0^2
//     b = mu (e / sigma0^2 + F^H W1 / sigma0) + F^H (W2 sqrt(1/P))
//     preconditioner F^H diag(1 / (1/sigma0^2 + 1/P)) F
// The Fourier-diagonal products run through the FFT passes (row modes 2 and
// 3); this file holds the vector work: right-hand side, the CG updates, their
// per-segment reductions and the scalar recurrences.
//
// Vectors are sweep-wide: segment s owns reals [2 ext_off, 2 ext_off + N) of
// each.  The Krylov vectors x, res, p and the transform output fout have the
// transform's type (FP32 in the mixed precision); every element update and
// every dot product is evaluated in FP64, and the scalar recurrences (alpha,
// beta, norms) are FP64.  p and res are the transforms' inputs as they stand.
// Elementwise kernels walk tiles of C3_CG_TILE reals of one segment; a tile
// writes one partial sum, and one wave per segment adds its tiles' partials
// in a fixed order (run-to-run reproducible, no atomics on the sums).
#include "common.h"

namespace {
using namespace c3;

__device__ __forceinline__ double ldd(const void *p, int f64, int64_t i) {
    return f64 ? ((const double *)p)[i] : (double)((const float *)p)[i];
}

// position of extended index t in the segment: the mirror of the extension;
// -1 in the pad (mask 1, value r_0)
__device__ __forceinline__ int64_t mirror(int64_t t, int n) {
    return t < n ? t : (t < 2 * (int64_t)n ? 2 * (int64_t)n - 1 - t : -1);
}

__device__ __forceinline__ double mu_at(const uint8_t *mask, int64_t s0, int n, int64_t t) {
    const int64_t u = mirror(t, n);
    return u < 0 ? 1.0 : (double)(mask[s0 + u] != 0);
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

// Elementwise kernels take the extended reals in pairs (t, t+1): N and every
// tile length are even and each segment's vector starts at an even real, so
// a pair is one aligned two-element access.
template <typename T>
using V2 = cx<T>;

template <typename T>
__device__ __forceinline__ V2<T> ld2(const T *v, int64_t i) {
    return *(const V2<T> *)(v + i);
}
template <typename T>
__device__ __forceinline__ void st2(T *v, int64_t i, double a, double b) {
    *(V2<T> *)(v + i) = V2<T>{(T)a, (T)b};
}

// b = mu (e / s0^2 + w1 / s0) + v2 -> res (v2 arrives in res); x = 0;
// partial sums of b^2
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_init(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                   const void *d, int d_f64, const void *s, int s_f64,
                                                   const uint8_t *__restrict__ mask, const T *__restrict__ w1,
                                                   const double *__restrict__ sigma0, int have_draw,
                                                   T *__restrict__ x, T *__restrict__ res,
                                                   double *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    const double s0 = sigma0[tl.x], is2 = 1.0 / (s0 * s0), is1 = 1.0 / s0;
    const int64_t base = 2 * sg.ext_off + tl.y;
    double acc = 0;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        double b[2];
        const V2<T> w = have_draw ? ld2(w1, base + i) : V2<T>{0, 0};
        const V2<T> v = have_draw ? ld2(res, base + i) : V2<T>{0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t u = mirror(tl.y + i + h, sg.n);
            const int64_t j = sg.samp_off + (u < 0 ? 0 : u);
            const double e = ldd(d, d_f64, j) - ldd(s, s_f64, j);
            const double m = u < 0 ? 1.0 : (double)(mask[j] != 0);
            b[h] = m * (e * is2 + (double)(h ? w.y : w.x) * is1) + (double)(h ? v.y : v.x);
            acc += b[h] * b[h];
        }
        st2(x, base + i, 0.0, 0.0);
        st2(res, base + i, b[0], b[1]);
    }
    block_sum(acc, part);
}

// partial sums of p . (A p), A p = fout + mu p / s0^2 (fout = F^H diag(1/P) F p)
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_pap(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                  const int32_t *__restrict__ act, const uint8_t *__restrict__ mask,
                                                  const double *__restrict__ sigma0, const T *__restrict__ p,
                                                  const T *__restrict__ fout, double *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    if (!act[tl.x]) return;
    const SegInfo sg = segs[tl.x];
    const double s0 = sigma0[tl.x], is2 = 1.0 / (s0 * s0);
    const int64_t base = 2 * sg.ext_off + tl.y;
    double acc = 0;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        const V2<T> pv = ld2(p, base + i), f = ld2(fout, base + i);
        const double m0 = mu_at(mask, sg.samp_off, sg.n, tl.y + i), m1 = mu_at(mask, sg.samp_off, sg.n, tl.y + i + 1);
        acc += (double)pv.x * ((double)f.x + m0 * (double)pv.x * is2);
        acc += (double)pv.y * ((double)f.y + m1 * (double)pv.y * is2);
    }
    block_sum(acc, part);
}

// x += alpha p; res -= alpha A p; partial sums of res^2 (of the stored res)
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_xr(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                 const int32_t *__restrict__ act, const CgState *__restrict__ cs,
                                                 const uint8_t *__restrict__ mask, const double *__restrict__ sigma0,
                                                 const T *__restrict__ p, const T *__restrict__ fout,
                                                 T *__restrict__ x, T *__restrict__ res, double *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    if (!act[tl.x]) return;
    const SegInfo sg = segs[tl.x];
    const double s0 = sigma0[tl.x], is2 = 1.0 / (s0 * s0);
    const double al = cs[tl.x].alpha;
    const int64_t base = 2 * sg.ext_off + tl.y;
    double acc = 0;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        const V2<T> pv = ld2(p, base + i), f = ld2(fout, base + i), xv = ld2(x, base + i), rv = ld2(res, base + i);
        const double m0 = mu_at(mask, sg.samp_off, sg.n, tl.y + i), m1 = mu_at(mask, sg.samp_off, sg.n, tl.y + i + 1);
        const double ap0 = (double)f.x + m0 * (double)pv.x * is2, ap1 = (double)f.y + m1 * (double)pv.y * is2;
        st2(x, base + i, (double)xv.x + al * (double)pv.x, (double)xv.y + al * (double)pv.y);
        const V2<T> r = {(T)((double)rv.x - al * ap0), (T)((double)rv.y - al * ap1)};
        *(V2<T> *)(res + base + i) = r;
        acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
    }
    block_sum(acc, part);
}

// partial sums of res . z (z = fout, the preconditioned residual)
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_rz(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                 const int32_t *__restrict__ act, const T *__restrict__ res,
                                                 const T *__restrict__ fout, double *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    if (!act[tl.x]) return;
    const int64_t base = 2 * segs[tl.x].ext_off + tl.y;
    double acc = 0;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        const V2<T> r = ld2(res, base + i), z = ld2(fout, base + i);
        acc += (double)r.x * (double)z.x + (double)r.y * (double)z.y;
    }
    block_sum(acc, part);
}

// p = z + beta p (beta = 0: p = z, the old p is not read)
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_p(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                const int32_t *__restrict__ act, const CgState *__restrict__ cs,
                                                const T *__restrict__ fout, T *__restrict__ p) {
    const int4 tl = tiles[blockIdx.x];
    if (!act[tl.x]) return;
    const int64_t base = 2 * segs[tl.x].ext_off + tl.y;
    const double be = cs[tl.x].beta;
    for (int i = 2 * threadIdx.x; i < tl.z; i += 2 * C3_NT) {
        const V2<T> z = ld2(fout, base + i);
        const V2<T> po = be != 0.0 ? ld2(p, base + i) : V2<T>{0, 0};
        st2(p, base + i, (double)z.x + be * (double)po.x, (double)z.y + be * (double)po.y);
    }
}

// one wave per segment: add the segment's tile partials in order, then step
// the scalar recurrence (see CgStep)
__global__ __launch_bounds__(C3_NT) void k_cg_finish(int nseg, const int2 *__restrict__ seg_tiles,
                                                     const double *__restrict__ part, CgState *__restrict__ cs,
                                                     int32_t *__restrict__ act, int step, double tol2,
                                                     int max_iter, int32_t *__restrict__ nactive) {
    const int seg = blockIdx.x * (C3_NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (step == CG_ALPHA && blockIdx.x == 0 && threadIdx.x == 0) *nactive = 0;  // counted by CG_RES
    if (seg >= nseg) return;
    if (step != CG_INIT && !act[seg]) return;
    const int2 tr = seg_tiles[seg];
    double v = 0;
    for (int i = lane; i < tr.y; i += 64) v += part[tr.x + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane != 0) return;
    CgState c = cs[seg];
    switch (step) {
    case CG_INIT:  // v = b . b
        c.bb = v;
        c.rz = c.alpha = c.beta = c.rr = 0;
        c.iters = 0;
        c.converged = v == 0.0 ? 1 : 0;  // b = 0: x = 0 is exact
        act[seg] = (v > 0.0 && tr.y > 0) ? 1 : 0;
        break;
    case CG_RZ0:  // v = res . z
        c.rz = v;
        c.beta = 0;
        break;
    case CG_ALPHA:  // v = p . A p
        c.alpha = v > 0.0 ? c.rz / v : 0.0;
        if (!(v > 0.0)) act[seg] = 0;  // breakdown (A is positive definite: only at x exact)
        break;
    case CG_RES:  // v = res . res
        c.rr = v;
        c.iters += 1;
        if (v <= tol2 * c.bb) {
            c.converged = 1;
            act[seg] = 0;
        } else if (c.iters >= max_iter) {
            act[seg] = 0;
        } else {
            atomicAdd(nactive, 1);
        }
        break;
    case CG_BETA:  // v = res . z (new)
        c.beta = c.rz != 0.0 ? v / c.rz : 0.0;
        c.rz = v;
        break;
    }
    cs[seg] = c;
}

// n_corr = x[0:n] of every segment, in the output type
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_cg_crop(const int4 *__restrict__ tiles, const SegInfo *__restrict__ segs,
                                                   const T *__restrict__ x, T *__restrict__ out) {
    const int4 tl = tiles[blockIdx.x];
    const SegInfo sg = segs[tl.x];
    const int64_t base = 2 * sg.ext_off;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const int64_t t = tl.y + i;
        out[sg.samp_off + t] = x[base + t];
    }
}

__global__ __launch_bounds__(C3_NT) void k_cg_iters(int nseg, const CgState *__restrict__ cs,
                                                    int32_t *__restrict__ out) {
    const int s = blockIdx.x * C3_NT + threadIdx.x;
    if (s < nseg) out[s] = cs[s].converged ? cs[s].iters : -cs[s].iters;
}

}  // namespace

namespace c3 {

hipError_t launch_cg_vec(hipStream_t st, int mixed, int op, const CgVecArgs &a) {
    if (a.ntile <= 0) return hipSuccess;
    const dim3 g((unsigned)a.ntile), b(C3_NT);
#define C3_CG_OPS(T)                                                                                         \
    switch (op) {                                                                                            \
    case CG_OP_INIT:                                                                                         \
        hipLaunchKernelGGL(k_cg_init<T>, g, b, 0, st, a.tiles, a.segs, a.d, a.d_f64, a.s, a.s_f64, a.mask,    \
                           (const T *)a.w1, a.sigma0, a.have_draw, (T *)a.x, (T *)a.res, a.part);             \
        break;                                                                                               \
    case CG_OP_PAP:                                                                                          \
        hipLaunchKernelGGL(k_cg_pap<T>, g, b, 0, st, a.tiles, a.segs, a.act, a.mask, a.sigma0,               \
                           (const T *)a.p, (const T *)a.fout, a.part);                                       \
        break;                                                                                               \
    case CG_OP_XR:                                                                                           \
        hipLaunchKernelGGL(k_cg_xr<T>, g, b, 0, st, a.tiles, a.segs, a.act, a.cs, a.mask, a.sigma0,          \
                           (const T *)a.p, (const T *)a.fout, (T *)a.x, (T *)a.res, a.part);                 \
        break;                                                                                               \
    case CG_OP_RZ:                                                                                           \
        hipLaunchKernelGGL(k_cg_rz<T>, g, b, 0, st, a.tiles, a.segs, a.act, (const T *)a.res,                \
                           (const T *)a.fout, a.part);                                                       \
        break;                                                                                               \
    case CG_OP_P:                                                                                            \
        hipLaunchKernelGGL(k_cg_p<T>, g, b, 0, st, a.tiles, a.segs, a.act, a.cs, (const T *)a.fout,          \
                           (T *)a.p);                                                                        \
        break;                                                                                               \
    case CG_OP_CROP:                                                                                         \
        hipLaunchKernelGGL(k_cg_crop<T>, g, b, 0, st, a.tiles, a.segs, (const T *)a.x, (T *)a.out);          \
        break;                                                                                               \
    default:                                                                                                 \
        return hipErrorInvalidValue;                                                                         \
    }
    if (mixed) {
        C3_CG_OPS(float)
    } else {
        C3_CG_OPS(double)
    }
#undef C3_CG_OPS
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
