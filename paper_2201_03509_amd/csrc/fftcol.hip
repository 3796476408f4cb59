// Column passes of the four-step n_corr FFT (section 4.2) with the column
// length M1 fixed at compile time.
//
// One lane owns one column j2 of a segment: it loads the M1 elements
// z[M2 j1 + j2] (consecutive lanes read consecutive addresses), runs the whole
// FFT_M1 in registers as unrolled Stockham stages whose twiddles are folded to
// constants at compile time, applies the four-step twiddle w_M^(j2 k1) and
// writes Y[k1][j2].  No LDS and no barriers: every lane keeps its column's
// loads (one 8-byte load per element) in flight, which is what hides HBM
// latency in this pass.  The inverse kernel
// takes Y[k1][j2] times w_M^(-j2 k1), inverts the column and writes the first
// n real samples.  The LDS-tiled column kernels in fft.hip cover every other
// M1 and the FP64 path.
#include <utility>

#include "common.h"
#include "fftdev.h"

namespace {
using c3::FftArgs;
using namespace c3fft;

// word 3 of a raw buffer resource on gfx9-family chips (untyped dword access)
#define C3_BUF_WORD3 0x00020000

// Loads and stores below address a uniform (scalar) base plus a 32-bit lane
// offset, so the compiler needs no 64-bit address per element.
template <typename V>
__device__ __forceinline__ V ld_off(const void *base, uint32_t byte_off) {
    return *(const V *)((const char *)base + byte_off);
}
template <typename V>
__device__ __forceinline__ void st_off(void *base, uint32_t byte_off, V v) {
    *(V *)((char *)base + byte_off) = v;
}

// reals t and t + 1 (t even) of the mirrored, padded extension of the n
// samples in the raw buffer rb (4 n bytes) as one complex value, from one
// 8-byte load: adjacent samples below n, the mirror image of an adjacent pair
// (in reverse order) from n to 2n, the last sample twice at t = n - 1 (odd
// n), and the first sample twice in the pad beyond 2n (the pad repeats r_0).
// Needs n > 1: every load stays inside the n samples.
__device__ __forceinline__ cx<float> ext_pair(__amdgpu_buffer_rsrc_t rb, uint32_t n, uint32_t t) {
    const uint32_t n2 = 2u * n;
    const bool lo = t + 1u < n, mir = t >= n, pad = t >= n2;
    const uint32_t b = lo ? t : (pad ? 0u : (mir ? n2 - 2u - t : n - 2u));
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rb, (int)(4u * b), 0, 0);
    const float v0 = __uint_as_float(v[0]), v1 = __uint_as_float(v[1]);
    return cx<float>{lo || pad ? v0 : v1, mir ? v0 : v1};
}

// f(k1, w_M^(j2 k1)) for k1 < M1, with w_M^(j2 (a Q + b)) = w_M^(j2 Q a) w_M^(j2 b)
// from the two-level w_N table (N = 2M); each factor is used as soon as it is
// formed, so no table of M1 twiddles is held in registers
template <int M1, int Q, typename F>
__device__ __forceinline__ void col_twiddles(const cx<float> *pool, const FftPlan &p, int j2, F &&f) {
    cx<float> wb[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) wb[b] = twN(pool, p, 2 * (int64_t)j2 * b);
#pragma unroll
    for (int ai = 0; ai * Q < M1; ++ai) {
        const cx<float> wa = twN(pool, p, 2 * (int64_t)j2 * Q * ai);
#pragma unroll
        for (int b = 0; b < Q; ++b)
            if (ai * Q + b < M1) f(ai * Q + b, cmul(wa, wb[b]));
    }
}

// ------------------------------------------------------------- pass 1
template <int M1>
__global__ __launch_bounds__(C3_COL_NT) void k_colr_fwd(FftArgs a) {
    // the column's loads need only the task: they are issued first, and the
    // segment's plan (twiddles) loads while they are in flight.  In the
    // masked draw a converged segment's block returns before any load.
    const ColTask sg = a.col_tasks[blockIdx.x];
    const int M2 = sg.M2;
    const int j2 = sg.c0 + (int)threadIdx.x;
    if (j2 >= M2) return;
    if (a.active && !a.active[sg.seg]) return;  // converged segment (whole block)
    const uint32_t n = (uint32_t)sg.n, n2 = 2u * (uint32_t)sg.n;
    cx<float> x[M1];
    if (a.full_io) {
        // a whole extended vector (N reals = M complex at the segment's offset)
        const cx<float> *v = (const cx<float> *)a.in_a + sg.ext_off;
        const uint32_t lo = 8u * (uint32_t)j2;
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) {
            x[j1] = ld_off<cx<float>>(v + (int64_t)j1 * M2, lo);
            if ((j1 & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
    } else if (!a.in_b && !a.in_a_f64) {
        // r = in_a (FP32): the sweep's residual (n > 12 here: M >= M1 >= 16
        // is the next 5-smooth length >= n)
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((float *)a.in_a + sg.samp_off, 0, 4 * sg.n, C3_BUF_WORD3);
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) {
            x[j1] = ext_pair(r, n, 2u * (uint32_t)(M2 * j1 + j2));
            // keep the scheduler from computing every offset before the first
            // load: 16 rows in flight is plenty
            if ((j1 & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
    } else if (a.in_b && !a.in_a_f64 && !a.in_b_f64) {
        // r = in_a - in_b, both FP32 (d and s of a standalone draw): every
        // load of the column is issued before the first subtraction
        const __amdgpu_buffer_rsrc_t ra =
            __builtin_amdgcn_make_buffer_rsrc((float *)a.in_a + sg.samp_off, 0, 4 * sg.n, C3_BUF_WORD3);
        const __amdgpu_buffer_rsrc_t rb =
            __builtin_amdgcn_make_buffer_rsrc((float *)a.in_b + sg.samp_off, 0, 4 * sg.n, C3_BUF_WORD3);
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) {
            const uint32_t t = 2u * (uint32_t)(M2 * j1 + j2);
            x[j1] = csub(ext_pair(ra, n, t), ext_pair(rb, n, t));
            if ((j1 & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        // r = in_a - in_b in any input precision, rounded to FP32
        const int64_t s0 = sg.samp_off;
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) {
            const uint32_t t = 2u * (uint32_t)(M2 * j1 + j2);
            float v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t th = t + (uint32_t)h;
                const uint32_t u = th < n ? th : (th < n2 ? n2 - 1u - th : 0u);
                v[h] = load_as<float>(a.in_a, a.in_a_f64, s0 + u);
                if (a.in_b) v[h] -= load_as<float>(a.in_b, a.in_b_f64, s0 + u);
            }
            x[j1] = cx<float>{v[0], v[1]};
        }
    }
    const FftPlan &p = a.plans[a.segs[sg.seg].plan];
    reg_fft<M1, -1>(x);
    // the twiddle-table loads below must not be hoisted into the FFT, where
    // every register already holds column data
    __builtin_amdgcn_sched_barrier(0);
    cx<float> *Y = (cx<float> *)a.work + sg.scr_off;
    const uint32_t lo = 8u * (uint32_t)j2;
    col_twiddles<M1, tw_split(M1)>((const cx<float> *)a.twpool, p, j2, [&](int k1, cx<float> w) {
        st_off(Y + (int64_t)k1 * M2, lo, cmul(x[k1], w));
    });
}

// ------------------------------------------------------------- pass 3
template <int M1>
__global__ __launch_bounds__(C3_COL_NT) void k_colr_inv(FftArgs a) {
    const ColTask sg = a.col_tasks[blockIdx.x];
    const int M2 = sg.M2;
    const int j2 = sg.c0 + (int)threadIdx.x;
    if (j2 >= M2) return;
    if (a.active && !a.active[sg.seg]) return;  // converged segment (whole block)
    const cx<float> *Y = (const cx<float> *)a.work + sg.scr_off;
    const uint32_t lo = 8u * (uint32_t)j2;
    cx<float> x[M1];
#pragma unroll
    for (int k1 = 0; k1 < M1; ++k1) x[k1] = ld_off<cx<float>>(Y + (int64_t)k1 * M2, lo);
    const FftPlan &p = a.plans[a.segs[sg.seg].plan];
    col_twiddles<M1, tw_split(M1)>((const cx<float> *)a.twpool, p, j2, [&](int k1, cx<float> w) {
        x[k1] = cmulc(x[k1], w);  // times w_M^(-j2 k1)
    });
    reg_fft<M1, 1>(x);
    if (a.full_io) {
        // the whole extended vector
        cx<float> *v = (cx<float> *)a.out + sg.ext_off;
        const uint32_t lo = 8u * (uint32_t)j2;
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) st_off(v + (int64_t)j1 * M2, lo, x[j1]);
        return;
    }
    // the first n real samples: a raw buffer of n floats, whose hardware range
    // check drops the stores at t >= n (no per-element branch)
    const __amdgpu_buffer_rsrc_t out =
        __builtin_amdgcn_make_buffer_rsrc((float *)a.out + sg.samp_off, 0, 4 * sg.n, C3_BUF_WORD3);
#pragma unroll
    for (int j1 = 0; j1 < M1; ++j1) {
        const uint32_t t = 2u * (uint32_t)(M2 * j1 + j2);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[j1].x), out, (int)(4u * t), 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[j1].y), out, (int)(4u * t + 4u), 0, 0);
    }
}

}  // namespace

namespace c3 {

bool fft_col_reg_supported(int mixed, int m1) {
    if (!mixed) return false;
    switch (m1) {
#define C3_SUP(M) case M:
        C3_COLREG_LIST(C3_SUP)
        return true;
#undef C3_SUP
    default:
        return false;
    }
}

hipError_t launch_fft_col_reg(hipStream_t st, int mixed, const FftArgs &a, int pass, int m1) {
    if (!mixed || (pass != 0 && pass != 2)) return hipErrorInvalidValue;
    if (a.ncol_tasks <= 0) return hipSuccess;
    const dim3 g(a.ncol_tasks), b(C3_COL_NT);
    switch (m1) {
#define C3_CASE(M)                                                     \
    case M:                                                            \
        if (pass == 0)                                                 \
            hipLaunchKernelGGL(k_colr_fwd<M>, g, b, 0, st, a);         \
        else                                                           \
            hipLaunchKernelGGL(k_colr_inv<M>, g, b, 0, st, a);         \
        break;
        C3_COLREG_LIST(C3_CASE)
#undef C3_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace c3
