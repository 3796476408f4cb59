// Gain draw g <- P(g | d, xi_n, sky) per segment (Eq. 3; the gain step of the
// TOD loop, whose FFTs section 4.2 counts with the correlated-noise step).
// n_corr is not conditioned on, so its covariance joins the white noise:
// N^-1 = F^H diag(1/(sigma0^2 + P_k)) F on the mirrored extension (h_0 = 0),
// applied by the FFT passes (row mode 2, filter 2) to the sky template t = P m
// and to the data d.  Here: A = t . K t and B = t . K d per segment in FP64,
// then g = B/A + eta/sqrt(A) with eta the Box-Muller normal of the segment's
// Philox stream at counter word 2^32 - 1 (no Fourier mode uses it).
#include "common.h"
#include "rng.h"

namespace {
using namespace c3;
using namespace c3rng;

// per sample tile (seg, first sample, length): partial sums of t.kt and t.kd
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_gain_dots(const int4 *__restrict__ tiles, const int64_t *__restrict__ seg_off,
                                                     const T *__restrict__ t, const T *__restrict__ kt,
                                                     const T *__restrict__ kd, double2 *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    const int64_t base = seg_off[tl.x] + tl.y;
    double a = 0, b = 0;
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const double tv = (double)t[base + i];
        a += tv * (double)kt[base + i];
        b += tv * (double)kd[base + i];
    }
    __shared__ double red[2][C3_NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0, sb = 0;
#pragma unroll
        for (int i = 0; i < C3_NT / 64; ++i) {
            sa += red[0][i];
            sb += red[1][i];
        }
        part[blockIdx.x] = make_double2(sa, sb);
    }
}

// one wave per segment: sum its tiles' partials in order, draw the gain
__global__ __launch_bounds__(C3_NT) void k_gain_finish(int nseg, const int2 *__restrict__ seg_tiles,
                                                       const double2 *__restrict__ part,
                                                       const uint64_t *__restrict__ seed_iter, int mean_only,
                                                       double *__restrict__ gain_out, double *__restrict__ sigma_out) {
    const int seg = blockIdx.x * (C3_NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (seg >= nseg) return;
    const int2 tr = seg_tiles[seg];
    double a = 0, b = 0;
    for (int i = lane; i < tr.y; i += 64) {
        const double2 v = part[tr.x + i];
        a += v.x;
        b += v.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if (lane != 0) return;
    if (!(a > 0.0)) {  // empty segment or a template without information
        gain_out[seg] = NAN;
        if (sigma_out) sigma_out[seg] = INFINITY;
        return;
    }
    const double sig = 1.0 / sqrt(a);
    double g = b / a;
    if (!mean_only) {
        const uint64_t seed = seed_iter[0], it = seed_iter[1];
        double z[4];
        normals4<double>(philox4x32_10(make_uint4(0xFFFFFFFFu, (uint32_t)it, (uint32_t)(it >> 32),
                                                  (uint32_t)(seed >> 32)),
                                       make_uint2((uint32_t)seed, (uint32_t)seg)),
                         z);
        g += sig * z[0];
    }
    gain_out[seg] = g;
    if (sigma_out) sigma_out[seg] = sig;
}

}  // namespace

namespace c3 {

hipError_t launch_gain_dots(hipStream_t st, int mixed, const int4 *tiles, int ntile, const int64_t *seg_off,
                            const void *t, const void *kt, const void *kd, double2 *part) {
    if (ntile <= 0) return hipSuccess;
    if (mixed)
        hipLaunchKernelGGL(k_gain_dots<float>, dim3((unsigned)ntile), dim3(C3_NT), 0, st, tiles, seg_off,
                           (const float *)t, (const float *)kt, (const float *)kd, part);
    else
        hipLaunchKernelGGL(k_gain_dots<double>, dim3((unsigned)ntile), dim3(C3_NT), 0, st, tiles, seg_off,
                           (const double *)t, (const double *)kt, (const double *)kd, part);
    return hipGetLastError();
}

hipError_t launch_gain_finish(hipStream_t st, int nseg, const int2 *seg_tiles, const double2 *part,
                              const uint64_t *seed_iter, int mean_only, double *gain_out, double *sigma_out) {
    if (nseg <= 0) return hipSuccess;
    const int per = C3_NT / 64;
    hipLaunchKernelGGL(k_gain_finish, dim3((unsigned)((nseg + per - 1) / per)), dim3(C3_NT), 0, st, nseg,
                       seg_tiles, part, seed_iter, mean_only, gain_out, sigma_out);
    return hipGetLastError();
}

}  // namespace c3
