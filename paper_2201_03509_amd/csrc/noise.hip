// Noise-parameter draw xi_n <- P(xi_n | d, g, n_corr, sky) per segment (Eq. 5;
// the correlated-noise PSD step, which needs only low-volume spectrum data).
//
// 1. White level: r = d - g t - n_corr; sigma0^2 = S / X, S = sum r^2 (FP64
//    tile partials here), X ~ chi^2_n by the Wilson-Hilferty transform.
// 2. The periodogram of n_corr on its mirrored extension, summed into integer
//    log-frequency bins J_b by the FFT row pass (mode 4).  Per bin the count
//    c_b and sum of ln k follow from its mode range [lo, hi] in closed form
//    (lgamma), f_b = (f_samp/N) exp(mean ln k).
// 3. alpha | f_knee, sigma0: binned Whittle ln L is strictly concave in alpha;
//    its maximiser by a bracketed, bisection-safeguarded Newton iteration,
//    alpha = alpha_hat + z1 / sqrt(-d2 lnL).
// 4. f_knee | alpha, sigma0: u = f_knee^alpha ~ Gamma(K, S_a / sigma0^2),
//    Wilson-Hilferty variate, f_knee = u^(1/alpha).
// z0, z1, z2: Box-Muller normals of the segment's Philox stream at counter
// word 2^32 - 2; mean_only: all zero.
#include "common.h"
#include "rng.h"

namespace {
using namespace c3;
using namespace c3rng;

// per sample tile: partial sum of (d - g t - n_corr)^2 (d of type TD, fixed at
// compile time so that the loads of several samples issue together)
template <typename T, typename TD>
__global__ __launch_bounds__(C3_NT) void k_xi_white(const int4 *__restrict__ tiles, const int64_t *__restrict__ seg_off,
                                                    const TD *__restrict__ d, const T *__restrict__ t,
                                                    const double *__restrict__ gain, const T *__restrict__ nc,
                                                    double *__restrict__ part) {
    const int4 tl = tiles[blockIdx.x];
    const int64_t base = seg_off[tl.x] + tl.y;
    const double g = gain[tl.x];
    double acc = 0;
#pragma unroll 4
    for (int i = threadIdx.x; i < tl.z; i += C3_NT) {
        const double r = (double)d[base + i] - g * (double)t[base + i] - (double)nc[base + i];
        acc += r * r;
    }
    __shared__ double red[C3_NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
#pragma unroll
        for (int i = 0; i < C3_NT / 64; ++i) s += red[i];
        part[blockIdx.x] = s;
    }
}

// wave-wide sum, every lane gets the result (fixed butterfly order)
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

#define C3_XI_PER_LANE ((C3_XI_NBIN + 63) / 64)

// one wave per segment
__global__ __launch_bounds__(C3_NT) void k_xi_sample(int nseg, const SegInfo *__restrict__ segs,
                                                     const FftPlan *__restrict__ plans,
                                                     const int32_t *__restrict__ seg_band,
                                                     const double *__restrict__ fsamp_band,
                                                     const int2 *__restrict__ seg_tiles,
                                                     const double *__restrict__ part,
                                                     const double *__restrict__ bins,
                                                     const double *__restrict__ fknee_in,
                                                     const uint64_t *__restrict__ seed_iter, int mean_only,
                                                     double *__restrict__ sigma0_out,
                                                     double *__restrict__ fknee_out,
                                                     double *__restrict__ alpha_out) {
    const int seg = blockIdx.x * (C3_NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (seg >= nseg) return;
    const SegInfo sg = segs[seg];
    if (sg.n <= 0 || sg.plan < 0) {
        if (lane == 0) sigma0_out[seg] = fknee_out[seg] = alpha_out[seg] = NAN;
        return;
    }
    const int64_t M = plans[sg.plan].M;
    const double N = 2.0 * (double)M;
    const double fs = fsamp_band[seg_band[seg]];
    const double fk_old = fknee_in[seg];

    double z[4] = {0, 0, 0, 0};
    if (!mean_only) {
        const uint64_t seed = seed_iter[0], it = seed_iter[1];
        normals4<double>(philox4x32_10(make_uint4(0xFFFFFFFEu, (uint32_t)it, (uint32_t)(it >> 32),
                                                  (uint32_t)(seed >> 32)),
                                       make_uint2((uint32_t)seed, (uint32_t)seg)),
                         z);
    }

    // 1. white level
    const int2 tr = seg_tiles[seg];
    double S = 0;
    for (int i = lane; i < tr.y; i += 64) S += part[tr.x + i];
    S = wsum(S);
    const double n = (double)sg.n;
    const double wh = 1.0 - 2.0 / (9.0 * n) + z[0] * sqrt(2.0 / (9.0 * n));
    const double s2 = S / (n * wh * wh * wh);

    // 2. bins of this segment: lane holds bins lane, lane + 64, ...
    const int nb = 1 + (M < 8 ? (int)M - 1 : 7 + 8 * ((63 - __builtin_clzll((unsigned long long)M)) - 3) +
                                             (int)(M >> ((63 - __builtin_clzll((unsigned long long)M)) - 3)) - 8);
    double Jb[C3_XI_PER_LANE], cb[C3_XI_PER_LANE], xb[C3_XI_PER_LANE], lf[C3_XI_PER_LANE];
    const double lscale = log(fs / N);
#pragma unroll
    for (int j = 0; j < C3_XI_PER_LANE; ++j) {
        const int b = lane + 64 * j;
        Jb[j] = cb[j] = xb[j] = lf[j] = 0;
        if (b >= nb) continue;
        int64_t lo, hi;  // mode range of bin b, clipped to M
        if (b < 7) {
            lo = hi = b + 1;
        } else {
            const int e = 3 + (b - 7) / 8, m = (b - 7) % 8;
            lo = (int64_t)(8 + m) << (e - 3);
            hi = ((int64_t)(9 + m) << (e - 3)) - 1;
        }
        if (hi > M) hi = M;
        if (lo > hi) continue;
        const double c = (double)(hi - lo + 1);
        const double L = lgamma((double)hi + 1.0) - lgamma((double)lo);  // sum of ln k, k = lo..hi
        Jb[j] = bins[(int64_t)seg * C3_XI_NBIN + b];
        cb[j] = c;
        lf[j] = lscale + L / c;                 // ln f_b
        xb[j] = lf[j] - log(fk_old);            // ln(f_b / f_knee)
    }

    // 3. alpha | f_knee: score(al) = sum a x e^(-al x) - sum c x, a = J / sigma0^2
    auto score = [&](double al, double *dscore) {
        double s = 0, ds = 0;
#pragma unroll
        for (int j = 0; j < C3_XI_PER_LANE; ++j) {
            if (cb[j] == 0.0) continue;
            const double ax = Jb[j] / s2 * xb[j] * exp(-al * xb[j]);
            s += ax - cb[j] * xb[j];
            ds -= ax * xb[j];
        }
        if (dscore) *dscore = wsum(ds);
        return wsum(s);
    };
    double lo = -1.0, hi = 1.0;
    bool ok = true;
    for (int i = 0; i < 60 && score(lo, nullptr) < 0.0; ++i) lo *= 2.0;
    for (int i = 0; i < 60 && score(hi, nullptr) > 0.0; ++i) hi *= 2.0;
    if (!(score(lo, nullptr) >= 0.0) || !(score(hi, nullptr) <= 0.0)) ok = false;
    double al = 0.5 * (lo + hi), H = 0;
    if (ok) {
        for (int i = 0; i < 200; ++i) {
            double ds;
            const double f = score(al, &ds);
            if (f > 0.0) lo = al; else hi = al;
            double nx = al - f / ds;                   // Newton step
            if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);  // bisection fallback
            const double step = fabs(nx - al);
            al = nx;
            if (step <= 1e-15 * fmax(1.0, fabs(al)) || hi - lo <= 1e-15 * fmax(1.0, fabs(al))) break;
        }
        score(al, &H);
        H = -H;
    }
    const double alpha = ok ? al + z[1] / sqrt(H) : NAN;

    // 4. f_knee | alpha: u = f_knee^alpha ~ Gamma(K, S_a / sigma0^2)
    double Sa = 0, K = 0;
#pragma unroll
    for (int j = 0; j < C3_XI_PER_LANE; ++j) {
        if (cb[j] == 0.0) continue;
        Sa += Jb[j] * exp(-alpha * lf[j]);
        K += cb[j];
    }
    Sa = wsum(Sa);
    K = wsum(K);
    const double gw = 1.0 - 1.0 / (9.0 * K) + z[2] / (3.0 * sqrt(K));
    const double u = K * gw * gw * gw * s2 / Sa;
    if (lane == 0) {
        sigma0_out[seg] = sqrt(s2);
        alpha_out[seg] = alpha;
        fknee_out[seg] = exp(log(u) / alpha);
    }
}

}  // namespace

namespace c3 {

hipError_t launch_xi_white(hipStream_t st, int mixed, const int4 *tiles, int ntile, const int64_t *seg_off,
                           const void *d, int d_f64, const void *t, const double *gain, const void *nc,
                           double *part) {
    if (ntile <= 0) return hipSuccess;
    const dim3 g((unsigned)ntile), b(C3_NT);
#define C3_XIW(T, TD)                                                                                    \
    hipLaunchKernelGGL((k_xi_white<T, TD>), g, b, 0, st, tiles, seg_off, (const TD *)d, (const T *)t, gain, \
                       (const T *)nc, part)
    if (mixed) {
        if (d_f64)
            C3_XIW(float, double);
        else
            C3_XIW(float, float);
    } else {
        if (d_f64)
            C3_XIW(double, double);
        else
            C3_XIW(double, float);
    }
#undef C3_XIW
    return hipGetLastError();
}

hipError_t launch_xi_sample(hipStream_t st, int nseg, const SegInfo *segs, const FftPlan *plans,
                            const int32_t *seg_band, const double *fsamp_band, const int2 *seg_tiles,
                            const double *part, const double *bins, const double *fknee_in,
                            const uint64_t *seed_iter, int mean_only, double *sigma0_out, double *fknee_out,
                            double *alpha_out) {
    if (nseg <= 0) return hipSuccess;
    const int per = C3_NT / 64;
    hipLaunchKernelGGL(k_xi_sample, dim3((unsigned)((nseg + per - 1) / per)), dim3(C3_NT), 0, st, nseg, segs,
                       plans, seg_band, fsamp_band, seg_tiles, part, bins, fknee_in, seed_iter, mean_only,
                       sigma0_out, fknee_out, alpha_out);
    return hipGetLastError();
}

}  // namespace c3
