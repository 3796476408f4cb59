// Per-mode arithmetic of the FFT row passes, shared by the generic row kernel
// (fft.hip) and the row kernels compiled per row length (rowc.hip): the
// real-spectrum constrained-realisation filter and draw of the n_corr step
// (Eq. 4), the Fourier-diagonal filters of the gain and masked draws, the
// Whittle sums of the chi^2 and the periodogram bins of the noise draw.
#pragma once
#include "common.h"
#include "fftdev.h"
#include "rng.h"

namespace c3fft {
using namespace c3rng;

struct ModeCtx {
    double sigma0, lbase, lbase2, malpha;      // lbase = ln(fsamp / (N fknee)), lbase2 = log2 of it
    double invsqrtN, outscale;                 // 1/sqrt(N), sqrt(N)/M
    double l2s0, iscale;                       // 2 ln sigma0, 1/(N sigma0^2)
    uint2 key;
    uint32_t it_lo, it_hi, seed_hi;
    int M;
    int mean_only;
};

// constrained-realisation value nhat_k from the unnormalised spectrum E_k
template <typename T>
__device__ __forceinline__ cx<T> cr_mode(const ModeCtx &mc, int64_t k, cx<T> E) {
    const T s0 = (T)mc.sigma0;
    T q = 0;
    if (k > 0) {
        if constexpr (sizeof(T) == 4)  // q = 2^(-alpha log2(f_k / f_knee)), hardware exp2/log2
            q = __builtin_amdgcn_exp2f((float)mc.malpha *
                                       (__builtin_amdgcn_logf((float)k) + (float)mc.lbase2));
        else
            q = exp(mc.malpha * (log((double)k) + mc.lbase));
    }
    T inv;
    if constexpr (sizeof(T) == 4)
        inv = __builtin_amdgcn_rcpf(1.0f + q);
    else
        inv = 1.0 / (1.0 + q);
    cx<T> R = cscale(E, (T)mc.invsqrtN);
    cx<T> out = R;
    if (!mc.mean_only) {
        T z[4];
        normals4<T>(philox4x32_10(make_uint4((uint32_t)k, mc.it_lo, mc.it_hi, mc.seed_hi), mc.key), z);
        cx<T> W1, W2;
        if (k == 0 || k == mc.M) {
            W1 = {z[0], 0};
            W2 = {z[2], 0};
        } else {
            const T h = (T)0.70710678118654752440;
            W1 = {z[0] * h, z[1] * h};
            W2 = {z[2] * h, z[3] * h};
        }
        T sq;
        if constexpr (sizeof(T) == 4)
            sq = __builtin_amdgcn_sqrtf(q);
        else
            sq = sqrt(q);
        out.x += s0 * (W1.x + sq * W2.x);
        out.y += s0 * (W1.y + sq * W2.y);
    }
    return cscale(out, inv);
}

// q_k = (f_k / f_knee)^(-alpha), i.e. 1/P_k = q_k / sigma0^2 (q_0 = 0)
template <typename T>
__device__ __forceinline__ T q_of(const ModeCtx &mc, int64_t k) {
    if (k == 0) return (T)0;
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_exp2f((float)mc.malpha * (__builtin_amdgcn_logf((float)k) + (float)mc.lbase2));
    else
        return exp(mc.malpha * (log((double)k) + mc.lbase));
}

// Fourier-diagonal filter of the unitary spectrum E / sqrt(N): 1/P_k
// (which = 0), 1 / (1/sigma0^2 + 1/P_k) (which = 1) or the inverse total
// noise spectrum 1 / (sigma0^2 + P_k) = q / (sigma0^2 (1 + q)) (which = 2)
template <typename T>
__device__ __forceinline__ cx<T> filt_mode(const ModeCtx &mc, int64_t k, cx<T> E, int which) {
    const T q = q_of<T>(mc, k);
    const T s2 = (T)(mc.sigma0 * mc.sigma0);
    T h;
    if constexpr (sizeof(T) == 4) {
        // the hardware reciprocal (about 1 ulp) in place of IEEE divisions,
        // whose scale and fix-up sequences would dominate the filter
        const float is2 = (float)(1.0 / (mc.sigma0 * mc.sigma0));
        const float i1q = __builtin_amdgcn_rcpf(1.0f + q);
        h = which == 0 ? q * is2 : (which == 1 ? s2 * i1q : q * is2 * i1q);
    } else {
        h = which == 0 ? q / s2 : (which == 1 ? s2 / ((T)1 + q) : q / (s2 * ((T)1 + q)));
    }
    return cscale(E, (T)mc.invsqrtN * h);
}

// drawn unitary spectrum: W1 (which = 0) or W2 sqrt(1/P_k) (which = 1), the
// same Philox modes as the n_corr draw
template <typename T>
__device__ __forceinline__ cx<T> draw_mode(const ModeCtx &mc, int64_t k, int which) {
    T z[4];
    normals4<T>(philox4x32_10(make_uint4((uint32_t)k, mc.it_lo, mc.it_hi, mc.seed_hi), mc.key), z);
    const bool real = (k == 0 || k == mc.M);
    const T h = real ? (T)1 : (T)0.70710678118654752440;
    cx<T> W = which ? cx<T>{z[2] * h, real ? (T)0 : z[3] * h} : cx<T>{z[0] * h, real ? (T)0 : z[1] * h};
    if (which) {
        const T q = q_of<T>(mc, k);
        T sq;
        if constexpr (sizeof(T) == 4)
            sq = __builtin_amdgcn_sqrtf(q);
        else
            sq = sqrt(q);
        W = cscale(W, sq / (T)mc.sigma0);
    }
    return W;
}

// x0 = M b of the masked draw without b's large drawn term in the time
// domain: M (mu u) from the transformed input plus M F^H (W2 sqrt(1/P)) added
// per mode, h1 W2 sqrt(q) / sigma0 with h1 = sigma0^2 / (1 + q) (which = 3)
template <typename T>
__device__ __forceinline__ cx<T> x0_mode(const ModeCtx &mc, int64_t k, cx<T> E) {
    cx<T> v = filt_mode(mc, k, E, 1);
    if (!mc.mean_only) {
        const T q = q_of<T>(mc, k);
        const T h1 = (T)(mc.sigma0 * mc.sigma0) / ((T)1 + q);
        const cx<T> w = draw_mode<T>(mc, k, 1);
        v.x += h1 * w.x;
        v.y += h1 * w.y;
    }
    return v;
}

// Whittle sums for one mode k >= 1
struct Wsum {
    double a, b, c;  // sum(I/P + ln P), sum(1 - I/P), sum((1 - I/P) ln(f/fknee))
};
// (FP32 path: I/P and ln(f_k/f_knee) from the hardware exp2/log2, summed in FP64)
template <typename T>
__device__ __forceinline__ void whittle_mode(const ModeCtx &mc, int64_t k, cx<T> E, Wsum &s) {
    double IP, lr;
    if constexpr (sizeof(T) == 4) {
        const float lr2 = __builtin_amdgcn_logf((float)k) + (float)mc.lbase2;  // log2(f_k / f_knee)
        // I/P = |E|^2 / (N sigma0^2) (f_k/f_knee)^-alpha
        IP = (double)((E.x * E.x + E.y * E.y) * (float)mc.iscale *
                      __builtin_amdgcn_exp2f((float)mc.malpha * lr2));
        lr = (double)lr2 * 0.69314718055994530942;
    } else {
        lr = log((double)k) + mc.lbase;  // ln(f_k / f_knee)
        IP = (E.x * E.x + E.y * E.y) * mc.iscale * exp(mc.malpha * lr);
    }
    const double lnP = mc.l2s0 - mc.malpha * lr;
    s.a += IP + lnP;
    s.b += 1.0 - IP;
    s.c += (1.0 - IP) * lr;
}

// integer log-frequency bin of mode k >= 1: k = 1..7 one bin each; above,
// eight bins per octave split by the three bits after the leading one
__device__ __forceinline__ int xi_bin(int64_t k) {
    if (k < 8) return (int)k - 1;
    const int e = 63 - __builtin_clzll((unsigned long long)k);
    return 7 + 8 * (e - 3) + (int)(k >> (e - 3)) - 8;
}

// hist[b] += v over the lanes of a wave (b < 0: the lane has no value).  When
// every lane with a value shares lane 0's bin the wave sums them and adds
// once; otherwise each lane adds its own.  All lanes of the wave call it
// together.
__device__ __forceinline__ void hist_add(double *hist, int b, double v) {
    const int b0 = __builtin_amdgcn_readfirstlane(b);
    if (b0 >= 0 && __all(b == b0 || b < 0)) {
        double x = b < 0 ? 0.0 : v;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(&hist[b0], x);
    } else if (b >= 0) {
        atomicAdd(&hist[b], v);
    }
}

// the block's mode context: noise parameters of segment seg, scales of the
// length-N = 2M transform, Philox key and counter words
template <int MODE>
__device__ __forceinline__ ModeCtx mode_ctx(const FftArgs &a, int seg, int band, int M) {
    ModeCtx mc;
    const double fs = a.fsamp_band[band];
    const double N = 2.0 * M;
    if constexpr (MODE != 4) {  // the periodogram needs no noise parameters
        mc.sigma0 = a.sigma0[seg];
        mc.malpha = -a.alpha[seg];
        mc.lbase = log(fs / (N * a.fknee[seg]));
        mc.lbase2 = mc.lbase * 1.4426950408889634;
        mc.l2s0 = 2.0 * log(mc.sigma0);
        mc.iscale = 1.0 / (N * mc.sigma0 * mc.sigma0);
    } else {
        mc.sigma0 = mc.malpha = mc.lbase = mc.lbase2 = mc.l2s0 = mc.iscale = 0.0;
    }
    mc.invsqrtN = 1.0 / sqrt(N);
    mc.outscale = sqrt(N) / M;
    const uint64_t seed = a.seed_iter ? a.seed_iter[0] : 0, it = a.seed_iter ? a.seed_iter[1] : 0;
    mc.key = make_uint2((uint32_t)seed, (uint32_t)seg);
    mc.it_lo = (uint32_t)it;
    mc.it_hi = (uint32_t)(it >> 32);
    mc.seed_hi = (uint32_t)(seed >> 32);
    mc.M = M;
    mc.mean_only = a.mean_only;
    return mc;
}

}  // namespace c3fft
