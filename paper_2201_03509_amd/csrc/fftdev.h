// Device helpers shared by the FFT passes: radix-2/3/4/5/8 butterflies, the
// two-level w_N table and the mirrored, padded extension of a segment.
#pragma once
#include "common.h"

namespace c3fft {
using c3::FftArgs;

// ---------------------------------------------------------------- DFT kernels
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {  // a * (DIR * i)
    return DIR < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T> *v) {
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T h = (T)0.86602540378443864676;  // sin(60 deg)
        cx<T> a = v[0], b = v[1], c = v[2];
        cx<T> t1 = cadd(b, c);
        cx<T> t2 = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
        cx<T> t3 = mul_i<DIR>(cscale(csub(b, c), h));
        v[0] = cadd(a, t1);
        v[1] = cadd(t2, t3);
        v[2] = csub(t2, t3);
    } else if constexpr (R == 4) {
        cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cx<T> s0 = cadd(a, c), d0 = csub(a, c);
        cx<T> s1 = cadd(b, d), d1 = mul_i<DIR>(csub(b, d));
        v[0] = cadd(s0, s1);
        v[2] = csub(s0, s1);
        v[1] = cadd(d0, d1);
        v[3] = csub(d0, d1);
    } else if constexpr (R == 8) {
        // split into two radix-4 transforms: a_k = x_k + x_k+4, b_k = (x_k - x_k+4) w8^k
        const T h = (T)0.70710678118654752440;
        cx<T> a[4], b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = cadd(v[k], v[k + 4]);
            b[k] = csub(v[k], v[k + 4]);
        }
        // w8 = (1 + DIR i)/sqrt2, w8^2 = DIR i, w8^3 = (-1 + DIR i)/sqrt2
        const cx<T> b1 = b[1], b3 = b[3];
        b[1] = cscale(cadd(b1, mul_i<DIR>(b1)), h);
        b[2] = mul_i<DIR>(b[2]);
        b[3] = cscale(csub(mul_i<DIR>(b3), b3), h);
        dft<4, DIR>(a);
        dft<4, DIR>(b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = a[k];
            v[2 * k + 1] = b[k];
        }
    } else {  // R == 5
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        cx<T> x0 = v[0];
        cx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        cx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        cx<T> a1 = {x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y};
        cx<T> a2 = {x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y};
        cx<T> b1 = mul_i<DIR>(cx<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
        cx<T> b2 = mul_i<DIR>(cx<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
        v[0] = cadd(x0, cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
}

// w_N^m for 0 <= m <= N from the two-level table
template <typename T>
__device__ __forceinline__ cx<T> twN(const cx<T> *pool, const FftPlan &p, int64_t m) {
    const cx<T> lo = pool[p.twlo + (m & 1023)];
    const cx<T> hi = pool[p.twhi + (m >> 10)];
    return cmul(hi, lo);
}

template <typename T>
__device__ __forceinline__ T load_as(const void *p, int f64, int64_t i) {
    return f64 ? (T)((const double *)p)[i] : (T)((const float *)p)[i];
}

// mirrored, padded extension of r = a - b at real index t
template <typename T>
__device__ __forceinline__ T ext_at(const FftArgs &a, int64_t s0, int n, int64_t t) {
    int64_t u = t < n ? t : (t < 2 * (int64_t)n ? 2 * (int64_t)n - 1 - t : 0);
    T v = load_as<T>(a.in_a, a.in_a_f64, s0 + u);
    if (a.in_b) v -= load_as<T>(a.in_b, a.in_b_f64, s0 + u);
    return v;
}

}  // namespace c3fft
