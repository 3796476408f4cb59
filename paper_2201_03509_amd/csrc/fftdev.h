// Device helpers shared by the FFT passes: radix-2/3/4/5/8 butterflies, the
// two-level w_N table, the mirrored, padded extension of a segment, and an
// in-register FFT of any 5-smooth length fixed at compile time (Stockham
// stages with their twiddles folded to constants).
#pragma once
#include <utility>

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

// ------------------------------------------ compile-time twiddle constants
// cos and sin of 2 pi m / L: the angle is reduced to [0, pi/2) with integer
// arithmetic (quarter turns are exact), then summed as Taylor series; 14
// terms at |x| <= pi/2 leave a truncation error below 1e-20.
constexpr double kQuarterTurn = 1.570796326794896619231321691639751442;

constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int i = 1; i < 14; ++i) {
        t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        s += t;
    }
    return s;
}
constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 14; ++i) {
        t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        s += t;
    }
    return s;
}
struct CS {
    double c, s;
};
constexpr CS cis2pi(long m, long L) {
    m %= L;
    if (m < 0) m += L;
    const long q = (4 * m) / L;      // whole quarter turns
    const long r = 4 * m - q * L;    // remainder, in units of (pi/2) / L
    const double th = kQuarterTurn * (double)r / (double)L;
    double c = taylor_cos(th), s = taylor_sin(th);
    for (long i = 0; i < q; ++i) {   // rotate by a quarter turn: (c, s) -> (-s, c)
        const double t = c;
        c = -s;
        s = t;
    }
    return {c, s};
}

// ------------------------------------------ radix plan of a 5-smooth length
struct RadPlan {
    int n;       // number of stages (-1: not 5-smooth)
    int r[16];   // radices in stage order
};
constexpr RadPlan rad_plan(int L) {
    RadPlan p{0, {0}};
    int a = 0, b = 0, c = 0;
    while (L % 2 == 0) { L /= 2; ++a; }
    while (L % 3 == 0) { L /= 3; ++b; }
    while (L % 5 == 0) { L /= 5; ++c; }
    while (a > 4 || a == 3) { p.r[p.n++] = 8; a -= 3; }
    if (a == 4) { p.r[p.n++] = 4; p.r[p.n++] = 4; }
    else if (a == 2) p.r[p.n++] = 4;
    else if (a == 1) p.r[p.n++] = 2;
    for (int i = 0; i < b; ++i) p.r[p.n++] = 3;
    for (int i = 0; i < c; ++i) p.r[p.n++] = 5;
    if (L != 1) p.n = -1;
    return p;
}
constexpr int stage_ns(int L, int s) {  // product of the radices before stage s
    const RadPlan p = rad_plan(L);
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= p.r[i];
    return ns;
}

// v *= w_NSR^E with w = e^(DIR 2 pi i / NSR); quarter turns as swaps
template <int DIR, int NSR, int E, typename T>
__device__ __forceinline__ void twiddle(cx<T> &v) {
    constexpr int m = ((DIR * E) % NSR + NSR) % NSR;
    if constexpr (m == 0) {
    } else if constexpr (4 * m == NSR) {
        v = cx<T>{-v.y, v.x};
    } else if constexpr (2 * m == NSR) {
        v = cx<T>{-v.x, -v.y};
    } else if constexpr (4 * m == 3 * NSR) {
        v = cx<T>{v.y, -v.x};
    } else {
        constexpr CS w = cis2pi(m, NSR);
        v = cmul(v, cx<T>{(T)w.c, (T)w.s});
    }
}

// butterfly J of a Stockham stage (radix R, NS points already combined):
// inputs x[J + t L/R], outputs y[(J / NS) NS R + J % NS + t NS]
template <int L, int DIR, int R, int NS, int J, typename T, int... t>
__device__ __forceinline__ void butterfly(const cx<T> *x, cx<T> *y, std::integer_sequence<int, t...>) {
    constexpr int LR = L / R, k = J % NS, jd = J / NS;
    cx<T> v[R] = {x[J + t * LR]...};
    (twiddle<DIR, NS * R, t * k>(v[t]), ...);
    dft<R, DIR>(v);
    ((y[jd * NS * R + k + t * NS] = v[t]), ...);
}

template <int L, int DIR, int S, typename T, int... J>
__device__ __forceinline__ void stage(const cx<T> *x, cx<T> *y, std::integer_sequence<int, J...>) {
    constexpr RadPlan P = rad_plan(L);
    constexpr int R = P.r[S];
    constexpr int NS = stage_ns(L, S);
    (butterfly<L, DIR, R, NS, J>(x, y, std::make_integer_sequence<int, R>{}), ...);
}

template <int L, int DIR, int S, typename T>
__device__ __forceinline__ void stages(cx<T> *x, cx<T> *y) {
    constexpr RadPlan P = rad_plan(L);
    if constexpr (S < P.n) {
        stage<L, DIR, S>(x, y, std::make_integer_sequence<int, L / P.r[S]>{});
        stages<L, DIR, S + 1>(y, x);
    }
}

// in-register FFT of length L (DIR -1 forward, +1 inverse, unnormalised)
template <int L, int DIR, typename T>
__device__ __forceinline__ void reg_fft(cx<T> (&x)[L]) {
    constexpr RadPlan P = rad_plan(L);
    static_assert(P.n > 0, "column length must be 5-smooth and > 1");
    cx<T> y[L];
    stages<L, DIR, 0>(x, y);
    if constexpr (P.n % 2 == 1) {
#pragma unroll
        for (int i = 0; i < L; ++i) x[i] = y[i];
    }
}

// split k1 = a Q + b for the four-step twiddle: Q + M1/Q table reads per lane
constexpr int tw_split(int M1) {
    int q = 1;
    while (q * q < M1) ++q;
    return q;
}

// coprime split R = A B of a composite radix for the prime-factor (Good-Thomas)
// algorithm, A the factor transformed first; 0 where R has no such split
constexpr int pfa_first(int R) {
    switch (R) {
    case 6: return 2;
    case 10: return 2;
    case 12: return 4;
    case 15: return 3;
    case 18: return 2;
    case 20: return 4;
    case 24: return 8;
    case 30: return 2;
    default: return 0;
    }
}
constexpr int inv_mod(int a, int m) {  // a^-1 mod m for coprime a, m > 1
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 0;
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_any(cx<T> *v);

// DFT of length R = A B, gcd(A, B) = 1, without twiddle factors: input n =
// (B n1 + A n2) mod R, output k = (B (B^-1 mod A) k1 + A (A^-1 mod B) k2) mod R,
// so that w_R^(n k) = w_A^(n1 k1) w_B^(n2 k2) (Chinese remainder theorem).  The
// index maps are compile-time constants: a permutation of registers.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_pfa(cx<T> *v) {
    constexpr int A = pfa_first(R), B = R / A;
    static_assert(A > 1 && B > 1 && A * B == R, "no coprime split");
    constexpr int EA = B * inv_mod(B % A, A), EB = A * inv_mod(A % B, B);
    cx<T> y[A][B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        cx<T> c[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) c[n1] = v[(B * n1 + A * n2) % R];
        dft_any<A, DIR>(c);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) y[k1][n2] = c[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        dft_any<B, DIR>(y[k1]);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[(EA * k1 + EB * k2) % R] = y[k1][k2];
    }
}

// radix-R butterfly of any 5-smooth R: the hand-written DFTs for 2, 3, 4, 5
// and 8, the prime-factor split for radices with coprime factors, the
// compile-time register FFT for prime powers (9, 16, 25, 27, 32)
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_any(cx<T> *v) {
    if constexpr (R == 2 || R == 3 || R == 4 || R == 5 || R == 8) {
        dft<R, DIR>(v);
    } else if constexpr (pfa_first(R) > 0) {
        dft_pfa<R, DIR>(v);
    } else {
        cx<T> x[R];
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = v[i];
        reg_fft<R, DIR>(x);
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = x[i];
    }
}

}  // namespace c3fft
