// Row lengths of the FFT row pass that have kernels compiled for them, and
// the stage plan of each (host and device): three radices, chosen at compile
// time, whose product is the row length L.
//
// Stage s of a length-L Stockham FFT with radix R_s, Ns = R_0 ... R_{s-1}:
// butterfly j (j < L/R) takes x[j + t L/R], t < R, multiplies input t by
// w_{Ns R}^(t (j mod Ns)), transforms, and writes y[(j / Ns) Ns R + j mod Ns
// + t Ns].  The twiddles of stages 1 and 2 sit in one table per row length:
// stage s, entry (k, t) at stage_off(L, s) + k (R_s - 1) + t - 1, the forward
// value e^(-2 pi i t k / (Ns R_s)) (the inverse transform uses its conjugate).
#pragma once

// every 5-smooth length in [2000, 5040] (the longest row the row pass takes)
#define C3_ROWC_LIST(X)                                                                          \
    X(2000) X(2025) X(2048) X(2160) X(2187) X(2250) X(2304) X(2400) X(2430) X(2500) X(2560)     \
    X(2592) X(2700) X(2880) X(2916) X(3000) X(3072) X(3125) X(3200) X(3240) X(3375) X(3456)     \
    X(3600) X(3645) X(3750) X(3840) X(3888) X(4000) X(4050) X(4096) X(4320) X(4374) X(4500)     \
    X(4608) X(4800) X(4860) X(5000)

namespace c3rowc {

// radices of a stage: 5-smooth, small enough that a butterfly's points fit a
// thread's registers
constexpr int kRadix[] = {4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32};
constexpr int kNRadix = sizeof(kRadix) / sizeof(kRadix[0]);

constexpr bool radix_ok(int r) {
    for (int i = 0; i < kNRadix; ++i)
        if (kRadix[i] == r) return true;
    return false;
}

struct Plan3 {
    int r[3];  // r[0] == 0: no three-stage plan
};

// the three-radix split of L with the smallest largest radix (ties: the
// largest smallest radix), in descending order
constexpr Plan3 plan(int L) {
    Plan3 best{{0, 0, 0}};
    int bmax = 1 << 30, bmin = 0;
    for (int i = 0; i < kNRadix; ++i) {
        const int a = kRadix[i];
        if (L % a) continue;
        for (int j = 0; j < kNRadix; ++j) {
            const int b = kRadix[j];
            if ((L / a) % b) continue;
            const int c = L / a / b;
            if (!radix_ok(c)) continue;
            const int mx = a > b ? (a > c ? a : c) : (b > c ? b : c);
            const int mn = a < b ? (a < c ? a : c) : (b < c ? b : c);
            if (mx < bmax || (mx == bmax && mn > bmin)) {
                bmax = mx;
                bmin = mn;
                const int md = a + b + c - mx - mn;
                best = Plan3{{mx, md, mn}};
            }
        }
    }
    return best;
}

constexpr int row_ns(int L, int s) {
    const Plan3 p = plan(L);
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= p.r[i];
    return ns;
}

// offset of stage s's twiddles (s = 1, 2) in the length's table, and its size
constexpr long stage_off(int L, int s) {
    const Plan3 p = plan(L);
    long off = 0;
    for (int i = 1; i < s; ++i) off += (long)row_ns(L, i) * (p.r[i] - 1);
    return off;
}
constexpr long table_size(int L) { return stage_off(L, 3); }

inline bool compiled(int L) {
    switch (L) {
#define C3_ROWC_CASE(LL) case LL:
        C3_ROWC_LIST(C3_ROWC_CASE)
#undef C3_ROWC_CASE
        return true;
    default:
        return false;
    }
}

}  // namespace c3rowc
