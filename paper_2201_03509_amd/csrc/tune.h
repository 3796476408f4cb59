// FFT plan choices: the default heuristic, the candidate set the autotuner
// times, and the table of measured winners (with a small JSON cache format).
//
// The paper measured FFT cost against length and cut each chunk to a cheap
// length (section 4.2); here every segment keeps all its samples, the length
// is padded to a 5-smooth size, and what is measured per size is the way the
// transform is split (M = M1 x M2), the column kernel (register columns for a
// compiled M1, or LDS tiles of B columns), the tile width and the radix order.
#pragma once
#include <stdint.h>

#include "common.h"
#include "rowc.h"

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace c3tune {

// largest binning stride (revisit period, samples) the strided kernels take
constexpr long kMaxStride = 1l << 26;

struct FftChoice {
    int M1 = 1, M2 = 1, B = 1;
    int colreg = 0;  // 1: register column kernels (M1 compiled in)
    std::vector<int> r1, r2;
};

// longest row the row pass takes: two rows in one in-place LDS buffer of at
// most 80 KB, so that two row blocks share a CU (the stage code is sized for it)
inline int row_cap(int mixed) { return mixed ? 5040 : 2520; }
// complex elements of one LDS column tile buffer (two buffers per block)
inline int col_tile(int mixed) { return mixed ? 4096 : 2048; }

inline bool colreg_ok(int mixed, int64_t m1) {
    if (!mixed) return false;
    switch (m1) {
#define C3_TUNE_OK(M) case M:
        C3_COLREG_LIST(C3_TUNE_OK)
        return true;
#undef C3_TUNE_OK
    default:
        return false;
    }
}

inline std::vector<int> factor235(int64_t L) {
    std::vector<int> f;
    int a = 0, b = 0, c = 0;
    while (L % 2 == 0) { L /= 2; ++a; }
    while (L % 3 == 0) { L /= 3; ++b; }
    while (L % 5 == 0) { L /= 5; ++c; }
    if (L != 1) return {};
    f.push_back(a);
    f.push_back(b);
    f.push_back(c);
    return f;
}

// radix order: order 0 = 8s, 4, 2, 3s, 5s; order 1 = 5s, 3s, 2, 4, 8s
inline std::vector<int> radices(int64_t L, int order) {
    std::vector<int> f = factor235(L), r;
    if (f.empty()) return r;
    const int n8 = f[0] / 3, rem = f[0] % 3;
    std::vector<int> r4(n8, 8), r2;
    if (rem == 2) r4.push_back(4);
    if (rem == 1) r2.push_back(2);
    std::vector<int> r3(f[1], 3), r5(f[2], 5);
    if (order == 0) {
        r.insert(r.end(), r4.begin(), r4.end());
        r.insert(r.end(), r2.begin(), r2.end());
        r.insert(r.end(), r3.begin(), r3.end());
        r.insert(r.end(), r5.begin(), r5.end());
    } else {
        r.insert(r.end(), r5.begin(), r5.end());
        r.insert(r.end(), r3.begin(), r3.end());
        r.insert(r.end(), r2.begin(), r2.end());
        r.insert(r.end(), r4.begin(), r4.end());
    }
    return r;
}

inline bool row_radix_ok(int mixed, int r) {
    switch (r) {
#define C3_TUNE_R(R) case R:
    C3_ROW_RADICES_F64(C3_TUNE_R)
        return true;
    default:
        break;
    }
    if (!mixed) return false;
    switch (r) {
        C3_ROW_RADICES_F32(C3_TUNE_R)
#undef C3_TUNE_R
        return true;
    default:
        return false;
    }
}

// row-pass radices: the largest compiled radix dividing what is left, each
// time (about three stages for rows of a few thousand points in FP32); order
// 1 runs them smallest first
inline std::vector<int> row_radices(int64_t L, int mixed, int order) {
    std::vector<int> r;
    if (factor235(L).empty()) return r;
    while (L > 1) {
        int best = 1;
        for (int c = 2; c <= 32; ++c)
            if (L % c == 0 && row_radix_ok(mixed, c)) best = c;
        if (best == 1) return {};  // cannot happen: 2, 3 and 5 are compiled
        r.push_back(best);
        L /= best;
    }
    if (order == 1) std::reverse(r.begin(), r.end());
    return r;
}

inline int pow2floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}
inline int pow2ceil(int x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

inline bool make_choice(int64_t M, int64_t M2, int mixed, int bmax, int order, int colreg,
                        FftChoice &c) {
    if (M2 < 1 || M % M2) return false;
    const int64_t M1 = M / M2;
    if (M2 > row_cap(mixed)) return false;
    if (colreg ? !colreg_ok(mixed, M1) : M1 > col_tile(mixed)) return false;
    c.M1 = (int)M1;
    c.M2 = (int)M2;
    c.colreg = colreg;
    int B = 1;
    if (!colreg) {
        B = pow2floor((int)(col_tile(mixed) / M1));
        if (B > bmax) B = bmax;
        const int bc = pow2ceil((int)M2);
        if (B > bc) B = bc;
        if (B < 1) B = 1;
    }
    c.B = B;
    c.r1 = radices(M1, order);
    c.r2 = row_radices(M2, mixed, order);
    if ((int)c.r1.size() > 16 || (int)c.r2.size() > 16) return false;
    return true;
}

// row lengths of the LDS-tiled splits, ascending
inline std::vector<int64_t> lds_rows(int64_t M, int mixed) {
    std::vector<int64_t> m2s;
    for (int64_t m2 = 1; m2 <= row_cap(mixed) && m2 <= M; ++m2)
        if (M % m2 == 0 && M / m2 <= col_tile(mixed)) m2s.push_back(m2);
    return m2s;
}
// column lengths of the register splits, ascending
inline std::vector<int64_t> reg_cols(int64_t M, int mixed) {
    std::vector<int64_t> m1s;
    for (int64_t m1 = 2; m1 <= 100 && m1 <= M; ++m1)
        if (M % m1 == 0 && M / m1 <= row_cap(mixed) && colreg_ok(mixed, m1)) m1s.push_back(m1);
    return m1s;
}

// a choice (e.g. read back from a cache file) that the kernels can run: the
// split multiplies out, its column kernel exists, and every radix list
// multiplies to its length using only radices with a compiled stage
inline bool choice_ok(const FftChoice &c, int64_t M, int mixed) {
    if (c.M1 < 1 || c.M2 < 1 || (int64_t)c.M1 * c.M2 != M || c.M2 > row_cap(mixed)) return false;
    if (c.r1.size() > 16 || c.r2.size() > 16) return false;
    int64_t p2 = 1;
    for (int r : c.r2) {
        if (!row_radix_ok(mixed, r)) return false;
        p2 *= r;
    }
    if (p2 != c.M2) return false;
    if (c.colreg) return colreg_ok(mixed, c.M1);
    // the LDS column kernels index a tile by shifts and masks of B
    if (c.M1 > col_tile(mixed) || c.B < 1 || (c.B & (c.B - 1)) != 0 || (int64_t)c.M1 * c.B > col_tile(mixed))
        return false;
    int64_t p1 = 1;
    for (int r : c.r1) {
        if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return false;  // LDS column stages
        p1 *= r;
    }
    return p1 == c.M1;
}

inline bool default_choice(int64_t M, int mixed, FftChoice &c) {
    // register columns where a compiled M1 fits: the largest M1 up to 64
    // (fewest row-pass stages at two waves per SIMD in the column kernels),
    // else the largest; otherwise LDS column tiles with the longest rows
    const std::vector<int64_t> m1s = reg_cols(M, mixed);
    if (!m1s.empty()) {
        int64_t pick = m1s.back();
        for (int64_t m1 : m1s)
            if (m1 <= 64) pick = m1;
        // a row length with a compiled row kernel first (the same rule)
        int64_t pc = 0;
        for (int64_t m1 : m1s)
            if (c3rowc::compiled((int)(M / m1)) && (pc == 0 || m1 <= 64)) pc = m1;
        if (pc) pick = pc;
        return make_choice(M, M / pick, mixed, 64, 0, 1, c);
    }
    const std::vector<int64_t> m2s = lds_rows(M, mixed);
    if (m2s.empty()) return false;
    return make_choice(M, m2s.back(), mixed, 64, 0, 0, c);
}

inline std::vector<FftChoice> candidates(int64_t M, int mixed) {
    std::vector<FftChoice> out;
    // longest register columns first (the tuner keeps an earlier candidate
    // unless a later one is clearly faster; long columns and short rows are
    // the usual winners)
    const std::vector<int64_t> cols = reg_cols(M, mixed);
    for (auto it = cols.rbegin(); it != cols.rend(); ++it)
        for (int order : {0, 1}) {
            const int64_t m1 = *it;
            FftChoice c;
            if (make_choice(M, M / m1, mixed, 64, order, 1, c)) out.push_back(c);
        }
    // the two longest LDS-tiled rows, two radix orders
    const std::vector<int64_t> m2s = lds_rows(M, mixed);
    const size_t k0 = m2s.size() > 2 ? m2s.size() - 2 : 0;
    for (size_t i = k0; i < m2s.size(); ++i)
        for (int order : {0, 1}) {
            FftChoice c;
            if (make_choice(M, m2s[i], mixed, 16, order, 0, c)) out.push_back(c);
        }
    return out;
}

struct Table {
    std::map<std::pair<int, int64_t>, FftChoice> m;  // (mixed, M)
    uint64_t version = 0;
    bool get(int mixed, int64_t M, FftChoice &c) const {
        auto it = m.find({mixed, M});
        if (it == m.end()) return false;
        c = it->second;
        return true;
    }
    void put(int mixed, int64_t M, const FftChoice &c) {
        m[{mixed, M}] = c;
        ++version;
    }
};

inline std::string to_json(const Table &t, const std::map<std::string, int> &strides) {
    std::string s = "{\n  \"fft\": [\n";
    bool first = true;
    for (auto &kv : t.m) {
        const FftChoice &c = kv.second;
        char buf[256];
        snprintf(buf, sizeof(buf),
                 "%s    {\"mixed\": %d, \"M\": %lld, \"M1\": %d, \"M2\": %d, \"B\": %d, \"colreg\": %d, \"r1\": [",
                 first ? "" : ",\n", kv.first.first, (long long)kv.first.second, c.M1, c.M2, c.B, c.colreg);
        s += buf;
        for (size_t i = 0; i < c.r1.size(); ++i) s += (i ? ", " : "") + std::to_string(c.r1[i]);
        s += "], \"r2\": [";
        for (size_t i = 0; i < c.r2.size(); ++i) s += (i ? ", " : "") + std::to_string(c.r2[i]);
        s += "]}";
        first = false;
    }
    s += "\n  ],\n  \"bin_stride\": {";
    first = true;
    for (auto &kv : strides) {
        s += (first ? "" : ", ") + std::string("\"") + kv.first + "\": " + std::to_string(kv.second);
        first = false;
    }
    s += "}\n}\n";
    return s;
}

// minimal reader for the format written above
inline bool from_json(const std::string &s, Table &t, std::map<std::string, int> &strides) {
    size_t p = s.find("\"fft\"");
    if (p == std::string::npos) return false;
    auto num_after = [&](size_t from, const char *key, long long &v) -> size_t {
        size_t q = s.find(key, from);
        if (q == std::string::npos) return std::string::npos;
        q = s.find(':', q);
        if (q == std::string::npos) return std::string::npos;
        v = strtoll(s.c_str() + q + 1, nullptr, 10);
        return q;
    };
    auto list_after = [&](size_t from, const char *key, std::vector<int> &v) -> size_t {
        size_t q = s.find(key, from);
        if (q == std::string::npos) return std::string::npos;
        size_t a = s.find('[', q), b = s.find(']', q);
        v.clear();
        if (a == std::string::npos || b == std::string::npos || b < a) return std::string::npos;
        const char *c = s.c_str() + a + 1;
        while (c < s.c_str() + b) {
            char *e;
            long x = strtol(c, &e, 10);
            if (e == c) { ++c; continue; }
            if (v.size() >= 64) return std::string::npos;  // no plan has that many stages
            v.push_back((int)x);
            c = e;
        }
        return b;
    };
    const size_t fend = s.find("\"bin_stride\"");
    size_t q = p;
    while (true) {
        size_t o = s.find('{', q + 1);
        if (o == std::string::npos || (fend != std::string::npos && o > fend)) break;
        long long mixed, M, M1, M2, B, colreg = 0;
        if (num_after(o, "\"mixed\"", mixed) == std::string::npos) break;
        {
            // optional field: only read if it belongs to this record
            const size_t q_end = s.find('}', o);
            const size_t q_cr = s.find("\"colreg\"", o);
            if (q_cr != std::string::npos && q_cr < q_end) num_after(o, "\"colreg\"", colreg);
        }
        num_after(o, "\"M\"", M);
        num_after(o, "\"M1\"", M1);
        num_after(o, "\"M2\"", M2);
        num_after(o, "\"B\"", B);
        // out-of-range numbers make a choice that choice_ok rejects later
        auto clip = [](long long x) { return (int)std::max<long long>(-1, std::min<long long>(x, 1 << 30)); };
        FftChoice c;
        c.M1 = clip(M1);
        c.M2 = clip(M2);
        c.B = clip(B);
        c.colreg = colreg != 0;
        list_after(o, "\"r1\"", c.r1);
        q = list_after(o, "\"r2\"", c.r2);
        if (q == std::string::npos) break;
        t.m[{(int)mixed, (int64_t)M}] = c;
    }
    ++t.version;
    if (fend != std::string::npos) {
        size_t a = s.find('{', fend), b = s.find('}', fend);
        if (a == std::string::npos || b == std::string::npos || b < a) return false;
        size_t c = a;
        while (c != std::string::npos && c < b) {
            size_t k0 = s.find('"', c + 1);
            if (k0 == std::string::npos || k0 > b) break;
            size_t k1 = s.find('"', k0 + 1);
            if (k1 == std::string::npos || k1 > b) return false;
            size_t col = s.find(':', k1);
            if (col == std::string::npos || col > b) return false;
            const long v = strtol(s.c_str() + col + 1, nullptr, 10);
            // a revisit period is a positive sample count; keep those the
            // strided kernels can step through in 32-bit arithmetic
            if (v > 0 && v <= kMaxStride) strides[s.substr(k0 + 1, k1 - k0 - 1)] = (int)v;
            c = s.find(',', col);
        }
    }
    return true;
}

}  // namespace c3tune
