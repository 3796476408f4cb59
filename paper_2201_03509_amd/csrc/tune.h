// FFT plan choices: the default heuristic, the candidate set the autotuner
// times, and the table of measured winners (with a small JSON cache format).
//
// The paper measured FFT cost against length and cut each chunk to a cheap
// length (section 4.2); here every segment keeps all its samples, the length
// is padded to a 5-smooth size, and what is measured per size is the way the
// transform is split (M = M1 x M2), the column-tile width and the radix order.
#pragma once
#include <stdint.h>

#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace c3tune {

struct FftChoice {
    int M1 = 1, M2 = 1, B = 1;
    std::vector<int> r1, r2;
};

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

// S: complex elements one block holds in LDS (8192 FP32, 4096 FP64)
inline bool make_choice(int64_t M, int64_t M2, int S, int bmax, int order, FftChoice &c) {
    if (M2 < 1 || M % M2) return false;
    const int64_t M1 = M / M2;
    if (2 * M2 > S || M1 > S) return false;
    c.M1 = (int)M1;
    c.M2 = (int)M2;
    int B = pow2floor((int)(S / M1));
    if (B > bmax) B = bmax;
    const int bc = pow2ceil((int)M2);
    if (B > bc) B = bc;
    if (B < 1) B = 1;
    c.B = B;
    c.r1 = radices(M1, order);
    c.r2 = radices(M2, order);
    if ((int)c.r1.size() > 16 || (int)c.r2.size() > 16) return false;
    return true;
}

inline bool default_choice(int64_t M, int S, FftChoice &c) {
    // largest row length that fits, so the row pass (which carries the filter
    // and the draws) sees long contiguous rows
    int64_t best = 0;
    for (int64_t m2 = 1; m2 * 2 <= S && m2 <= M; ++m2)
        if (M % m2 == 0 && M / m2 <= S) best = m2;
    if (!best) return false;
    return make_choice(M, best, S, 64, 0, c);
}

inline std::vector<FftChoice> candidates(int64_t M, int S) {
    std::vector<FftChoice> out;
    std::vector<int64_t> m2s;
    for (int64_t m2 = 1; m2 * 2 <= S && m2 <= M; ++m2)
        if (M % m2 == 0 && M / m2 <= S) m2s.push_back(m2);
    // the few largest row lengths, two tile widths, two radix orders
    const size_t k0 = m2s.size() > 3 ? m2s.size() - 3 : 0;
    for (size_t i = k0; i < m2s.size(); ++i)
        for (int bmax : {16, 64})
            for (int order : {0, 1}) {
                FftChoice c;
                if (make_choice(M, m2s[i], S, bmax, order, c)) out.push_back(c);
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
        snprintf(buf, sizeof(buf), "%s    {\"mixed\": %d, \"M\": %lld, \"M1\": %d, \"M2\": %d, \"B\": %d, \"r1\": [",
                 first ? "" : ",\n", kv.first.first, (long long)kv.first.second, c.M1, c.M2, c.B);
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
        const char *c = s.c_str() + a + 1;
        while (c < s.c_str() + b) {
            char *e;
            long x = strtol(c, &e, 10);
            if (e == c) { ++c; continue; }
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
        long long mixed, M, M1, M2, B;
        if (num_after(o, "\"mixed\"", mixed) == std::string::npos) break;
        num_after(o, "\"M\"", M);
        num_after(o, "\"M1\"", M1);
        num_after(o, "\"M2\"", M2);
        num_after(o, "\"B\"", B);
        FftChoice c;
        c.M1 = (int)M1;
        c.M2 = (int)M2;
        c.B = (int)B;
        list_after(o, "\"r1\"", c.r1);
        q = list_after(o, "\"r2\"", c.r2);
        if (q == std::string::npos) break;
        t.m[{(int)mixed, (int64_t)M}] = c;
    }
    ++t.version;
    if (fend != std::string::npos) {
        size_t a = s.find('{', fend), b = s.find('}', fend);
        size_t c = a;
        while (c != std::string::npos && c < b) {
            size_t k0 = s.find('"', c + 1);
            if (k0 == std::string::npos || k0 > b) break;
            size_t k1 = s.find('"', k0 + 1);
            size_t col = s.find(':', k1);
            strides[s.substr(k0 + 1, k1 - k0 - 1)] = (int)strtol(s.c_str() + col + 1, nullptr, 10);
            c = s.find(',', col);
        }
    }
    return true;
}

}  // namespace c3tune
