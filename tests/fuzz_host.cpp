// Host fuzz of the C-ABI's input parsing and validation, built with the
// address and undefined-behaviour sanitizers (tests/test_host_sanitizers.py):
// the tuning-cache JSON reader (mutated and random files, every choice it
// returns checked by choice_ok against its length), and the layout and
// stream checks on random tables (offsets, bands, sizes, NULL arrays) whose
// host arrays hold as many entries as the structs claim.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../paper_2201_03509_amd/csrc/tune.h"
#include "../paper_2201_03509_amd/csrc/validate.h"

static std::mt19937_64 rng(20220109);
static int64_t pick(const std::vector<int64_t> &v) { return v[rng() % v.size()]; }

static std::string valid_json() {
    c3tune::Table t;
    std::map<std::string, int> st;
    for (int i = 0; i < 4; ++i) {
        c3tune::FftChoice c;
        const int64_t M = pick({4096, 12800, 259200, 270000, 291600, 40000});
        if (!c3tune::default_choice(M, (int)(rng() & 1), c)) continue;
        t.put((int)(rng() & 1), M, c);
    }
    st["1024:78.8"] = 4728;
    st["512:32.5"] = 1950;
    return c3tune::to_json(t, st);
}

static std::string mutate(std::string s) {
    const int k = 1 + (int)(rng() % 8);
    const char alphabet[] = "{}[]:,\"-0123456789 abcdefMBr\n";
    for (int i = 0; i < k && !s.empty(); ++i) {
        const size_t p = rng() % s.size();
        switch (rng() % 5) {
        case 0: s[p] = alphabet[rng() % (sizeof(alphabet) - 1)]; break;
        case 1: s.erase(p, 1 + rng() % 8); break;
        case 2: s.insert(p, 1, alphabet[rng() % (sizeof(alphabet) - 1)]); break;
        case 3: s.resize(p); break;
        default: s.insert(p, std::to_string((long long)(rng() % 4) == 0 ? -((long long)rng() >> 1) : (long long)(rng() >> 1))); break;
        }
    }
    return s;
}

static void fuzz_json(int iters) {
    const std::string base = valid_json();
    for (int i = 0; i < iters; ++i) {
        std::string s = (i % 10 == 0) ? std::string() : mutate(base);
        if (i % 10 == 1) {  // random bytes
            s.resize(rng() % 200);
            for (char &c : s) c = (char)(rng() % 256);
        }
        c3tune::Table t;
        std::map<std::string, int> st;
        if (!c3tune::from_json(s, t, st)) continue;
        for (auto &kv : t.m) (void)c3tune::choice_ok(kv.second, kv.first.second, kv.first.first);
        for (auto &kv : st)
            if (kv.second <= 0 || kv.second > c3tune::kMaxStride) {
                std::fprintf(stderr, "stride %d accepted\n", kv.second);
                std::exit(2);
            }
    }
}

static void fuzz_layout(int iters) {
    const void *dev = (const void *)0x1000;  // device pointers are never dereferenced on the host
    for (int i = 0; i < iters; ++i) {
        const int nseg = (int)(rng() % 40) - 2;
        const int nband = (int)(rng() % 20) - 2;
        const int ns = nseg < 0 ? 0 : nseg;
        const int nb = nband < 1 ? 1 : nband;
        std::vector<int64_t> off(ns + 1, 0);
        std::vector<int32_t> band(ns + 1, 0);
        std::vector<tod_band> bands(nb);
        int64_t t = 0;
        for (int s = 0; s < ns; ++s) {
            const int64_t step = (rng() % 16 == 0) ? (int64_t)(rng() >> 2) * ((rng() & 1) ? -1 : 1)
                                                   : (int64_t)(rng() % 300000);
            t = (rng() % 32 == 0) ? (int64_t)rng() : (int64_t)((uint64_t)t + (uint64_t)step);
            off[s + 1] = t;
            band[s] = (int32_t)(rng() % (nb + 2)) - 1;
        }
        if (rng() % 8 == 0) off[0] = (int64_t)rng();
        int64_t poff = 0;
        for (int b = 0; b < nb; ++b) {
            const int64_t nside = (rng() % 8 == 0) ? (int64_t)(int32_t)rng() : (1 << (rng() % 14));
            bands[b].nside = (int32_t)nside;
            bands[b].npsi = (rng() % 16 == 0) ? 4095 : 4096;
            bands[b].npix = (rng() % 16 == 0) ? (int64_t)rng() : (int64_t)(12ull * (uint64_t)nside * (uint64_t)nside);
            bands[b].pix_off = (rng() % 16 == 0) ? (int64_t)rng() : poff;
            bands[b].fsamp = (rng() % 16 == 0) ? -1.0 : 32.5;
            poff = (int64_t)((uint64_t)poff + (uint64_t)bands[b].npix);  // wraps: the harness's own arithmetic
        }
        tod_layout L{};
        L.nseg = nseg;
        L.nband = nband;
        L.ndet = (int)(rng() % 4) - 1;
        L.nsamp = (rng() % 8 == 0) ? (int64_t)rng() : off[ns];
        L.npix_total = (rng() % 8 == 0) ? (int64_t)rng() : poff;
        L.seg_off = (const int64_t *)dev;
        L.seg_band = (const int32_t *)dev;
        L.seg_det = (const int32_t *)dev;
        L.h_seg_off = (rng() % 32 == 0) ? nullptr : off.data();
        L.h_seg_band = band.data();
        L.bands = bands.data();
        // the struct claims at most as many entries as the host arrays hold
        if (nband > nb) L.nband = nb;
        std::string msg;
        (void)c3val::check_layout(rng() % 64 == 0 ? nullptr : &L, msg);
    }
}

static void fuzz_huff(int iters) {
    const void *dev = (const void *)0x1000;
    for (int i = 0; i < iters; ++i) {
        tod_huff h{};
        const void **p[] = {(const void **)&h.words, (const void **)&h.seg_word_off, (const void **)&h.seg_table,
                            (const void **)&h.tables, (const void **)&h.table_off, (const void **)&h.chunk_bit,
                            (const void **)&h.chunk_prev, (const void **)&h.seg_chunk_off};
        for (auto q : p) *q = (rng() % 16 == 0) ? nullptr : dev;
        h.chunk_len = (int32_t)((rng() % 4 == 0) ? (int32_t)rng() : 32 * (int32_t)(rng() % 140));
        h.ntable = (int32_t)rng();
        std::string msg;
        (void)c3val::check_huff(rng() % 64 == 0 ? nullptr : &h, "fuzz", msg);
    }
}

int main(int argc, char **argv) {
    const int iters = argc > 1 ? std::atoi(argv[1]) : 20000;
    fuzz_json(iters);
    fuzz_layout(iters);
    fuzz_huff(iters);
    std::printf("fuzz ok: %d iterations each\n", iters);
    return 0;
}
