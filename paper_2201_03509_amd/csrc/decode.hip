// Huffman decode + undifferencing of the pointing streams (section 4.1), and
// of the TOD and flag streams (k_decode1: one stream, same format).
//
// Two kernels per call.
//
// k_tables turns every table blob into a DecTab: the canonical limits and a
// 12-bit prefix table giving the code length of every prefix whose codes all
// share one length.  The limit of a length L <= 12 is a multiple of 2^20 and
// never splits a prefix, and each longer length splits at most one, so the
// prefix table resolves the short codes and almost every long one too (the
// psi differences are near-uniform on +-4095: almost all psi codes are longer
// than 12 bits); only codes behind one of the <= 20 split prefixes search the
// limits.
//
// k_decode: a block owns up to C3_DEC_NT consecutive chunks of one segment; each
// thread parses one chunk of both streams from the side index, G codes per
// round, adds the symbol values to its running value (x_i = x_{i-1} + d_i),
// range-checks, and leaves the samples in an LDS tile; the block then writes
// the tile in rows of 16 consecutive samples of a chunk.
#include <mutex>

#include "common.h"

namespace {

constexpr int G = 16;          // symbols per thread per round
constexpr int GP = G + 1;      // padded LDS row (no bank conflicts on the column writes)
constexpr int SPLIT = 32 - C3_KLUT;

// smallest L in [from, maxlen] with w < lim[L]; 0 if there is none
__device__ __forceinline__ int code_len(const DecTab &T, unsigned long long w, int from) {
    for (int L = from; L <= T.maxlen; ++L)
        if (w < T.lim[L]) return L;
    return 0;
}
__device__ __forceinline__ int code_len(const DecTab &T, unsigned long long w) { return code_len(T, w, T.minlen); }

// length of the code at the top of win from its prefix-table entry e: e itself
// when the prefix resolves it (0 < e < 64); otherwise a search of the limits
// from the shortest length under the prefix (e = 64 | that length) or from
// minlen (e = 0: no code starts the prefix).  0: invalid code.
__device__ __forceinline__ int resolve_len(const DecTab &T, uint32_t win, int e) {
    if (e > 0 && e < 64) return e;
    return code_len(T, win, e ? (e & 63) : T.minlen);
}

__global__ __launch_bounds__(C3_NT) void k_tables(HuffDev hp, HuffDev hs, DecTab *tabs) {
    __shared__ DecTab T;
    const int b = blockIdx.x;
    const bool is_p = b < hp.ntable;
    const uint32_t *tables = is_p ? hp.tables : hs.tables;
    const int64_t *table_off = is_p ? hp.table_off : hs.table_off;
    const int t = is_p ? b : b - hp.ntable;
    const uint32_t *blob = tables + table_off[t];
    if (threadIdx.x == 0) {
        // blob: [nsym, maxlen, count_1 .. count_32, symbols...]
        unsigned long long first = 0;
        int64_t off = 0;
        int ok = 1;
        T.minlen = 33;
        T.maxlen = 0;
        for (int L = 1; L <= 32; ++L) {
            const uint32_t cnt = blob[1 + L];
            T.delta[L] = (int32_t)(off - (int64_t)first);
            const unsigned long long end = first + cnt;
            if (end > (1ull << L)) ok = 0;  // more codes of length <= L than L bits hold
            T.lim[L] = end << (32 - L);
            if (cnt) {
                if (T.minlen > 32) T.minlen = L;
                T.maxlen = L;
            }
            off += cnt;
            first = end << 1;
        }
        T.lim[0] = 0;
        T.delta[0] = 0;
        T.lim[33] = T.lim[32];
        T.delta[33] = 0;
        if (T.maxlen == 0 || off != (int64_t)blob[0]) ok = 0;
        if (T.minlen > 32) T.minlen = 32;
        T.nsym = ok ? (int32_t)off : 0;
        T.ok = ok;
        T.pad[0] = T.pad[1] = 0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (1 << C3_KLUT); e += C3_NT) {
        uint8_t v = 0;
        if (T.ok) {
            // code lengths only grow with the code value, so the prefix's
            // codes have lengths from L0 (its first) to L1 (its last)
            const unsigned long long w0 = (unsigned long long)e << SPLIT;
            const unsigned long long w1 = w0 | ((1ull << SPLIT) - 1);
            const int L0 = code_len(T, w0);
            const int L1 = code_len(T, w1);
            v = L0 == 0 ? 0 : (uint8_t)(L0 == L1 ? L0 : 64 | L0);
        }
        T.lut[e] = v;
    }
    __syncthreads();
    const uint4 *src = (const uint4 *)&T;
    uint4 *dst = (uint4 *)(tabs + b);
    for (int i = threadIdx.x; i < (int)(sizeof(DecTab) / 16); i += C3_NT) dst[i] = src[i];
}

// word 3 of a raw buffer resource on gfx9-family chips (untyped dword access)
#define C3_BUF_WORD3 0x00020000

// block-uniform values (one segment per block) moved to scalar registers, so
// that the buffer resources built from them are scalar
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ const void *uni(const void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const void *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *base, int32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)uni(base), 0, uni(bytes), C3_BUF_WORD3);
}

// dword i of a raw buffer: 0 past its end (the hardware range check)
__device__ __forceinline__ uint32_t buf_word(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)(4u * i), 0, 0);
}

// MSB-first bit reader over one segment's stream (a raw buffer, so reads
// past the end give zero bits).  Look-ahead: three pairs of words in stream
// order, kept as loaded (no reordering at load time).  A pair is loaded two
// pair-lengths before its first word is used, so the wait for it falls long
// after the load was issued.
struct BitReader {
    __amdgpu_buffer_rsrc_t rs;
    unsigned long long buf;  // next bits, MSB first; nbits of them valid
    uint2 n0, n1, n2;        // look-ahead words n0.x, n0.y, n1.x, ... in stream order
    uint32_t wp;             // next word to load
    int nbits, nh;           // nh: words of n0 not yet taken (2, 1 or 0)

    __device__ __forceinline__ uint2 load2(uint32_t p) const {
        return make_uint2(buf_word(rs, p), buf_word(rs, p + 1u));
    }
    __device__ void init(__amdgpu_buffer_rsrc_t r, uint32_t bit) {
        rs = r;
        const uint32_t p = bit >> 5;
        const int s = bit & 31;
        const uint2 w = load2(p);
        buf = (((unsigned long long)w.x << 32) | w.y) << s;
        nbits = 64 - s;
        n0 = load2(p + 2u);
        n1 = load2(p + 4u);
        n2 = load2(p + 6u);
        nh = 2;
        wp = p + 8u;
    }
    __device__ __forceinline__ void refill() {
        const bool need = nbits < 32;
        const uint32_t word = nh == 2 ? n0.x : n0.y;
        const int sh = need ? 32 - nbits : 0;
        buf |= need ? (unsigned long long)word << sh : 0ull;
        nbits += need ? 32 : 0;
        nh -= need ? 1 : 0;
        if (nh == 0) {  // every second refill: the pairs move up, one more is loaded
            n0 = n1;
            n1 = n2;
            nh = 2;
            n2 = load2(wp);
            wp += 2u;
        }
    }
    // the next 32 bits, the next code at the top (refilled first)
    __device__ __forceinline__ uint32_t window() {
        refill();
        return (uint32_t)(buf >> 32);
    }
    // drop the Lc bits of the code just read
    __device__ __forceinline__ void consume(int Lc) {
        buf <<= Lc;
        nbits -= Lc;
    }
    // symbol index of the next code; L = its length (0: invalid code)
    __device__ __forceinline__ int32_t next(const DecTab &T, int &L) {
        const uint32_t win = window();
        L = resolve_len(T, win, T.lut[win >> SPLIT]);
        const int Lc = L ? L : 1;
        const int32_t idx = (int32_t)(win >> (32 - Lc)) + T.delta[Lc];
        consume(Lc);
        return L ? idx : -1;
    }
};

__global__ __launch_bounds__(C3_DEC_NT) void k_decode(LayoutDev Ld, HuffDev hp, HuffDev hs,
                                                  const DecTab *__restrict__ tabs,
                                                  const DecodeTask *__restrict__ tasks,
                                                  int32_t *__restrict__ pix_out,
                                                  uint16_t *__restrict__ psi_out, uint32_t *err) {
    __shared__ DecTab cp, cq;
    __shared__ int32_t tp[C3_DEC_NT * GP];
    __shared__ uint16_t tq[C3_DEC_NT * GP];  // psi symbol indices, then psi values
    __shared__ uint32_t blk_err;

    const DecodeTask task = tasks[blockIdx.x];
    const int seg = task.seg;
    const int tid = threadIdx.x;
    const int64_t s0 = Ld.seg_off[seg];
    const int n = (int)(Ld.seg_off[seg + 1] - s0);
    const int C = hp.chunk_len;
    const int band = Ld.seg_band[seg];
    const uint32_t npix = (uint32_t)Ld.band[band].npix;
    const uint32_t npsi = (uint32_t)Ld.band[band].npsi;

    // this segment's two tables (an out-of-range table id is an invalid code)
    const int tpi = hp.seg_table[seg], tqi = hs.seg_table[seg];
    const bool tabs_ok = tpi >= 0 && tpi < hp.ntable && tqi >= 0 && tqi < hs.ntable;
    {
        const uint4 *sp = (const uint4 *)(tabs + (tabs_ok ? tpi : 0));
        const uint4 *sq = (const uint4 *)(tabs + hp.ntable + (tabs_ok ? tqi : 0));
        uint4 *dp = (uint4 *)&cp, *dq = (uint4 *)&cq;
        for (int i = tid; i < (int)(sizeof(DecTab) / 16); i += C3_DEC_NT) {
            dp[i] = sp[i];
            dq[i] = sq[i];
        }
        if (tid == 0) blk_err = 0;
    }
    __syncthreads();
    const bool codes_ok = tabs_ok && cp.ok && cq.ok && cq.nsym < 65535;
    // symbol arrays as raw buffers of nsym entries: an invalid index reads 0
    const __amdgpu_buffer_rsrc_t symp =
        raw_buffer(hp.tables + hp.table_off[tabs_ok ? tpi : 0] + 34, 4 * cp.nsym);
    const __amdgpu_buffer_rsrc_t symq =
        raw_buffer(hs.tables + hs.table_off[tabs_ok ? tqi : 0] + 34, 4 * cq.nsym);

    const int l = tid;
    const int c = task.chunk0 + l;
    // the side index must hold ceil(n / C) chunks for this segment
    const int nch_idx = (int)min(hp.seg_chunk_off[seg + 1] - hp.seg_chunk_off[seg],
                                 hs.seg_chunk_off[seg + 1] - hs.seg_chunk_off[seg]);
    const bool active = l < task.nchunk && c < nch_idx;
    uint32_t bad = codes_ok ? 0u : C3_ERR_CODE;
    if (l < task.nchunk && c >= nch_idx) bad |= C3_ERR_CHUNK;
    BitReader rp, rq;
    int ns = 0;
    int32_t xp = 0, xq = 0;      // running (undifferenced) values
    int32_t bitp = 0, bitq = 0;  // bits consumed by this chunk's codes
    uint32_t start_p = 0, start_q = 0;
    // the two streams of this segment as raw buffers (below 2^29 words each)
    const int64_t wp0 = hp.seg_word_off[seg], wq0 = hs.seg_word_off[seg];
    const int64_t nwp = hp.seg_word_off[seg + 1] - wp0, nwq = hs.seg_word_off[seg + 1] - wq0;
    const bool words_ok = nwp >= 0 && nwq >= 0 && nwp < (1ll << 29) && nwq < (1ll << 29);
    if (!words_ok) bad |= C3_ERR_CHUNK;
    const __amdgpu_buffer_rsrc_t rsp = raw_buffer(hp.words + wp0, words_ok ? (int32_t)(4 * nwp) : 0);
    const __amdgpu_buffer_rsrc_t rsq = raw_buffer(hs.words + wq0, words_ok ? (int32_t)(4 * nwq) : 0);
    if (active) {
        const int64_t gp = hp.seg_chunk_off[seg] + c;
        const int64_t gq = hs.seg_chunk_off[seg] + c;
        start_p = hp.chunk_bit[gp];
        start_q = hs.chunk_bit[gq];
        rp.init(rsp, start_p);
        rq.init(rsq, start_q);
        xp = hp.chunk_prev[gp];
        xq = hs.chunk_prev[gq];
        ns = (codes_ok && words_ok) ? min(C, n - c * C) : 0;
    }
    const int nround = (C + G - 1) / G;

    // one round: parse G codes of both streams per chunk (symbol indices into
    // this thread's tile row; psi tables hold at most 65535 symbols, checked
    // with the table), then their symbol values (gathers issued in groups),
    // running sums and range checks.  Values go to the thread's tile row, or
    // to registers (v0p, v0q) when the caller asks for them there.
    auto round = [&](int k0, bool to_regs, int32_t *v0p, uint16_t *v0q) {
        if (!(active && k0 < ns)) return;
#pragma unroll 4  // full unrolling runs out of scalar registers
        for (int k = 0; k < G; ++k) {
            // the two streams' table reads are issued together: both
            // prefix-table entries, then (after the rare searches) both
            // index offsets
            const uint32_t wp = rp.window(), wq = rq.window();
            const int ep = cp.lut[wp >> SPLIT], eq = cq.lut[wq >> SPLIT];
            const int Lp = resolve_len(cp, wp, ep), Lq = resolve_len(cq, wq, eq);
            const int Lcp = Lp ? Lp : 1, Lcq = Lq ? Lq : 1;
            const int32_t ip = (int32_t)(wp >> (32 - Lcp)) + cp.delta[Lcp];
            const int32_t iq = (int32_t)(wq >> (32 - Lcq)) + cq.delta[Lcq];
            rp.consume(Lcp);
            rq.consume(Lcq);
            const bool v = k0 + k < ns;
            bad |= (v && (Lp == 0 || Lq == 0)) ? C3_ERR_CODE : 0u;
            bitp += v ? Lp : 0;
            bitq += v ? Lq : 0;
            tp[l * GP + k] = Lp ? ip : -1;
            tq[l * GP + k] = (uint16_t)(Lq ? iq : 0xFFFF);
        }
#pragma unroll
        for (int h = 0; h < G; h += G / 2) {
            int32_t gp_[G / 2], gq_[G / 2];
#pragma unroll
            for (int k = 0; k < G / 2; ++k) {
                gp_[k] = (int32_t)buf_word(symp, (uint32_t)tp[l * GP + h + k]);
                gq_[k] = (int32_t)buf_word(symq, (uint32_t)tq[l * GP + h + k]);
            }
#pragma unroll
            for (int k = 0; k < G / 2; ++k) {
                const bool v = k0 + h + k < ns;
                xp += v ? gp_[k] : 0;
                xq += v ? gq_[k] : 0;
                const bool okp = (uint32_t)xp < npix, okq = (uint32_t)xq < npsi;
                bad |= (v && !okp) ? C3_ERR_PIX : 0u;
                bad |= (v && !okq) ? C3_ERR_PSI : 0u;
                if (to_regs) {
                    v0p[h + k] = okp ? xp : 0;
                    v0q[h + k] = (uint16_t)(okq ? xq : 0);
                } else {
                    tp[l * GP + h + k] = okp ? xp : 0;
                    tq[l * GP + h + k] = (uint16_t)(okq ? xq : 0);
                }
            }
        }
    };
    // write the tile of the round at k0: 16-lane rows of consecutive samples
    // of one chunk
    auto write_tile = [&](int k0) {
#pragma unroll 4
        for (int m = 0; m < G; ++m) {
            const int q = m * C3_DEC_NT + tid;
            const int ll = q >> 4, kk = q & 15;
            const int cc = task.chunk0 + ll;
            const int t = cc * C + k0 + kk;
            if (ll < task.nchunk && cc < nch_idx && k0 + kk < C && t < n && codes_ok && words_ok) {
                pix_out[s0 + t] = tp[ll * GP + kk];
                psi_out[s0 + t] = tq[ll * GP + kk];
            }
        }
    };
    if (nround == 2) {
        // a chunk of two rounds: every store after every load.  Stores and
        // loads share one in-order completion counter, so a store followed by
        // a load that is waited on costs the store's whole latency; the first
        // round's values wait in registers until the second round's loads
        // are done.
        int32_t v0p[G];
        uint16_t v0q[G];
        round(0, true, v0p, v0q);
        round(G, false, nullptr, nullptr);
        __syncthreads();
        write_tile(G);
        __syncthreads();
        if (active && ns > 0) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                tp[l * GP + k] = v0p[k];
                tq[l * GP + k] = v0q[k];
            }
        }
        __syncthreads();
        write_tile(0);
    } else {
        for (int rd = 0; rd < nround; ++rd) {
            round(rd * G, false, nullptr, nullptr);
            __syncthreads();
            write_tile(rd * G);
            __syncthreads();
        }
    }
    // chunk boundary consistency with the side index: the codes of chunk c end
    // where chunk c + 1 starts, and the running value meets its stored one
    if (active && codes_ok && c + 1 < nch_idx) {
        const int64_t gp = hp.seg_chunk_off[seg] + c + 1;
        const int64_t gq = hs.seg_chunk_off[seg] + c + 1;
        if ((int64_t)start_p + bitp != (int64_t)hp.chunk_bit[gp] || xp != hp.chunk_prev[gp]) bad |= C3_ERR_CHUNK;
        if ((int64_t)start_q + bitq != (int64_t)hs.chunk_bit[gq] || xq != hs.chunk_prev[gq]) bad |= C3_ERR_CHUNK;
    }
    if (active && ns > 0) {
        if ((int64_t)start_p + bitp > 32 * nwp) bad |= C3_ERR_CHUNK;
        if ((int64_t)start_q + bitq > 32 * nwq) bad |= C3_ERR_CHUNK;
    }
    if (bad) atomicOr(&blk_err, bad);
    __syncthreads();
    if (tid == 0 && blk_err) atomicOr(err, blk_err);
}

// ------------------------------------------------------- allocation-free variant
// Scratch of decode_pointing_noalloc: the decoding tables of both streams,
// then the work list, in one static array per device (held until the process
// ends).  Host code uses only the address hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[C3_NOALLOC_BYTES];

// The work list of k_decode in segment order: segment s takes
// ceil(ceil(n_s / C) / C3_DEC_NT) tasks, starting at the sum of the counts before
// it.  One block scans the counts 1024 segments at a time.  Exactly ntask
// entries are written: the host counts them from its mirror of the offsets;
// entries the device offsets do not fill are empty tasks (no chunk), and
// none is written past ntask, whatever the device offsets hold.
__global__ __launch_bounds__(1024) void k_decode_tasks(const int64_t *__restrict__ seg_off, int nseg, int C,
                                                       int ntask, DecodeTask *__restrict__ tasks) {
    __shared__ int32_t pre[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nseg; base += 1024) {
        const int s = base + tid;
        int nch = 0, cnt = 0;
        if (s < nseg) {
            const int64_t n = seg_off[s + 1] - seg_off[s];
            nch = n > 0 ? (int)((n + C - 1) / C) : 0;
            cnt = (nch + C3_DEC_NT - 1) / C3_DEC_NT;
        }
        pre[tid] = cnt;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
            const int v = tid >= o ? pre[tid - o] : 0;
            __syncthreads();
            pre[tid] += v;
            __syncthreads();
        }
        const int64_t start = carry + pre[tid] - cnt;
        for (int j = 0; j < cnt && start + j < ntask; ++j)
            tasks[start + j] = DecodeTask{s, j * C3_DEC_NT, min(C3_DEC_NT, nch - j * C3_DEC_NT), 0};
        __syncthreads();
        if (tid == 1023) carry += pre[1023];
        __syncthreads();
    }
    for (int64_t i = carry + tid; i < ntask; i += 1024) tasks[i] = DecodeTask{0, 0, 0, 0};
}

// One integer stream per segment (the TOD or the flag words): the same chunk
// parse and undifferencing as k_decode, without range checks; the tile is
// written as KIND 0: FP32 quantum * x, 1: FP64 quantum * x, 2: flag words
// (and, if mask_out, the mask byte (x & flag_mask) == 0).
template <int KIND>
__global__ __launch_bounds__(C3_DEC_NT) void k_decode1(LayoutDev Ld, HuffDev h, const DecTab *__restrict__ tabs,
                                                   const DecodeTask *__restrict__ tasks, double quantum,
                                                   uint32_t flag_mask, void *__restrict__ out,
                                                   uint8_t *__restrict__ mask_out, uint32_t *err) {
    __shared__ DecTab cp;
    __shared__ int32_t tp[C3_DEC_NT * GP];
    __shared__ uint32_t blk_err;

    const DecodeTask task = tasks[blockIdx.x];
    const int seg = task.seg;
    const int tid = threadIdx.x;
    const int64_t s0 = Ld.seg_off[seg];
    const int n = (int)(Ld.seg_off[seg + 1] - s0);
    const int C = h.chunk_len;

    const int ti = h.seg_table[seg];
    const bool tabs_ok = ti >= 0 && ti < h.ntable;
    {
        const uint4 *sp = (const uint4 *)(tabs + (tabs_ok ? ti : 0));
        uint4 *dp = (uint4 *)&cp;
        for (int i = tid; i < (int)(sizeof(DecTab) / 16); i += C3_DEC_NT) dp[i] = sp[i];
        if (tid == 0) blk_err = 0;
    }
    __syncthreads();
    const bool codes_ok = tabs_ok && cp.ok;
    const __amdgpu_buffer_rsrc_t sym = raw_buffer(h.tables + h.table_off[tabs_ok ? ti : 0] + 34, 4 * cp.nsym);

    const int l = tid;
    const int c = task.chunk0 + l;
    const int nch_idx = (int)(h.seg_chunk_off[seg + 1] - h.seg_chunk_off[seg]);
    const bool active = l < task.nchunk && c < nch_idx;
    uint32_t bad = codes_ok ? 0u : C3_ERR_CODE;
    if (l < task.nchunk && c >= nch_idx) bad |= C3_ERR_CHUNK;
    BitReader rd;
    int ns = 0;
    int32_t x = 0, bits = 0;
    uint32_t start = 0;
    const int64_t w0 = h.seg_word_off[seg];
    const int64_t nw = h.seg_word_off[seg + 1] - w0;
    const bool words_ok = nw >= 0 && nw < (1ll << 29);
    if (!words_ok) bad |= C3_ERR_CHUNK;
    const __amdgpu_buffer_rsrc_t rs = raw_buffer(h.words + w0, words_ok ? (int32_t)(4 * nw) : 0);
    if (active) {
        const int64_t g = h.seg_chunk_off[seg] + c;
        start = h.chunk_bit[g];
        rd.init(rs, start);
        x = h.chunk_prev[g];
        ns = (codes_ok && words_ok) ? min(C, n - c * C) : 0;
    }
    const int nround = (C + G - 1) / G;
    for (int r = 0; r < nround; ++r) {
        const int k0 = r * G;
        if (active && k0 < ns) {
#pragma unroll 4
            for (int k = 0; k < G; ++k) {
                int L;
                const int32_t ix = rd.next(cp, L);
                const bool v = k0 + k < ns;
                bad |= (v && L == 0) ? C3_ERR_CODE : 0u;
                bits += v ? L : 0;
                tp[l * GP + k] = ix;
            }
#pragma unroll
            for (int hh = 0; hh < G; hh += G / 2) {
                int32_t gv[G / 2];
#pragma unroll
                for (int k = 0; k < G / 2; ++k) gv[k] = (int32_t)buf_word(sym, (uint32_t)tp[l * GP + hh + k]);
#pragma unroll
                for (int k = 0; k < G / 2; ++k) {
                    x += (k0 + hh + k < ns) ? gv[k] : 0;
                    tp[l * GP + hh + k] = x;
                }
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int m = 0; m < G; ++m) {
            const int q = m * C3_DEC_NT + tid;
            const int ll = q >> 4, kk = q & 15;
            const int cc = task.chunk0 + ll;
            const int t = cc * C + k0 + kk;
            if (ll < task.nchunk && cc < nch_idx && k0 + kk < C && t < n && codes_ok && words_ok) {
                const int32_t v = tp[ll * GP + kk];
                if constexpr (KIND == 0) {
                    ((float *)out)[s0 + t] = (float)(quantum * (double)v);
                } else if constexpr (KIND == 1) {
                    ((double *)out)[s0 + t] = quantum * (double)v;
                } else {
                    if (out) ((uint32_t *)out)[s0 + t] = (uint32_t)v;
                    if (mask_out) mask_out[s0 + t] = ((uint32_t)v & flag_mask) == 0u;
                }
            }
        }
        __syncthreads();
    }
    if (active && codes_ok && c + 1 < nch_idx) {
        const int64_t g = h.seg_chunk_off[seg] + c + 1;
        if ((int64_t)start + bits != (int64_t)h.chunk_bit[g] || x != h.chunk_prev[g]) bad |= C3_ERR_CHUNK;
    }
    if (active && ns > 0 && (int64_t)start + bits > 32 * nw) bad |= C3_ERR_CHUNK;
    if (bad) atomicOr(&blk_err, bad);
    __syncthreads();
    if (tid == 0 && blk_err) atomicOr(err, blk_err);
}

}  // namespace

namespace c3 {

hipError_t launch_decode_stream(hipStream_t st, const LayoutDev &L, const HuffDev &h, DecTab *tabs,
                                const DecodeTask *tasks, int ntask, int kind, double quantum,
                                uint32_t flag_mask, void *out, uint8_t *mask_out, uint32_t *err) {
    if (ntask <= 0) return hipSuccess;
    HuffDev none = h;
    none.ntable = 0;
    hipLaunchKernelGGL(k_tables, dim3(h.ntable), dim3(C3_NT), 0, st, h, none, tabs);
    if (kind == 0)
        hipLaunchKernelGGL(k_decode1<0>, dim3(ntask), dim3(C3_DEC_NT), 0, st, L, h, tabs, tasks, quantum, flag_mask,
                           out, mask_out, err);
    else if (kind == 1)
        hipLaunchKernelGGL(k_decode1<1>, dim3(ntask), dim3(C3_DEC_NT), 0, st, L, h, tabs, tasks, quantum, flag_mask,
                           out, mask_out, err);
    else
        hipLaunchKernelGGL(k_decode1<2>, dim3(ntask), dim3(C3_DEC_NT), 0, st, L, h, tabs, tasks, quantum, flag_mask,
                           out, mask_out, err);
    return hipGetLastError();
}

hipError_t noalloc_scratch(void **ptr) {
    // one address per device, looked up once with that device current
    static std::mutex mu;
    static void *addr[C3_MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= C3_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_decode_noalloc(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                                 void *scratch_ptr, int ntask, int32_t *pix_out, uint16_t *psi_out,
                                 uint32_t *err) {
    if (ntask <= 0) return hipSuccess;
    DecTab *tabs = (DecTab *)scratch_ptr;
    DecodeTask *tasks = (DecodeTask *)((char *)scratch_ptr + noalloc_task_offset(hp.ntable + hs.ntable));
    hipLaunchKernelGGL(k_decode_tasks, dim3(1), dim3(1024), 0, st, L.seg_off, L.nseg, hp.chunk_len, ntask, tasks);
    return launch_decode(st, L, hp, hs, tabs, tasks, ntask, pix_out, psi_out, err);
}

hipError_t launch_decode(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                         DecTab *tabs, const DecodeTask *tasks, int ntask, int32_t *pix_out,
                         uint16_t *psi_out, uint32_t *err) {
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tables, dim3(hp.ntable + hs.ntable), dim3(C3_NT), 0, st, hp, hs, tabs);
    hipLaunchKernelGGL(k_decode, dim3(ntask), dim3(C3_DEC_NT), 0, st, L, hp, hs, tabs, tasks, pix_out,
                       psi_out, err);
    return hipGetLastError();
}

}  // namespace c3
