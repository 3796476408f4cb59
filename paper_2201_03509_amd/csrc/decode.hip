// Huffman decode + undifferencing of the pointing streams (section 4.1).
//
// Work split: a block owns up to C3_NT consecutive chunks of one segment; each
// thread parses one chunk of both streams (pixel and psi) from the side index,
// G codes per round, and leaves symbol *indices* in an LDS tile.  The block
// then walks the tile row by row (16 consecutive samples of one chunk per
// 16-lane row): it fetches the symbol values, undoes the differencing with a
// 16-lane inclusive scan plus the row's running value, range-checks and writes
// contiguous runs.  The per-thread critical path is bit parsing only.
//
// Canonical decoding: with the next 32 bits w of the stream left-justified,
// the code length is the smallest L with w < lim[L], lim[L] = (first_L +
// count_L) << (32 - L) (looked up on the first 12 bits when L <= 12); the
// symbol is sym[off_L + (w >> (32-L)) - first_L].
#include "common.h"

namespace {

constexpr int G = 16;          // symbols per thread per round (one 16-lane row each)
constexpr int GP = G + 1;      // padded LDS row (no bank conflicts on the column writes)
constexpr int KLUT = 12;       // code-length lookup on the first 12 bits

struct Canon {
    unsigned long long lim[34];
    int32_t delta[34];         // off_L - first_L
    int32_t minlen, maxlen;
    const int32_t *sym;
    uint8_t lut[1 << KLUT];    // code length for codes <= KLUT bits, else 0
};

__device__ void build_canon_serial(Canon &c, const uint32_t *blob) {
    unsigned long long first = 0;
    int32_t off = 0;
    c.minlen = 33;
    c.maxlen = 0;
    for (int L = 1; L <= 32; ++L) {
        uint32_t cnt = blob[1 + L];
        c.delta[L] = off - (int32_t)first;
        c.lim[L] = (first + cnt) << (32 - L);
        if (cnt) {
            if (c.minlen > 32) c.minlen = L;
            c.maxlen = L;
        }
        off += cnt;
        first = (first + cnt) << 1;
    }
    c.lim[0] = 0;
    c.delta[0] = 0;
    c.lim[33] = c.lim[32];
    c.delta[33] = 0;
    if (c.minlen > 32) c.minlen = 32;
    c.sym = (const int32_t *)(blob + 34);
}

__device__ void build_lut(Canon &c, int tid) {
    const int top = min(c.maxlen, KLUT);
    for (int e = tid; e < (1 << KLUT); e += C3_NT) {
        const unsigned long long w = (unsigned long long)e << (32 - KLUT);
        uint8_t L = 0;
        for (int l = c.minlen; l <= top; ++l)
            if (w < c.lim[l]) {
                L = (uint8_t)l;
                break;
            }
        c.lut[e] = L;
    }
}

// MSB-first bit reader with two doublewords of look-ahead in registers
struct BitReader {
    const uint32_t *w;
    int64_t wp, wend;
    unsigned long long buf, n0, n1;
    int nbits, nh;
    int64_t consumed;

    __device__ __forceinline__ unsigned long long load2(int64_t p) const {
        const unsigned long long a = p < wend ? w[p] : 0u;
        const unsigned long long b = p + 1 < wend ? w[p + 1] : 0u;
        return (a << 32) | b;
    }
    __device__ void init(const uint32_t *words, int64_t nw, uint32_t bit) {
        w = words;
        wend = nw;
        const int64_t p = bit >> 5;
        const int s = bit & 31;
        buf = load2(p) << s;
        nbits = 64 - s;
        n0 = load2(p + 2);
        n1 = load2(p + 4);
        nh = 2;
        wp = p + 6;
        consumed = bit;
    }
    __device__ __forceinline__ void refill() {
        if (nbits < 32) {
            buf |= (n0 >> 32) << (32 - nbits);
            nbits += 32;
            n0 <<= 32;
            if (--nh == 0) {
                n0 = n1;
                nh = 2;
                n1 = load2(wp);
                wp += 2;
            }
        }
    }
    // index of the next code's symbol in the table; sets bad on an invalid code
    __device__ __forceinline__ int32_t next(const Canon &c, uint32_t &bad) {
        refill();
        const uint32_t win = (uint32_t)(buf >> 32);
        int L = c.lut[win >> (32 - KLUT)];
        if (L == 0) {
            L = KLUT + 1;
            while (L < c.maxlen && (unsigned long long)win >= c.lim[L]) ++L;
            if (L > 32 || (unsigned long long)win >= c.lim[L]) {
                bad |= C3_ERR_CODE;
                L = c.maxlen;
                buf <<= L;
                nbits -= L;
                consumed += L;
                return 0;
            }
        }
        const int32_t idx = (int32_t)(win >> (32 - L)) + c.delta[L];
        buf <<= L;
        nbits -= L;
        consumed += L;
        return idx;
    }
};

__global__ __launch_bounds__(C3_NT) void k_decode(LayoutDev Ld, HuffDev hp, HuffDev hs,
                                                  const DecodeTask *__restrict__ tasks,
                                                  int32_t *__restrict__ pix_out,
                                                  uint16_t *__restrict__ psi_out, uint32_t *err) {
    __shared__ Canon cp, cq;
    __shared__ int32_t tp[C3_NT * GP];
    __shared__ int32_t tq[C3_NT * GP];
    __shared__ int32_t carp[C3_NT], carq[C3_NT];
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

    if (tid == 0) {
        build_canon_serial(cp, hp.tables + hp.table_off[hp.seg_table[seg]]);
        blk_err = 0;
    }
    if (tid == 64) build_canon_serial(cq, hs.tables + hs.table_off[hs.seg_table[seg]]);
    __syncthreads();
    build_lut(cp, tid);
    build_lut(cq, tid);

    const int l = tid;
    const int c = task.chunk0 + l;
    // the side index must hold ceil(n / C) chunks for this segment
    const int nch_idx = (int)min(hp.seg_chunk_off[seg + 1] - hp.seg_chunk_off[seg],
                                 hs.seg_chunk_off[seg + 1] - hs.seg_chunk_off[seg]);
    const bool active = l < task.nchunk && c < nch_idx;
    uint32_t bad = 0;
    if (l < task.nchunk && c >= nch_idx) bad |= C3_ERR_CHUNK;
    BitReader rp, rq;
    int ns = 0;
    if (active) {
        const int64_t gp = hp.seg_chunk_off[seg] + c;
        const int64_t gq = hs.seg_chunk_off[seg] + c;
        const int64_t wp0 = hp.seg_word_off[seg], wq0 = hs.seg_word_off[seg];
        rp.init(hp.words + wp0, hp.seg_word_off[seg + 1] - wp0, hp.chunk_bit[gp]);
        rq.init(hs.words + wq0, hs.seg_word_off[seg + 1] - wq0, hs.chunk_bit[gq]);
        carp[l] = hp.chunk_prev[gp];
        carq[l] = hs.chunk_prev[gq];
        ns = min(C, n - c * C);
    }
    __syncthreads();
    const int nround = (C + G - 1) / G;
    const int lane16 = tid & 15;

    for (int rd = 0; rd < nround; ++rd) {
        const int k0 = rd * G;
        if (active) {
#pragma unroll 4
            for (int k = 0; k < G; ++k) {
                if (k0 + k < ns) {
                    tp[l * GP + k] = rp.next(cp, bad);
                    tq[l * GP + k] = rq.next(cq, bad);
                }
            }
        }
        __syncthreads();
        // rows of 16 samples: resolve symbols (every gather issued before the
        // first scan), undo the differencing with a 16-lane inclusive scan plus
        // the row's running value, write out
        int32_t valp[G], valq[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int q = m * C3_NT + tid;
            const int ll = q >> 4, kk = q & 15;
            const int t = (task.chunk0 + ll) * C + k0 + kk;
            const bool valid = ll < task.nchunk && task.chunk0 + ll < nch_idx && t < n;
            valp[m] = valid ? cp.sym[tp[ll * GP + kk]] : 0;
            valq[m] = valid ? cq.sym[tq[ll * GP + kk]] : 0;
        }
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int q = m * C3_NT + tid;
            const int ll = q >> 4, kk = q & 15;
            const int t = (task.chunk0 + ll) * C + k0 + kk;
            const bool valid = ll < task.nchunk && task.chunk0 + ll < nch_idx && t < n;
            int32_t vp = valp[m], vq = valq[m];
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int yp = __shfl_up(vp, o, 16), yq = __shfl_up(vq, o, 16);
                if (lane16 >= o) {
                    vp += yp;
                    vq += yq;
                }
            }
            if (ll < task.nchunk) {
                const int32_t xp = carp[ll] + vp, xq = carq[ll] + vq;
                if (kk == 15) {
                    carp[ll] = xp;
                    carq[ll] = xq;
                }
                if (valid) {
                    int32_t pp = xp, bb = xq;
                    if ((uint32_t)pp >= npix) {
                        bad |= C3_ERR_PIX;
                        pp = 0;
                    }
                    if ((uint32_t)bb >= npsi) {
                        bad |= C3_ERR_PSI;
                        bb = 0;
                    }
                    pix_out[s0 + t] = pp;
                    psi_out[s0 + t] = (uint16_t)bb;
                }
            }
        }
        __syncthreads();
    }
    // chunk boundary consistency with the side index
    if (active && c + 1 < nch_idx) {
        const int64_t gp = hp.seg_chunk_off[seg] + c + 1;
        const int64_t gq = hs.seg_chunk_off[seg] + c + 1;
        if (rp.consumed != (int64_t)hp.chunk_bit[gp] || carp[l] != hp.chunk_prev[gp]) bad |= C3_ERR_CHUNK;
        if (rq.consumed != (int64_t)hs.chunk_bit[gq] || carq[l] != hs.chunk_prev[gq]) bad |= C3_ERR_CHUNK;
    }
    if (active && ns > 0) {
        if (rp.consumed > 32 * rp.wend) bad |= C3_ERR_CHUNK;
        if (rq.consumed > 32 * rq.wend) bad |= C3_ERR_CHUNK;
    }
    if (bad) atomicOr(&blk_err, bad);
    __syncthreads();
    if (tid == 0 && blk_err) atomicOr(err, blk_err);
}

}  // namespace

namespace c3 {

hipError_t launch_decode(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                         const DecodeTask *tasks, int ntask, int32_t *pix_out, uint16_t *psi_out,
                         uint32_t *err) {
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_decode, dim3(ntask), dim3(C3_NT), 0, st, L, hp, hs, tasks, pix_out, psi_out,
                       err);
    return hipGetLastError();
}

}  // namespace c3
