// Huffman decode + undifferencing of the pointing streams (section 4.1), with an
// optional fused projection and residual r = d - g P m for the sweep.
//
// Work split: a block owns up to C3_NT consecutive chunks of one segment; each
// thread decodes one chunk of both streams (pixel and psi) from the side
// index, C3_G symbols per round, into an LDS tile.  The block then walks the
// tile in sample order, so global writes (and the d/map reads of the fused
// residual) are contiguous runs instead of one address stream per thread.
//
// Canonical decoding: with the next 32 bits w of the stream left-justified,
// the code length is the smallest L with w < lim[L], lim[L] = (first_L +
// count_L) << (32 - L); the symbol is sym[off_L + (w >> (32-L)) - first_L].
#include "common.h"

namespace {

constexpr int G = 16;          // symbols per thread per round
constexpr int GP = G + 1;      // padded LDS row (no bank conflicts on the column writes)

struct Canon {
    unsigned long long lim[33];
    int32_t delta[33];         // off_L - first_L
    int32_t minlen, maxlen;
    const int32_t *sym;
};

__device__ void build_canon(Canon &c, const uint32_t *blob) {
    // serial: 32 lengths
    uint32_t nsym = blob[0];
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
    if (c.minlen > 32) c.minlen = 32;
    c.sym = (const int32_t *)(blob + 34);
    (void)nsym;
}

struct BitReader {
    const uint32_t *w;
    int64_t wp, wend;
    unsigned long long buf;
    int nbits;
    int64_t consumed;

    __device__ void init(const uint32_t *words, int64_t nw, uint32_t bit) {
        w = words;
        wend = nw;
        int64_t p = bit >> 5;
        unsigned long long w0 = p < nw ? w[p] : 0u;
        unsigned long long w1 = p + 1 < nw ? w[p + 1] : 0u;
        int s = bit & 31;
        buf = ((w0 << 32) | w1) << s;
        nbits = 64 - s;
        wp = p + 2;
        consumed = bit;
    }
    __device__ __forceinline__ void refill() {
        if (nbits < 32) {
            unsigned long long nx = wp < wend ? w[wp] : 0u;
            buf |= nx << (32 - nbits);
            nbits += 32;
            ++wp;
        }
    }
    // returns symbol value; sets bad on an invalid code
    __device__ __forceinline__ int32_t next(const Canon &c, uint32_t &bad) {
        refill();
        uint32_t win = (uint32_t)(buf >> 32);
        int L = c.minlen;
        while (L < c.maxlen && (unsigned long long)win >= c.lim[L]) ++L;
        int32_t v;
        if ((unsigned long long)win >= c.lim[L]) {
            bad |= C3_ERR_CODE;
            v = 0;
        } else {
            const uint32_t code = win >> (32 - L);
            v = c.sym[(int32_t)code + c.delta[L]];
        }
        buf <<= L;
        nbits -= L;
        consumed += L;
        return v;
    }
};

template <typename T, bool RESID>
__global__ __launch_bounds__(C3_NT) void k_decode(LayoutDev Ld, HuffDev hp, HuffDev hs,
                                                  const DecodeTask *__restrict__ tasks,
                                                  int32_t *__restrict__ pix_out,
                                                  uint16_t *__restrict__ psi_out, const void *d,
                                                  int d_f64, const T *__restrict__ maps,
                                                  const double *__restrict__ gain,
                                                  const cx<T> *__restrict__ trig_g,
                                                  T *__restrict__ r_out, uint32_t *err) {
    __shared__ Canon cp, cq;
    __shared__ int32_t tp[C3_NT * GP];
    __shared__ int32_t tq[C3_NT * GP];
    __shared__ cx<T> trig[RESID ? 4096 : 1];
    __shared__ uint32_t blk_err;

    const DecodeTask task = tasks[blockIdx.x];
    const int seg = task.seg;
    const int tid = threadIdx.x;
    const int64_t s0 = Ld.seg_off[seg];
    const int n = (int)(Ld.seg_off[seg + 1] - s0);
    const int C = hp.chunk_len;
    const int band = Ld.seg_band[seg];
    const int64_t npix = Ld.band[band].npix;
    const int npsi = Ld.band[band].npsi;

    if (tid == 0) {
        build_canon(cp, hp.tables + hp.table_off[hp.seg_table[seg]]);
        blk_err = 0;
    }
    if (tid == 1) build_canon(cq, hs.tables + hs.table_off[hs.seg_table[seg]]);
    if (RESID) {
        for (int b = tid; b < 4096; b += C3_NT) trig[b] = trig_g[b];
    }
    __syncthreads();

    const int l = tid;
    const int c = task.chunk0 + l;
    // the side index must hold ceil(n / C) chunks for this segment
    const int nch_idx = (int)min(hp.seg_chunk_off[seg + 1] - hp.seg_chunk_off[seg],
                                 hs.seg_chunk_off[seg + 1] - hs.seg_chunk_off[seg]);
    const bool active = l < task.nchunk && c < nch_idx;
    if (l < task.nchunk && c >= nch_idx) atomicOr(&blk_err, C3_ERR_CHUNK);
    BitReader rp, rq;
    int32_t xp = 0, xq = 0;
    int ns = 0;
    uint32_t bad = 0;
    if (active) {
        const int64_t gp = hp.seg_chunk_off[seg] + c;
        const int64_t gq = hs.seg_chunk_off[seg] + c;
        const int64_t wp0 = hp.seg_word_off[seg], wq0 = hs.seg_word_off[seg];
        rp.init(hp.words + wp0, hp.seg_word_off[seg + 1] - wp0, hp.chunk_bit[gp]);
        rq.init(hs.words + wq0, hs.seg_word_off[seg + 1] - wq0, hs.chunk_bit[gq]);
        xp = hp.chunk_prev[gp];
        xq = hs.chunk_prev[gq];
        ns = min(C, n - c * C);
    }
    const int nround = (C + G - 1) / G;
    const double g = gain ? gain[seg] : 1.0;
    const int64_t poff = Ld.band[band].pix_off;
    const int64_t npt = Ld.npix_total;

    for (int rd = 0; rd < nround; ++rd) {
        const int k0 = rd * G;
        if (active) {
#pragma unroll 4
            for (int k = 0; k < G; ++k) {
                if (k0 + k < ns) {
                    xp += rp.next(cp, bad);
                    xq += rq.next(cq, bad);
                    tp[l * GP + k] = xp;
                    tq[l * GP + k] = xq;
                }
            }
        }
        __syncthreads();
        // tile walk in sample order: row l holds samples (c*C + k0 .. +G) of chunk c
        for (int q = tid; q < task.nchunk * G; q += C3_NT) {
            const int ll = q / G, kk = q - ll * G;
            const int t = (task.chunk0 + ll) * C + k0 + kk;
            if (k0 + kk < C && t < n) {
                int32_t p = tp[ll * GP + kk];
                int32_t b = tq[ll * GP + kk];
                if (p < 0 || (int64_t)p >= npix) {
                    bad |= C3_ERR_PIX;
                    p = 0;
                }
                if (b < 0 || b >= npsi) {
                    bad |= C3_ERR_PSI;
                    b = 0;
                }
                const int64_t i = s0 + t;
                pix_out[i] = p;
                psi_out[i] = (uint16_t)b;
                if (RESID) {
                    const int64_t gpx = poff + p;
                    const cx<T> cs = trig[b];
                    T sv = maps[gpx] + maps[npt + gpx] * cs.x + maps[2 * npt + gpx] * cs.y;
                    T dv = d_f64 ? (T)((const double *)d)[i] : (T)((const float *)d)[i];
                    r_out[i] = dv - (T)g * sv;
                }
            }
        }
        __syncthreads();
    }
    // chunk boundary consistency with the side index
    if (active && c + 1 < (int)(hp.seg_chunk_off[seg + 1] - hp.seg_chunk_off[seg])) {
        const int64_t gp = hp.seg_chunk_off[seg] + c + 1;
        const int64_t gq = hs.seg_chunk_off[seg] + c + 1;
        if (rp.consumed != (int64_t)hp.chunk_bit[gp] || xp != hp.chunk_prev[gp]) bad |= C3_ERR_CHUNK;
        if (rq.consumed != (int64_t)hs.chunk_bit[gq] || xq != hs.chunk_prev[gq]) bad |= C3_ERR_CHUNK;
    }
    if (active && ns > 0) {
        const int64_t wp0 = hp.seg_word_off[seg], wq0 = hs.seg_word_off[seg];
        if (rp.consumed > 32 * (hp.seg_word_off[seg + 1] - wp0)) bad |= C3_ERR_CHUNK;
        if (rq.consumed > 32 * (hs.seg_word_off[seg + 1] - wq0)) bad |= C3_ERR_CHUNK;
    }
    if (bad) atomicOr(&blk_err, bad);
    __syncthreads();
    if (tid == 0 && blk_err) atomicOr(err, blk_err);
}

}  // namespace

namespace c3 {

hipError_t launch_decode(hipStream_t st, const LayoutDev &L, const HuffDev &hp, const HuffDev &hs,
                         const DecodeTask *tasks, int ntask, int32_t *pix_out, uint16_t *psi_out,
                         int mode, int prec_mixed, const void *d, int d_f64, const void *maps,
                         const double *gain, const void *trig, void *r_out, uint32_t *err) {
    if (ntask <= 0) return hipSuccess;
    dim3 grid(ntask), block(C3_NT);
    if (mode == DEC_POINTING) {
        hipLaunchKernelGGL((k_decode<float, false>), grid, block, 0, st, L, hp, hs, tasks, pix_out,
                           psi_out, nullptr, 0, nullptr, nullptr, nullptr, nullptr, err);
    } else if (prec_mixed) {
        hipLaunchKernelGGL((k_decode<float, true>), grid, block, 0, st, L, hp, hs, tasks, pix_out,
                           psi_out, d, d_f64, (const float *)maps, gain, (const cx<float> *)trig,
                           (float *)r_out, err);
    } else {
        hipLaunchKernelGGL((k_decode<double, true>), grid, block, 0, st, L, hp, hs, tasks, pix_out,
                           psi_out, d, d_f64, (const double *)maps, gain, (const cx<double> *)trig,
                           (double *)r_out, err);
    }
    return hipGetLastError();
}

}  // namespace c3
