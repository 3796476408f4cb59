// FFT row pass (pass 2 of the n_corr transform, section 4.2) compiled per row
// length L: FP32, the rows k1 and M1 - k1 of one segment (0 < k1 < M1/2, the
// rows holding each other's mirror modes) in one block of 512 threads.
//
// Everything the generic row kernel (fft.hip) decides at run time is fixed
// here at compile time: the three stage radices (rowc.h), each thread's
// butterflies, the LDS strides and the index arithmetic; the stage
// twiddles are loaded whole from a per-length table (one base address per
// butterfly) instead of being built by chained products, and the mode loop
// takes w_N^k = w_N^k1 w_2L^k2 from a block constant and a table of L values.
// The first forward stage reads the two rows from memory and the last inverse
// stage writes them back.  Modes: 0 (n_corr constrained realisation), 1 (the
// chi^2's Whittle sums) and 4 (the periodogram of the noise-parameter draw):
// forward stages only, nothing written back; 2 (Fourier-diagonal filters).
// Mode 3 runs on the generic kernel.  The
// rows k1 = 0 and k1 = M1/2, each holding its own mirror modes, come two to a
// task (of one segment or two).
#include "fftmode.h"
#include "rowc.h"

namespace {
using c3::FftArgs;
using namespace c3fft;
using namespace c3rowc;

constexpr int NT = C3_ROW_NT_F32;

extern __shared__ __attribute__((aligned(16))) unsigned char c3_rowc_lds[];

// one Stockham stage of the two interleaved rows (row b's element i at LDS
// index 2 i + b).  IO 1: inputs from the rows in memory (first forward
// stage); IO 2: outputs to the rows in memory (last inverse stage).
template <int L, int S, int DIR, int IO>
__device__ __forceinline__ void rstage(cx<float> *buf, const cx<float> *g0, const cx<float> *g1, cx<float> *o0,
                                       cx<float> *o1, const cx<float> *__restrict__ tw) {
    constexpr Plan3 P = plan(L);
    constexpr int R = P.r[S];
    constexpr int NS = row_ns(L, S);
    constexpr int LR = L / R;
    constexpr int NB = 2 * LR;  // butterflies of both rows
    constexpr int KB = (NB + NT - 1) / NT;
    constexpr long TOFF = S > 0 ? stage_off(L, S) : 0;
    cx<float> v[KB][R];
    int ob[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int q = (int)threadIdx.x + kb * NT;
        ob[kb] = -1;
        if (NB % NT == 0 || q < NB) {
            const int b = q & 1, j = q >> 1;
            if constexpr (IO == 1) {
                const cx<float> *g = b ? g1 : g0;
#pragma unroll
                for (int t = 0; t < R; ++t) v[kb][t] = g[j + t * LR];
            } else {
#pragma unroll
                for (int t = 0; t < R; ++t) v[kb][t] = buf[2 * (j + t * LR) + b];
            }
            const int jd = j / NS, k = j - jd * NS;
            if constexpr (S > 0) {
                const cx<float> *w = tw + TOFF + k * (R - 1);
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    const cx<float> wt = w[t - 1];
                    v[kb][t] = DIR < 0 ? cmul(v[kb][t], wt) : cmulc(v[kb][t], wt);
                }
            }
            dft_any<R, DIR>(v[kb]);
            if constexpr (IO == 2) {
                cx<float> *o = b ? o1 : o0;  // last stage: jd = 0
#pragma unroll
                for (int t = 0; t < R; ++t) o[k + t * NS] = v[kb][t];
            } else {
                ob[kb] = 2 * (jd * NS * R + k) + b;
            }
        }
    }
    if constexpr (IO == 2) return;
    if constexpr (IO == 0) __syncthreads();  // in place: every read before any write
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
        if (ob[kb] >= 0) {
#pragma unroll
            for (int t = 0; t < R; ++t) buf[ob[kb] + 2 * t * NS] = v[kb][t];
        }
    __syncthreads();
}

// nhat_k of the n_corr draw (the same value as cr_mode) with the draw's
// constants folded: s0 W1 = sqrt(c log2 u0) (cos 2 pi u1, sin 2 pi u1) with
// c = -sigma0^2 ln 2 (Box-Muller radius sqrt(-2 ln u0) times 1/sqrt 2 and
// sigma0), and s0 sqrt(q) W2 = sqrt(c q log2 u2) (cos 2 pi u3, sin 2 pi u3).
// k > 0 and k < M here, so both draws are complex.
struct FastCtx {
    float c;        // -sigma0^2 ln 2
    float isq;      // 1 / sqrt(N), times the 1/2 of the real-spectrum split
    float oscale;   // the output scale sqrt(N)/M, times the 1/2 of the re-pack
    float malpha, lbase2;
};

__device__ __forceinline__ cx<float> cr_fast(const ModeCtx &mc, const FastCtx &fc, uint32_t k, cx<float> E) {
    const float x = fc.malpha * (__builtin_amdgcn_logf((float)k) + fc.lbase2);
    const float q = __builtin_amdgcn_exp2f(x);  // (f_k / f_knee)^-alpha = sigma0^2 / P_k
    const float inv = __builtin_amdgcn_rcpf(1.0f + q) * fc.oscale;
    cx<float> out = {E.x * fc.isq, E.y * fc.isq};
    if (!mc.mean_only) {
        const uint4 w = philox4x32_10(make_uint4(k, mc.it_lo, mc.it_hi, mc.seed_hi), mc.key);
        const float sc = 2.3283064365386963e-10f, off = 1.1641532182693481e-10f;  // (x + 1/2) 2^-32
        const float u0 = fmaf((float)w.x, sc, off), u1 = fmaf((float)w.y, sc, off);
        const float u2 = fmaf((float)w.z, sc, off), u3 = fmaf((float)w.w, sc, off);
        const float a0 = __builtin_amdgcn_sqrtf(fc.c * __builtin_amdgcn_logf(u0));
        const float a1 = __builtin_amdgcn_sqrtf(fc.c * q * __builtin_amdgcn_logf(u2));
        out.x = fmaf(a0, __builtin_amdgcn_cosf(u1), fmaf(a1, __builtin_amdgcn_cosf(u3), out.x));
        out.y = fmaf(a0, __builtin_amdgcn_sinf(u1), fmaf(a1, __builtin_amdgcn_sinf(u3), out.y));
    }
    return {out.x * inv, out.y * inv};
}

__device__ __forceinline__ FastCtx fast_ctx(const ModeCtx &mc) {
    FastCtx fc;
    fc.c = (float)(-mc.sigma0 * mc.sigma0 * 0.69314718055994530942);
    fc.isq = (float)(0.5 * mc.invsqrtN);
    fc.oscale = (float)(0.5 * mc.outscale);
    fc.malpha = (float)mc.malpha;
    fc.lbase2 = (float)mc.lbase2;
    return fc;
}

// The real-spectrum split of a mirror pair: from Z_k (za) and Z_{M-k} (zb) of
// the packed transform and w = w_N^k, twice E_k and twice E_{M-k}:
// 2A = Zk + conj Zp, 2B = -i (Zk - conj Zp), 2 E_k = 2A + w_N^k 2B, and the
// partner from conj A, conj B and w_N^(M-k) = -conj(w_N^k).
__device__ __forceinline__ void split_pair(cx<float> za, cx<float> zb, cx<float> w, cx<float> &ek,
                                           cx<float> &ep) {
    const cx<float> A = {za.x + zb.x, za.y - zb.y};
    const cx<float> D = {za.x - zb.x, za.y + zb.y};
    const cx<float> B = {D.y, -D.x};
    ek = cadd(A, cmul(w, B));
    const cx<float> wp = {-w.x, w.y};
    ep = cadd(cconj(A), cmul(wp, cconj(B)));
}

// The re-pack of a mirror pair: Z'_k = (nk + conj np)/2 + i (nk - conj np)
// conj(w_N^k)/2 and its partner (the factors 1/2 are in the modes' scales).
__device__ __forceinline__ void repack_pair(cx<float> nk, cx<float> np, cx<float> w, cx<float> &zk,
                                            cx<float> &zq) {
    const cx<float> A = {nk.x + np.x, nk.y - np.y};
    const cx<float> D = {nk.x - np.x, nk.y + np.y};
    const cx<float> B = cmulc(D, w);
    zk = cx<float>{A.x - B.y, A.y + B.x};
    const cx<float> Bq = cmul(cconj(D), w);
    zq = cx<float>{A.x - Bq.y, -A.y + Bq.x};
}

// The modes of a row that holds its own mirror modes (modes 0 and 2), in LDS
// row b: k1 = 0 pairs k = M1 k2 with M - k at k2' = (L - k2) mod L and holds
// k = 0 and k = M (both real, from Z_0); k1 = M1/2 pairs k2 with
// L - 1 - k2.  A pair with k2' = k2 is the single mode k = M/2.
template <int L, int MODE>
__device__ __forceinline__ void self_row_modes(const FftArgs &a, cx<float> *buf, int seg, int k1, int b,
                                               const cx<float> *twh) {
    const SegInfo sg = a.segs[seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M = p.M;
    const ModeCtx mc = mode_ctx<MODE>(a, seg, sg.band, M);
    const FastCtx fc = fast_ctx(mc);
    const float osc2 = (float)(0.5 * mc.outscale), osc4 = (float)(0.25 * mc.outscale);
    const cx<float> wa = twN((const cx<float> *)a.twpool, p, k1);
    const bool zero = k1 == 0;
    const int npair = zero ? L / 2 + 1 : (L + 1) / 2;
    for (int k2 = threadIdx.x; k2 < npair; k2 += NT) {
        const int e = 2 * k2 + b;
        if (zero && k2 == 0) {
            // E_0 = Re Z_0 + Im Z_0 and E_M = Re Z_0 - Im Z_0, real modes
            const cx<float> z = buf[e];
            const cx<float> E0 = {z.x + z.y, 0.f}, EM = {z.x - z.y, 0.f};
            cx<float> n0, nM;
            if constexpr (MODE == 0) {
                n0 = cr_mode<float>(mc, 0, E0);
                nM = cr_mode<float>(mc, M, EM);
            } else {
                n0 = a.which == 3 ? x0_mode(mc, 0, E0) : filt_mode(mc, 0, E0, a.which);
                nM = a.which == 3 ? x0_mode(mc, M, EM) : filt_mode(mc, M, EM, a.which);
            }
            const float h = 0.5f * (float)mc.outscale;
            buf[e] = cx<float>{h * (n0.x + nM.x), h * (n0.x - nM.x)};
            continue;
        }
        const int pk2 = zero ? L - k2 : L - 1 - k2;
        const int ep = 2 * pk2 + b;
        const cx<float> w = cmul(wa, twh[k2]);
        const int64_t k = k1 + (int64_t)M1 * k2, kp = (int64_t)M - k;
        cx<float> Ek, Ep;
        split_pair(buf[e], buf[ep], w, Ek, Ep);
        cx<float> nk, np;
        if constexpr (MODE == 0) {
            nk = cr_fast(mc, fc, (uint32_t)k, Ek);
            np = pk2 == k2 ? nk : cr_fast(mc, fc, (uint32_t)kp, Ep);
        } else if (a.which == 3) {  // not linear in E (its drawn term): E itself
            nk = cscale(x0_mode(mc, k, cscale(Ek, 0.5f)), osc2);
            np = pk2 == k2 ? nk : cscale(x0_mode(mc, kp, cscale(Ep, 0.5f)), osc2);
        } else {
            nk = cscale(filt_mode(mc, k, Ek, a.which), osc4);
            np = pk2 == k2 ? nk : cscale(filt_mode(mc, kp, Ep, a.which), osc4);
        }
        cx<float> zk, zq;
        repack_pair(nk, np, w, zk, zq);
        buf[e] = zk;
        if (pk2 != k2) buf[ep] = zq;
    }
}

// The modes of rows k1 and M1 - k1 (LDS rows 0 and 1), which hold each
// other's mirror modes: mode k = k1 + M1 k2 of row 0 pairs with M - k at
// k2' = L - 1 - k2 of row 1.
template <int L, int MODE>
__device__ __forceinline__ void pair_row_modes(const FftArgs &a, cx<float> *buf, int seg, const SegInfo &sg,
                                               const FftPlan &p, int ka, const cx<float> *twh) {
    const int M1 = p.M1, M = p.M;
    const cx<float> *pool = (const cx<float> *)a.twpool;
    const ModeCtx mc = mode_ctx<MODE>(a, seg, sg.band, M);
    const FastCtx fc = fast_ctx(mc);
    const cx<float> wa = twN(pool, p, ka);  // w_N^k1; w_N^(k1 + M1 k2) = w_N^k1 w_2L^k2
    const float osc2 = (float)(0.5 * mc.outscale), osc4 = (float)(0.25 * mc.outscale);
    // The two factors 1/2 of the split and of the re-pack and the output
    // scale are applied once per mode: E below is twice the spectrum value
    // (halved in fc.isq or the mode scales) and nk, np come out already
    // times sqrt(N)/(2M).
    for (int k2 = threadIdx.x; k2 < L; k2 += NT) {
        const int pk2 = L - 1 - k2;  // the partner mode M - k sits in row 1
        const cx<float> Za = buf[2 * k2], Zb = buf[2 * pk2 + 1];
        const cx<float> w = cmul(wa, twh[k2]);
        const int64_t k = ka + (int64_t)M1 * k2, kp = (int64_t)M - k;
        cx<float> Ek, Ep;
        split_pair(Za, Zb, w, Ek, Ep);
        cx<float> nk, np;
        if constexpr (MODE == 0) {
            nk = cr_fast(mc, fc, (uint32_t)k, Ek);
            np = cr_fast(mc, fc, (uint32_t)kp, Ep);
        } else {
            if (a.which == 3) {  // not linear in E (its drawn term): E itself
                nk = cscale(x0_mode(mc, k, cscale(Ek, 0.5f)), osc2);
                np = cscale(x0_mode(mc, kp, cscale(Ep, 0.5f)), osc2);
            } else {
                nk = cscale(filt_mode(mc, k, Ek, a.which), osc4);
                np = cscale(filt_mode(mc, kp, Ep, a.which), osc4);
            }
        }
        cx<float> zk, zq;
        repack_pair(nk, np, w, zk, zq);
        buf[2 * k2] = zk;
        buf[2 * pk2 + 1] = zq;
    }
}

// Whittle sums (the chi^2's noise term, mode 1) of rows k1 and M1 - k1: every
// mode k and its partner M - k, E_k from the split (halved: the split gives
// twice E)
template <int L>
__device__ __forceinline__ Wsum pair_row_whittle(const FftArgs &a, const cx<float> *buf, int seg,
                                                 const SegInfo &sg, const FftPlan &p, int ka,
                                                 const cx<float> *twh) {
    const ModeCtx mc = mode_ctx<1>(a, seg, sg.band, p.M);
    const cx<float> wa = twN((const cx<float> *)a.twpool, p, ka);
    Wsum ws = {0, 0, 0};
    for (int k2 = threadIdx.x; k2 < L; k2 += NT) {
        const int pk2 = L - 1 - k2;
        const cx<float> w = cmul(wa, twh[k2]);
        const int64_t k = ka + (int64_t)p.M1 * k2;
        cx<float> Ek, Ep;
        split_pair(buf[2 * k2], buf[2 * pk2 + 1], w, Ek, Ep);
        whittle_mode(mc, k, cscale(Ek, 0.5f), ws);
        whittle_mode(mc, (int64_t)p.M - k, cscale(Ep, 0.5f), ws);
    }
    return ws;
}

// the same for a row that holds its own mirror modes (pairs as in
// self_row_modes; row 0 adds the real mode k = M, E_M = Re Z_0 - Im Z_0, and
// leaves out the mean)
template <int L>
__device__ __forceinline__ Wsum self_row_whittle(const FftArgs &a, const cx<float> *buf, int seg, int k1, int b,
                                                 const cx<float> *twh) {
    const SegInfo sg = a.segs[seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M = p.M;
    const ModeCtx mc = mode_ctx<1>(a, seg, sg.band, M);
    const cx<float> wa = twN((const cx<float> *)a.twpool, p, k1);
    const bool zero = k1 == 0;
    const int npair = zero ? L / 2 + 1 : (L + 1) / 2;
    Wsum ws = {0, 0, 0};
    for (int k2 = threadIdx.x; k2 < npair; k2 += NT) {
        if (zero && k2 == 0) {
            const cx<float> z = buf[b];
            whittle_mode(mc, (int64_t)M, cx<float>{z.x - z.y, 0.f}, ws);
            continue;
        }
        const int pk2 = zero ? L - k2 : L - 1 - k2;
        const cx<float> w = cmul(wa, twh[k2]);
        const int64_t k = k1 + (int64_t)M1 * k2;
        cx<float> Ek, Ep;
        split_pair(buf[2 * k2 + b], buf[2 * pk2 + b], w, Ek, Ep);
        whittle_mode(mc, k, cscale(Ek, 0.5f), ws);
        if (pk2 != k2) whittle_mode(mc, (int64_t)M - k, cscale(Ep, 0.5f), ws);
    }
    return ws;
}

// Periodogram of a row pair's modes into the block's LDS bins (mode 4, the
// noise-parameter draw): |E_k|^2 / N for every mode k and its partner M - k
// of rows k1 and M1 - k1 (E from the split, halved).  Every lane of a wave
// walks the same number of steps (hist_add is a wave operation).
template <int L>
__device__ __forceinline__ void pair_row_periodogram(const FftArgs &a, const cx<float> *buf, int seg,
                                                     const SegInfo &sg, const FftPlan &p, int ka,
                                                     const cx<float> *twh, double *hist) {
    const ModeCtx mc = mode_ctx<4>(a, seg, sg.band, p.M);
    const double s2 = 0.25 * mc.invsqrtN * mc.invsqrtN;  // the split gives twice E
    const cx<float> wa = twN((const cx<float> *)a.twpool, p, ka);
    for (int base = 0; base < L; base += NT) {
        const int k2 = base + (int)threadIdx.x;
        int bk = -1, bp = -1;
        double vk = 0.0, vp = 0.0;
        if (k2 < L) {
            const int pk2 = L - 1 - k2;
            const cx<float> w = cmul(wa, twh[k2]);
            const int64_t k = ka + (int64_t)p.M1 * k2;
            cx<float> Ek, Ep;
            split_pair(buf[2 * k2], buf[2 * pk2 + 1], w, Ek, Ep);
            vk = ((double)Ek.x * Ek.x + (double)Ek.y * Ek.y) * s2;
            vp = ((double)Ep.x * Ep.x + (double)Ep.y * Ep.y) * s2;
            bk = xi_bin(k);
            bp = xi_bin((int64_t)p.M - k);
        }
        hist_add(hist, bk, vk);
        hist_add(hist, bp, vp);
    }
}

// the same for a row that holds its own mirror modes (pairs as in
// self_row_modes; row 0 adds the real mode k = M and leaves out the mean)
template <int L>
__device__ __forceinline__ void self_row_periodogram(const FftArgs &a, const cx<float> *buf, int seg, int k1,
                                                     int b, const cx<float> *twh, double *hist) {
    const SegInfo sg = a.segs[seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M = p.M;
    const ModeCtx mc = mode_ctx<4>(a, seg, sg.band, M);
    const double s1 = mc.invsqrtN * mc.invsqrtN, s2 = 0.25 * s1;
    const cx<float> wa = twN((const cx<float> *)a.twpool, p, k1);
    const bool zero = k1 == 0;
    const int npair = zero ? L / 2 + 1 : (L + 1) / 2;
    for (int base = 0; base < npair; base += NT) {
        const int k2 = base + (int)threadIdx.x;
        int bk = -1, bp = -1;
        double vk = 0.0, vp = 0.0;
        if (k2 < npair) {
            if (zero && k2 == 0) {
                const cx<float> z = buf[b];
                const double em = (double)(z.x - z.y);  // E_M, real
                vk = em * em * s1;
                bk = xi_bin(M);
            } else {
                const int pk2 = zero ? L - k2 : L - 1 - k2;
                const cx<float> w = cmul(wa, twh[k2]);
                const int64_t k = k1 + (int64_t)M1 * k2;
                cx<float> Ek, Ep;
                split_pair(buf[2 * k2 + b], buf[2 * pk2 + b], w, Ek, Ep);
                vk = ((double)Ek.x * Ek.x + (double)Ek.y * Ek.y) * s2;
                bk = xi_bin(k);
                if (pk2 != k2) {
                    vp = ((double)Ep.x * Ep.x + (double)Ep.y * Ep.y) * s2;
                    bp = xi_bin((int64_t)M - k);
                }
            }
        }
        hist_add(hist, bk, vk);
        hist_add(hist, bp, vp);
    }
}

// the block's bins added to the segment's (FP64 atomics), then cleared
__device__ __forceinline__ void hist_flush(const FftArgs &a, double *hist, int seg) {
    __syncthreads();
    for (int i = threadIdx.x; i < C3_XI_NBIN; i += NT)
        if (hist[i] != 0.0) {
            atomicAdd(&a.bins[(int64_t)seg * C3_XI_NBIN + i], hist[i]);
            hist[i] = 0.0;
        }
    __syncthreads();
}

// block sum of a thread's Whittle sums, added to the segment's; red: 3 NT/64
// doubles of LDS that no thread reads or writes otherwise
__device__ __forceinline__ void whittle_flush(const FftArgs &a, double *red, Wsum ws, int seg) {
    double v[3] = {ws.a, ws.b, ws.c};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double x = v[j];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if ((threadIdx.x & 63) == 0) red[j * (NT / 64) + (threadIdx.x >> 6)] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double x = 0;
        for (int w = 0; w < NT / 64; ++w) x += red[threadIdx.x * (NT / 64) + w];
        atomicAdd(&a.whittle[(int64_t)seg * 4 + threadIdx.x], x);
    }
    __syncthreads();
}

template <int L, int MODE>
__global__ __launch_bounds__(NT) void k_rowc(FftArgs a) {
    static_assert(plan(L).r[0] > 0, "row length without a three-stage plan");
    cx<float> *buf = (cx<float> *)c3_rowc_lds;  // 2 L elements
    const RowTask task = a.row_tasks[blockIdx.x];
    if (task.seg < 0) return;                      // an empty task (launch padding)
    // a task of two rows that each hold their own mirror modes (k1 = 0 or
    // M1/2): pad[0] = 1 + the second row's segment, pad[1] = its k1
    const bool self = task.pad[0] > 0;
    // converged segments (masked draw): no load.  A task of two segments runs
    // while either is active; the workspace rows of a converged one are not
    // read again (its column passes return before any load or store).
    if (a.active && !a.active[task.seg] && !(self && a.active[task.pad[0] - 1])) return;
    // the rows' loads need only the task: they are issued first, and the
    // segment's record and plan load while they are in flight
    cx<float> *ya = (cx<float> *)a.work + task.off_a, *yb = (cx<float> *)a.work + task.off_b;
    rstage<L, 0, -1, 1>(buf, ya, yb, nullptr, nullptr, nullptr);
    const int seg = task.seg;
    const SegInfo sg = a.segs[seg];
    const FftPlan &p = a.plans[sg.plan];
    const int ka = task.k1;  // 0 < ka < M1 / 2 (rows ka and M1 - ka), or a row of a self task
    const cx<float> *pool = (const cx<float> *)a.twpool;
    const cx<float> *tws = pool + p.twr;
    const cx<float> *twh = pool + p.twh;

    rstage<L, 1, -1, 0>(buf, nullptr, nullptr, nullptr, nullptr, tws);
    rstage<L, 2, -1, 0>(buf, nullptr, nullptr, nullptr, nullptr, tws);

    if constexpr (MODE == 4) {
        __shared__ double hist[C3_XI_NBIN];
        for (int i = threadIdx.x; i < C3_XI_NBIN; i += NT) hist[i] = 0.0;
        __syncthreads();
        if (self) {
            const int seg1 = task.pad[0] - 1;
            self_row_periodogram<L>(a, buf, seg, ka, 0, twh, hist);
            hist_flush(a, hist, seg);
            self_row_periodogram<L>(a, buf, seg1, task.pad[1], 1, twh, hist);
            hist_flush(a, hist, seg1);
        } else {
            pair_row_periodogram<L>(a, buf, seg, sg, p, ka, twh, hist);
            hist_flush(a, hist, seg);
        }
    } else if constexpr (MODE == 1) {
        // the rows' buffer is not written back: after the sums, it holds the
        // block's partial sums
        double *red = (double *)buf;
        if (self) {
            const int seg1 = task.pad[0] - 1;
            const Wsum w0 = self_row_whittle<L>(a, buf, seg, ka, 0, twh);
            const Wsum w1 = self_row_whittle<L>(a, buf, seg1, task.pad[1], 1, twh);
            __syncthreads();
            whittle_flush(a, red, w0, seg);
            whittle_flush(a, red, w1, seg1);
        } else {
            const Wsum w = pair_row_whittle<L>(a, buf, seg, sg, p, ka, twh);
            __syncthreads();
            whittle_flush(a, red, w, seg);
        }
    } else {
        if (self) {
            // the stage and w_2L tables depend on L alone: the first row's serve both
            self_row_modes<L, MODE>(a, buf, seg, ka, 0, twh);
            self_row_modes<L, MODE>(a, buf, task.pad[0] - 1, task.pad[1], 1, twh);
        } else {
            pair_row_modes<L, MODE>(a, buf, seg, sg, p, ka, twh);
        }
        __syncthreads();

        rstage<L, 0, 1, 0>(buf, nullptr, nullptr, nullptr, nullptr, tws);
        rstage<L, 1, 1, 0>(buf, nullptr, nullptr, nullptr, nullptr, tws);
        rstage<L, 2, 1, 2>(buf, nullptr, nullptr, ya, yb, tws);
    }
}

}  // namespace

namespace c3 {

bool rowc_supported(int mixed, int L, int mode) {
    return mixed && (mode == 0 || mode == 1 || mode == 2 || mode == 4) && c3rowc::compiled(L);
}

hipError_t rowc_init_attributes() {
    hipError_t e = hipSuccess;
    auto set = [&](const void *f) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, C3_LDS_MAX - 4096);
        if (r != hipSuccess) e = r;
    };
#define C3_ROWC_ATTR(LL)                       \
    set((const void *)k_rowc<LL, 0>);          \
    set((const void *)k_rowc<LL, 1>);          \
    set((const void *)k_rowc<LL, 2>);          \
    set((const void *)k_rowc<LL, 4>);
    C3_ROWC_LIST(C3_ROWC_ATTR)
#undef C3_ROWC_ATTR
    return e;
}

hipError_t launch_rowc(hipStream_t st, const FftArgs &a, int L) {
    if (a.nrow_tasks <= 0) return hipSuccess;
    const dim3 g(a.nrow_tasks), b(NT);
    const unsigned lds = 2u * (unsigned)L * (unsigned)sizeof(cx<float>);
    switch (L) {
#define C3_ROWC_LAUNCH(LL)                                                    \
    case LL:                                                                  \
        if (a.mode == 0)                                                      \
            hipLaunchKernelGGL((k_rowc<LL, 0>), g, b, lds, st, a);            \
        else if (a.mode == 1)                                                 \
            hipLaunchKernelGGL((k_rowc<LL, 1>), g, b, lds, st, a);            \
        else if (a.mode == 2)                                                 \
            hipLaunchKernelGGL((k_rowc<LL, 2>), g, b, lds, st, a);            \
        else if (a.mode == 4)                                                 \
            hipLaunchKernelGGL((k_rowc<LL, 4>), g, b, lds, st, a);            \
        else                                                                  \
            return hipErrorInvalidValue;                                      \
        break;
        C3_ROWC_LIST(C3_ROWC_LAUNCH)
#undef C3_ROWC_LAUNCH
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace c3
