// Batched mixed-radix real FFTs for the correlated-noise draw (section 4.2) and
// the Fourier-domain chi^2 terms, as a three-pass four-step transform.
//
// A segment of n samples is mirrored and padded to N = 2M real points (M
// 5-smooth), packed as M complex points z_j = e_2j + i e_2j+1, and transformed
// with M = M1 x M2:
//   pass 1 (columns): for each column j2, FFT_M1 over z[M2 j1 + j2], times
//           w_M^(j2 k1); written row-major Y[k1][j2].
//   pass 2 (rows):    block k1 takes rows k1 and M1-k1 (the rows holding the
//           mirror modes M-k of its modes k), FFT_M2 each, splits the complex
//           spectrum into the real-FFT spectrum E_k (k = 0..M), applies the
//           constrained-realisation filter and draw per mode, re-packs, runs
//           the inverse FFT_M2 and writes back.
//   pass 3 (columns): times w_M^(-j2 k1), inverse FFT_M1 per column; the
//           first n real samples are the output.
// This file holds the row pass and the LDS form of the column passes (tiles
// of B columns, any M1); fftcol.hip holds the register form for fixed M1.
// Every sub-transform is an in-LDS Stockham FFT with radix 2/3/4/5 stages.
#include "common.h"
#include "fftdev.h"
#include "fftmode.h"
#include "rng.h"

namespace {
using c3::FftArgs;
using namespace c3fft;
using namespace c3rng;

// explicit LDS / global address spaces for the out-of-line stage functions
// (only meaningful in the device compilation pass)
#if defined(__HIP_DEVICE_COMPILE__)
#define LDSP __attribute__((address_space(3)))
#define GLBP __attribute__((address_space(1)))
#else
#define LDSP
#define GLBP
#endif

// One Stockham stage of radix R on B = 1 << lb transforms of length L in LDS;
// element i of transform b lives at [(i << lsi) + b].  Twiddles: w^k and w^2k
// from the table, higher powers by multiplication (R <= 8), or products of
// table entries w^(Q a) w^b (R > 8).  In place: every thread reads its
// butterflies of the stage into registers, the block synchronises, and the
// results are written back over the inputs, so one LDS buffer serves (two
// row blocks fit on a CU).  KB bounds the butterflies per thread.
template <typename T>
constexpr int row_elems() { return sizeof(T) == 4 ? 2 * 5040 : 2 * 2520; }  // longest row pair

// IO = 0: LDS -> LDS in place; 1: the first stage (Ns = 1) reads its inputs
// straight from the two rows in memory (element i of row b at g_b[i]; lanes
// with consecutive j read consecutive elements); 2: the last stage (Ns R = L)
// writes its outputs straight to the rows (output i = k + t Ns, again
// consecutive across lanes).  The global forms skip one LDS round trip each.
// E: the most elements a call holds (fixes KB, the butterflies per thread).
template <int R, int DIR, int NT, int IO, typename T, int E = row_elems<T>()>
__device__ __attribute__((noinline)) void fft_stage_ip(LDSP cx<T> *buf, const GLBP cx<T> *g0,
                                                       const GLBP cx<T> *g1, GLBP cx<T> *o0,
                                                       GLBP cx<T> *o1, int L, int lb, int lsi, int Ns,
                                                       const GLBP cx<T> *__restrict__ tw) {
    constexpr int KB = (E / R + NT - 1) / NT;
    const int LR = L / R;
    const int nb = LR << lb;
    const int bm = (1 << lb) - 1;
    const int step = L / (Ns * R);
    const int in_stride = LR << lsi;
    const int out_stride = Ns << lsi;
    const int NsR = Ns * R;
    const uint32_t magic = 0xFFFFFFFFu / (uint32_t)Ns + 1u;  // j / Ns == umulhi(j, magic)
    cx<T> v[KB][R];
    int ob[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int q = (int)threadIdx.x + kb * NT;
        ob[kb] = -1;
        if (q < nb) {
            const int b = q & bm, j = q >> lb;
            if constexpr (IO == 1) {
                const GLBP cx<T> *g = b ? g1 : g0;
#pragma unroll
                for (int t = 0; t < R; ++t) v[kb][t] = g[j + t * LR];
            } else {
                int ia = (j << lsi) + b;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    v[kb][t] = buf[ia];
                    ia += in_stride;
                }
            }
            const int jd = (Ns == 1) ? j : (int)__umulhi((uint32_t)j, magic);
            const int k = j - jd * Ns;
            if (Ns > 1) {
                const int ks = k * step;  // v_t *= w_L^(t ks)
                if constexpr (R <= 8) {
                    // w^1 and w^2 from the table, higher powers by products
                    const cx<T> w1 = tw[ks];
                    v[kb][1] = DIR < 0 ? cmul(v[kb][1], w1) : cmulc(v[kb][1], w1);
                    if constexpr (R > 2) {
                        const cx<T> w2 = tw[2 * ks];
                        v[kb][2] = DIR < 0 ? cmul(v[kb][2], w2) : cmulc(v[kb][2], w2);
                        cx<T> wa = w1, wb = w2;
#pragma unroll
                        for (int t = 3; t < R; ++t) {
                            const cx<T> w = cmul((t & 1) ? wa : wb, w2);
                            if (t & 1)
                                wa = w;
                            else
                                wb = w;
                            v[kb][t] = DIR < 0 ? cmul(v[kb][t], w) : cmulc(v[kb][t], w);
                        }
                    }
                } else {
                    // w^(Q a + b) = w^(Q a) w^b, both factors from the table
                    constexpr int Q = tw_split(R);
                    cx<T> wq[Q];
                    wq[0] = cx<T>{(T)1, (T)0};
#pragma unroll
                    for (int q = 1; q < Q; ++q) wq[q] = tw[q * ks];
#pragma unroll
                    for (int ai = 0; ai * Q < R; ++ai) {
                        cx<T> wa = cx<T>{(T)1, (T)0};
                        if (ai) wa = tw[ai * Q * ks];
#pragma unroll
                        for (int q = 0; q < Q; ++q) {
                            const int t = ai * Q + q;
                            if (t == 0 || t >= R) continue;
                            const cx<T> w = ai ? (q ? cmul(wa, wq[q]) : wa) : wq[q];
                            v[kb][t] = DIR < 0 ? cmul(v[kb][t], w) : cmulc(v[kb][t], w);
                        }
                    }
                }
            }
            dft_any<R, DIR>(v[kb]);
            if constexpr (IO == 2) {
                GLBP cx<T> *o = b ? o1 : o0;  // jd = 0 in the last stage
#pragma unroll
                for (int t = 0; t < R; ++t) o[k + t * Ns] = v[kb][t];
            } else {
                ob[kb] = ((jd * NsR + k) << lsi) + b;
            }
        }
    }
    if constexpr (IO == 2) return;  // nothing written to LDS
    if constexpr (IO == 0) __syncthreads();  // in place: all reads before any write
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        if (ob[kb] >= 0) {
            int o = ob[kb];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                buf[o] = v[kb][t];
                o += out_stride;
            }
        }
    }
    __syncthreads();
}

// Row FFT over the LDS buffer; with g0 set the first stage loads the rows
// from memory, with o0 set the last stage stores them (both need >= 2 stages)
template <int DIR, int NT, typename T>
__device__ void row_fft(cx<T> *b, const cx<T> *g0, const cx<T> *g1, cx<T> *o0, cx<T> *o1, int L,
                        int lb, int lsi, const int8_t *rad, int nrad, const cx<T> *tw_) {
    const GLBP cx<T> *tw = (const GLBP cx<T> *)tw_;
    LDSP cx<T> *lb_ = (LDSP cx<T> *)b;
    const GLBP cx<T> *G0 = (const GLBP cx<T> *)g0, *G1 = (const GLBP cx<T> *)g1;
    GLBP cx<T> *O0 = (GLBP cx<T> *)o0, *O1 = (GLBP cx<T> *)o1;
    int Ns = 1;
    for (int s = 0; s < nrad; ++s) {
        const int R = rad[s];
        const int io = (s == 0 && g0) ? 1 : (s == nrad - 1 && o0) ? 2 : 0;
#define C3_RADIX_IO(RR, IO)                                                          \
    case RR:                                                                         \
        fft_stage_ip<RR, DIR, NT, IO>(lb_, G0, G1, O0, O1, L, lb, lsi, Ns, tw);      \
        break;
#define C3_RADIX0(RR) C3_RADIX_IO(RR, 0)
#define C3_RADIX1(RR) C3_RADIX_IO(RR, 1)
#define C3_RADIX2(RR) C3_RADIX_IO(RR, 2)
        if constexpr (sizeof(T) == 4) {
            if (io == 0) {
                switch (R) { C3_ROW_RADICES_F32(C3_RADIX0) default: break; }
            } else if (DIR < 0 && io == 1) {
                switch (R) { C3_ROW_RADICES_F32(C3_RADIX1) default: break; }
            } else if (DIR > 0 && io == 2) {
                switch (R) { C3_ROW_RADICES_F32(C3_RADIX2) default: break; }
            }
        } else {
            if (io == 0) {
                switch (R) { C3_ROW_RADICES_F64(C3_RADIX0) default: break; }
            } else if (DIR < 0 && io == 1) {
                switch (R) { C3_ROW_RADICES_F64(C3_RADIX1) default: break; }
            } else if (DIR > 0 && io == 2) {
                switch (R) { C3_ROW_RADICES_F64(C3_RADIX2) default: break; }
            }
        }
#undef C3_RADIX0
#undef C3_RADIX1
#undef C3_RADIX2
#undef C3_RADIX_IO
        Ns *= R;
    }
}

// Column FFT of B interleaved columns of L points in one LDS buffer, in place
// with the row pass's stage form; radices 2, 3, 4, 5 and 8 (the LDS column
// plans' radices), at most col_elems elements per block
template <typename T>
constexpr int col_elems() { return sizeof(T) == 4 ? 4096 : 2048; }

template <int DIR, int NT, typename T>
__device__ void col_fft(cx<T> *b, int L, int lb, const int8_t *rad, int nrad, const cx<T> *tw_) {
    const GLBP cx<T> *tw = (const GLBP cx<T> *)tw_;
    LDSP cx<T> *lb_ = (LDSP cx<T> *)b;
    constexpr int E = col_elems<T>();
    int Ns = 1;
    for (int s = 0; s < nrad; ++s) {
        const int R = rad[s];
        switch (R) {
        case 2: fft_stage_ip<2, DIR, NT, 0, T, E>(lb_, nullptr, nullptr, nullptr, nullptr, L, lb, lb, Ns, tw); break;
        case 3: fft_stage_ip<3, DIR, NT, 0, T, E>(lb_, nullptr, nullptr, nullptr, nullptr, L, lb, lb, Ns, tw); break;
        case 4: fft_stage_ip<4, DIR, NT, 0, T, E>(lb_, nullptr, nullptr, nullptr, nullptr, L, lb, lb, Ns, tw); break;
        case 5: fft_stage_ip<5, DIR, NT, 0, T, E>(lb_, nullptr, nullptr, nullptr, nullptr, L, lb, lb, Ns, tw); break;
        default: fft_stage_ip<8, DIR, NT, 0, T, E>(lb_, nullptr, nullptr, nullptr, nullptr, L, lb, lb, Ns, tw); break;
        }
        Ns *= R;
    }
}

// ------------------------------------------------------------- pass 1
extern __shared__ __attribute__((aligned(16))) unsigned char c3_dyn_lds[];

template <typename T>
__global__ __launch_bounds__(C3_NT) void k_col_fwd(FftArgs a) {
    cx<T> *buf = (cx<T> *)c3_dyn_lds;  // M1 * B elements (sized per launch)
    const ColTask task = a.col_tasks[blockIdx.x];
    if (a.active && !a.active[task.seg]) return;  // converged segment (whole block)
    const SegInfo sg = a.segs[task.seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M2 = p.M2, B = p.B;
    const int lb = __ffs(B) - 1;
    const int col0 = task.c0;
    const cx<T> *pool = (const cx<T> *)a.twpool;
    cx<T> *Y = (cx<T> *)a.work + sg.scr_off;
    const int tot = M1 * B;
    if (!a.full_io && !a.in_b && a.in_a_f64 == (sizeof(T) == 8)) {
        // one input of the transform's own type (the sweep's residual): plain
        // loads with no type branch, several elements' loads in flight
        const T *r = (const T *)a.in_a + sg.samp_off;
        const int64_t n = sg.n, n2 = 2 * (int64_t)sg.n;
#pragma unroll 4
        for (int i = threadIdx.x; i < tot; i += C3_NT) {
            const int j1 = i >> lb, c = i & (B - 1);
            const int j2 = col0 + c;
            cx<T> v = {0, 0};
            if (j2 < M2) {
                const int64_t t = 2 * ((int64_t)M2 * j1 + j2);
                const int64_t u0 = t < n ? t : (t < n2 ? n2 - 1 - t : 0);
                const int64_t u1 = t + 1 < n ? t + 1 : (t + 1 < n2 ? n2 - 2 - t : 0);
                v = cx<T>{r[u0], r[u1]};
            }
            buf[i] = v;
        }
    } else {
        for (int i = threadIdx.x; i < tot; i += C3_NT) {
            const int j1 = i >> lb, c = i & (B - 1);
            const int j2 = col0 + c;
            cx<T> v = {0, 0};
            if (j2 < M2) {
                const int64_t j = (int64_t)M2 * j1 + j2;
                if (a.full_io) {
                    v = ((const cx<T> *)a.in_a)[sg.ext_off + j];
                } else {
                    v.x = ext_at<T>(a, sg.samp_off, sg.n, 2 * j);
                    v.y = ext_at<T>(a, sg.samp_off, sg.n, 2 * j + 1);
                }
            }
            buf[i] = v;
        }
    }
    __syncthreads();
    col_fft<-1, C3_NT>(buf, M1, lb, p.r1, p.nr1, pool + p.tw1);  // in place
    const cx<T> *res = buf;
    for (int i = threadIdx.x; i < tot; i += C3_NT) {
        const int k1 = i >> lb, c = i & (B - 1);
        const int j2 = col0 + c;
        if (j2 < M2) {
            const cx<T> w = twN(pool, p, 2 * (int64_t)j2 * k1);  // w_M^(j2 k1)
            Y[(int64_t)k1 * M2 + j2] = cmul(res[i], w);
        }
    }
}

// ------------------------------------------------------------- pass 3
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_col_inv(FftArgs a) {
    cx<T> *buf = (cx<T> *)c3_dyn_lds;
    const ColTask task = a.col_tasks[blockIdx.x];
    if (a.active && !a.active[task.seg]) return;  // converged segment (whole block)
    const SegInfo sg = a.segs[task.seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M2 = p.M2, B = p.B;
    const int lb = __ffs(B) - 1;
    const int col0 = task.c0;
    const cx<T> *pool = (const cx<T> *)a.twpool;
    const cx<T> *Y = (const cx<T> *)a.work + sg.scr_off;
    const int tot = M1 * B;
    for (int i = threadIdx.x; i < tot; i += C3_NT) {
        const int k1 = i >> lb, c = i & (B - 1);
        const int j2 = col0 + c;
        // times w_M^(-j2 k1) = conj(w_N^(2 j2 k1)), the inverse of pass 1's twiddle
        buf[i] = j2 < M2 ? cmulc(Y[(int64_t)k1 * M2 + j2], twN(pool, p, 2 * (int64_t)j2 * k1))
                         : cx<T>{0, 0};
    }
    __syncthreads();
    col_fft<1, C3_NT>(buf, M1, lb, p.r1, p.nr1, pool + p.tw1);  // in place
    const cx<T> *res = buf;
    T *out = (T *)a.out + sg.samp_off;
    const int n = sg.n;
    for (int i = threadIdx.x; i < tot; i += C3_NT) {
        const int j1 = i >> lb, c = i & (B - 1);
        const int j2 = col0 + c;
        if (j2 < M2) {
            const int64_t t = 2 * ((int64_t)M2 * j1 + j2);
            const cx<T> v = res[i];
            if (a.full_io) {
                ((cx<T> *)a.out)[sg.ext_off + t / 2] = v;
            } else {
                if (t < n) out[t] = v.x;
                if (t + 1 < n) out[t + 1] = v.y;
            }
        }
    }
}

// ------------------------------------------------------------- pass 2
template <typename T>
constexpr int row_nt() { return sizeof(T) == 4 ? C3_ROW_NT_F32 : C3_ROW_NT_F64; }

template <typename T, int MODE>
__global__ __launch_bounds__(row_nt<T>()) void k_row(FftArgs a) {
    constexpr int NT = row_nt<T>();
    cx<T> *buf = (cx<T> *)c3_dyn_lds;  // 2 * M2 elements (sized per launch)
    __shared__ double red[3][NT / 64];
    const RowTask task = a.row_tasks[blockIdx.x];
    if (task.seg < 0) return;                      // an empty task (launch padding)
    if (task.pad[0] > 0) return;  // a pair of rows k1 = 0, M1/2 for the compiled kernel
    if (a.active && !a.active[task.seg]) return;  // converged segment (whole block)
    const int seg = task.seg;
    const SegInfo sg = a.segs[seg];
    const FftPlan &p = a.plans[sg.plan];
    const int M1 = p.M1, M2 = p.M2, M = p.M;
    const int ka = task.k1, kb = (M1 - ka) % M1;
    const int two = (kb != ka) ? 1 : 0;      // second row present
    const int lb = two;                      // rows interleaved: element (k2, row) at 2*k2 + row
    const int si = two ? 2 : 1;
    const cx<T> *pool = (const cx<T> *)a.twpool;
    cx<T> *Y = (cx<T> *)a.work + sg.scr_off;
    double *hist = nullptr;  // mode 4: per-block periodogram bins
    if constexpr (MODE == 4) {
        __shared__ double hist_lds[C3_XI_NBIN];
        hist = hist_lds;
        for (int i = threadIdx.x; i < C3_XI_NBIN; i += NT) hist[i] = 0.0;
        __syncthreads();
    }

    // the first forward stage reads the two rows from memory and the last
    // inverse stage writes them back (rows of two or more stages)
    cx<T> *ya = Y + (int64_t)ka * M2, *yb = Y + (int64_t)kb * M2;
    const bool direct = p.nr2 >= 2;
    if constexpr (MODE != 3) {  // mode 3 synthesises its spectrum: no input
        if (!direct) {
            for (int i = threadIdx.x; i < M2; i += NT) {
                buf[i * si] = ya[i];
                if (two) buf[i * si + 1] = yb[i];
            }
            __syncthreads();
        }
        row_fft<-1, NT>(buf, direct ? ya : nullptr, yb, (cx<T> *)nullptr, (cx<T> *)nullptr, M2, lb, two,
                        p.r2, p.nr2, pool + p.tw2);
    }

    const ModeCtx mc = mode_ctx<MODE>(a, seg, sg.band, M);
    Wsum ws = {0, 0, 0};
    const T half = (T)0.5;
    const T osc = (T)mc.outscale;

    if constexpr (MODE == 4) {
        // periodogram of the spectrum into the block's LDS histogram.  A wave
        // covers 64 consecutive k2, modes M1 apart: above k ~ 2^15 its lanes
        // mostly share one bin, and one wave sum replaces 64 colliding atomics
        const double s2 = mc.invsqrtN * mc.invsqrtN;
        for (int base = 0; base < M2; base += NT) {
            const int k2 = base + (int)threadIdx.x;
            int bk = -1, bp = -1;
            double vk = 0.0, vp = 0.0;
            if (k2 < M2) {
                int pk2, prow;  // partner position
                if (ka == 0) {
                    pk2 = (M2 - k2) % M2;
                    prow = 0;
                } else {
                    pk2 = M2 - 1 - k2;
                    prow = two;
                }
                const int ea = k2 * si, eb = pk2 * si + prow;
                const int64_t k = ka + (int64_t)M1 * k2;
                const cx<T> Za = buf[ea], Zb = buf[eb];
                if (k == 0) {  // E_M = Re Z0 - Im Z0 (real); the DC mode is left out
                    const T em = Za.x - Za.y;
                    vk = (double)em * em * s2;
                    bk = xi_bin(M);
                } else if (two || pk2 >= k2) {  // single row: each pair once
                    const cx<T> w = twN(pool, p, k);
                    const cx<T> Ak = {half * (Za.x + Zb.x), half * (Za.y - Zb.y)};
                    const cx<T> Dk = {half * (Za.x - Zb.x), half * (Za.y + Zb.y)};
                    const cx<T> Bk = {Dk.y, -Dk.x};
                    const cx<T> Ek = cadd(Ak, cmul(w, Bk));
                    const cx<T> wp = {-w.x, w.y};
                    const cx<T> Ep = cadd(cconj(Ak), cmul(wp, cconj(Bk)));
                    vk = ((double)Ek.x * Ek.x + (double)Ek.y * Ek.y) * s2;
                    bk = xi_bin(k);
                    const int64_t kp = (int64_t)M - k;
                    if (kp != k) {
                        vp = ((double)Ep.x * Ep.x + (double)Ep.y * Ep.y) * s2;
                        bp = xi_bin(kp);
                    }
                }
            }
            hist_add(hist, bk, vk);
            hist_add(hist, bp, vp);
        }
    } else {
        // pair (element e of row a, its mirror-mode partner); w_N^k of the next
        // iteration is fetched while this one computes
        cx<T> w_next = twN(pool, p, ka + (int64_t)M1 * min((int)threadIdx.x, M2 - 1));
        for (int k2 = threadIdx.x; k2 < M2; k2 += NT) {
            const cx<T> w = w_next;  // w_N^k
            if (k2 + NT < M2) w_next = twN(pool, p, ka + (int64_t)M1 * (k2 + NT));
            int pk2, prow;  // partner position
            if (ka == 0) {
                pk2 = (M2 - k2) % M2;
                prow = 0;
            } else {
                pk2 = M2 - 1 - k2;
                prow = two;  // row b (or row a when single)
            }
            if (!two && pk2 < k2) continue;  // single row: each pair once
            const int ea = k2 * si, eb = pk2 * si + prow;
            const int64_t k = ka + (int64_t)M1 * k2;
            cx<T> Za = {0, 0}, Zb = {0, 0};
            if constexpr (MODE != 3) {
                Za = buf[ea];
                Zb = buf[eb];
            }
            if (k == 0) {
                // E_0 = Re Z0 + Im Z0, E_M = Re Z0 - Im Z0 (both real)
                const cx<T> E0 = {Za.x + Za.y, 0}, EM = {Za.x - Za.y, 0};
                if constexpr (MODE == 1) {
                    whittle_mode(mc, M, EM, ws);
                } else {
                    cx<T> n0, nM;
                    if constexpr (MODE == 0) {
                        n0 = cr_mode(mc, 0, E0);
                        nM = cr_mode(mc, M, EM);
                    } else if constexpr (MODE == 2) {
                        n0 = a.which == 3 ? x0_mode(mc, 0, E0) : filt_mode(mc, 0, E0, a.which);
                        nM = a.which == 3 ? x0_mode(mc, M, EM) : filt_mode(mc, M, EM, a.which);
                    } else {
                        n0 = draw_mode<T>(mc, 0, a.which);
                        nM = draw_mode<T>(mc, M, a.which);
                    }
                    buf[ea] = cx<T>{half * osc * (n0.x + nM.x), half * osc * (n0.x - nM.x)};
                }
                continue;
            }
            const int64_t kp = (int64_t)M - k;
            // A = (Zk + conj Zp)/2, B = -i (Zk - conj Zp)/2, E_k = A + w_N^k B
            const cx<T> Ak = {half * (Za.x + Zb.x), half * (Za.y - Zb.y)};
            const cx<T> Dk = {half * (Za.x - Zb.x), half * (Za.y + Zb.y)};
            const cx<T> Bk = {Dk.y, -Dk.x};
            const cx<T> Ek = cadd(Ak, cmul(w, Bk));
            // partner: A_p = conj A_k, B_p = conj B_k, w_N^p = -conj(w_N^k)
            const cx<T> wp = {-w.x, w.y};
            const cx<T> Ep = cadd(cconj(Ak), cmul(wp, cconj(Bk)));
            if constexpr (MODE != 1) {
                cx<T> nk, np;
                if constexpr (MODE == 0) {
                    nk = cr_mode(mc, k, Ek);
                    np = (kp == k) ? nk : cr_mode(mc, kp, Ep);
                } else if constexpr (MODE == 2) {
                    if (a.which == 3) {
                        nk = x0_mode(mc, k, Ek);
                        np = (kp == k) ? nk : x0_mode(mc, kp, Ep);
                    } else {
                        nk = filt_mode(mc, k, Ek, a.which);
                        np = (kp == k) ? nk : filt_mode(mc, kp, Ep, a.which);
                    }
                } else {
                    nk = draw_mode<T>(mc, k, a.which);
                    np = (kp == k) ? nk : draw_mode<T>(mc, kp, a.which);
                }
                // Z'_k = (nk + conj np)/2 + i (nk - conj np) conj(w_N^k)/2, scaled
                const cx<T> Ap = {half * (nk.x + np.x), half * (nk.y - np.y)};
                const cx<T> Dp = {half * (nk.x - np.x), half * (nk.y + np.y)};
                const cx<T> Bp = cmulc(Dp, w);
                const cx<T> Zk = {osc * (Ap.x - Bp.y), osc * (Ap.y + Bp.x)};
                // partner: A'_p = conj A'_k, B'_p = -conj(D') conj(w_N^p) = conj(D') w_N^k
                const cx<T> Bq = cmul(cconj(Dp), w);
                const cx<T> Zq = {osc * (Ap.x - Bq.y), osc * (-Ap.y + Bq.x)};
                buf[ea] = Zk;
                if (eb != ea) buf[eb] = Zq;
            } else {
                whittle_mode(mc, k, Ek, ws);
                if (kp != k) whittle_mode(mc, kp, Ep, ws);
            }
        }
    }  // MODE != 4
    if constexpr (MODE == 4) {
        __syncthreads();
        for (int i = threadIdx.x; i < C3_XI_NBIN; i += NT)
            if (hist[i] != 0.0) atomicAdd(&a.bins[(int64_t)seg * C3_XI_NBIN + i], hist[i]);
    } else if constexpr (MODE != 1) {
        __syncthreads();
        row_fft<1, NT>(buf, (const cx<T> *)nullptr, (const cx<T> *)nullptr, direct ? ya : nullptr, yb,
                       M2, lb, two, p.r2, p.nr2, pool + p.tw2);
        if (!direct) {
            for (int i = threadIdx.x; i < M2; i += NT) {
                ya[i] = buf[i * si];
                if (two) yb[i] = buf[i * si + 1];
            }
        }
    } else {
        // block reduction of the Whittle sums
        double v[3] = {ws.a, ws.b, ws.c};
        for (int j = 0; j < 3; ++j) {
            double x = v[j];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = x;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double x = 0;
            for (int w = 0; w < NT / 64; ++w) x += red[threadIdx.x][w];
            atomicAdd(&a.whittle[(int64_t)seg * 4 + threadIdx.x], x);
        }
    }
}

}  // namespace

namespace c3 {

hipError_t fft_init_attributes() {
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    // room for the kernels' static arrays (reduction sums, periodogram bins: under
    // 2 KB); the largest dynamic request (two rows of 5040 FP32 points) is 80 KB
    const int lim = C3_LDS_MAX - 4096;
    hipError_t e = hipSuccess;
    auto set = [&](const void *f) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (r != hipSuccess) e = r;
    };
    set((const void *)k_col_fwd<float>);
    set((const void *)k_col_inv<float>);
    set((const void *)k_col_fwd<double>);
    set((const void *)k_col_inv<double>);
    set((const void *)k_row<float, 0>);
    set((const void *)k_row<float, 1>);
    set((const void *)k_row<double, 0>);
    set((const void *)k_row<double, 1>);
    set((const void *)k_row<float, 2>);
    set((const void *)k_row<float, 3>);
    set((const void *)k_row<double, 2>);
    set((const void *)k_row<double, 3>);
    set((const void *)k_row<float, 4>);
    set((const void *)k_row<double, 4>);
    const hipError_t ec = rowc_init_attributes();
    if (ec != hipSuccess) e = ec;
    done = e;
    return e;
}

hipError_t launch_fft_pass(hipStream_t st, int mixed, const FftArgs &a, int pass, int m1reg) {
    if (pass == 1 && a.nrow_tasks <= 0) return hipSuccess;
    if (pass != 1 && a.ncol_tasks <= 0) return hipSuccess;
    if (pass != 1 && m1reg > 0) return launch_fft_col_reg(st, mixed, a, pass, m1reg);
    const unsigned lc = (unsigned)a.col_lds, lr = (unsigned)a.row_lds;
    if ((pass == 1 ? lr : lc) > 65536u) {
        hipError_t e = fft_init_attributes();
        if (e != hipSuccess) return e;
    }
    const dim3 b(C3_NT), br(mixed ? C3_ROW_NT_F32 : C3_ROW_NT_F64);
    const dim3 gc(a.ncol_tasks), gr(a.nrow_tasks);
    if (mixed) {
        if (pass == 0) hipLaunchKernelGGL(k_col_fwd<float>, gc, b, lc, st, a);
        else if (pass == 2) hipLaunchKernelGGL(k_col_inv<float>, gc, b, lc, st, a);
        else if (a.mode == 0) hipLaunchKernelGGL((k_row<float, 0>), gr, br, lr, st, a);
        else if (a.mode == 1) hipLaunchKernelGGL((k_row<float, 1>), gr, br, lr, st, a);
        else if (a.mode == 2) hipLaunchKernelGGL((k_row<float, 2>), gr, br, lr, st, a);
        else if (a.mode == 3) hipLaunchKernelGGL((k_row<float, 3>), gr, br, lr, st, a);
        else hipLaunchKernelGGL((k_row<float, 4>), gr, br, lr, st, a);
    } else {
        if (pass == 0) hipLaunchKernelGGL(k_col_fwd<double>, gc, b, lc, st, a);
        else if (pass == 2) hipLaunchKernelGGL(k_col_inv<double>, gc, b, lc, st, a);
        else if (a.mode == 0) hipLaunchKernelGGL((k_row<double, 0>), gr, br, lr, st, a);
        else if (a.mode == 1) hipLaunchKernelGGL((k_row<double, 1>), gr, br, lr, st, a);
        else if (a.mode == 2) hipLaunchKernelGGL((k_row<double, 2>), gr, br, lr, st, a);
        else if (a.mode == 3) hipLaunchKernelGGL((k_row<double, 3>), gr, br, lr, st, a);
        else hipLaunchKernelGGL((k_row<double, 4>), gr, br, lr, st, a);
    }
    return hipGetLastError();
}

}  // namespace c3
