// Pixel-domain kernels: projection P m, binning P^T N^-1 (d - n_corr) and
// P^T N^-1 P, the per-pixel 3x3 solve, the time-domain chi^2 terms with their
// map adjoint, and small helpers.
//
// Binning and the map adjoint walk a segment in *strided tiles*: thread phi of
// a tile visits samples phi, phi + S, phi + 2S, ... where S is the segment's
// revisit period (the spin period in samples for a spinning scan, found by
// the autotuner's repeat probe).  Consecutive visits of one thread then hit
// the same pixel, so each thread accumulates its pixel's 3-vector and 3x3 in
// registers and touches global memory (FP64 atomics) only when the pixel
// changes.  Any S is correct; only the atomic traffic depends on it.
#include <algorithm>

#include "common.h"

namespace {

// ---------------------------------------------------------------- binning
// acc is pixel-major, [npt][10]: a flush adds to the ten words of one
// pixel's record (one or two cache lines), not to ten lines npt apart.
__device__ __forceinline__ void flush_acc(double *acc, int64_t npt, int64_t gp, const double *a) {
    (void)npt;
#pragma unroll
    for (int j = 0; j < 10; ++j) atomicAdd(acc + gp * 10 + j, a[j]);
}

// Bin tile (x = first entry of the run list, y = first phase, z = stride S,
// w = phases | entries << 16); run entry = (segment, phase offset o).  Lane
// phase Phi visits t = (Phi - o) mod S, + S, ... of each of the run's
// segments in turn, so segments that see the same pixels (the two radiometers
// of a horn, and the same horn's consecutive scans at equal spin phase) share
// one register accumulation and its flushes.
// TD: type of d, TN: type of n_corr (NC = false: no n_corr).  Both are
// compile-time, so a revisit's loads issue back to back with no branch
// between them and are converted only once all of them are in flight.
template <typename TN, typename TD, bool NC>
__global__ __launch_bounds__(C3_NT) void k_bin(LayoutDev Ld, const int4 *__restrict__ tiles,
                                               const int2 *__restrict__ runs,
                                               const int32_t *__restrict__ pix,
                                               const uint16_t *__restrict__ psi,
                                               const TD *__restrict__ d,
                                               const TN *__restrict__ ncorr,
                                               const double *__restrict__ gain,
                                               const double *__restrict__ sigma0,
                                               const cx<double> *__restrict__ trig,
                                               double *__restrict__ acc, uint32_t *__restrict__ err) {
    // cos/sin 2psi repeat every 2048 psi bins
    __shared__ cx<double> tr[2048];
    const int4 tl = tiles[blockIdx.x];
    for (int b = threadIdx.x; b < 2048; b += C3_NT) tr[b] = trig[b];
    __syncthreads();
    const int S = tl.z;
    const int nph = tl.w & 0xFFFF, ngrp = tl.w >> 16;
    const int phi = tl.y + threadIdx.x;
    if ((int)threadIdx.x >= nph) return;
    const int seg0 = runs[tl.x].x;
    const int64_t poff = Ld.band[Ld.seg_band[seg0]].pix_off;
    const uint32_t npix = (uint32_t)Ld.band[Ld.seg_band[seg0]].npix;
    const int64_t npt = Ld.npix_total;
    // three register accumulators, the current pixel and the two before it
    // (most recent first), so a phase that crosses pixel edges or alternates
    // between pixels rarely flushes before its tile ends.  A flush inside the
    // loop is costly beyond its atomics: loads and atomics share one in-order
    // completion counter, so the next revisit's loads also wait for them.  On
    // the 70 GHz-like set no lane meets a fourth pixel within a tile.
    double a[10], o[10], q[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) a[j] = o[j] = q[j] = 0.0;
    int cur = -1, old = -1, older = -1;
    double w = 0, gw = 0;
    bool bad = false;  // a binned d - n_corr is not finite
    auto step = [&](int p, int b, double v) {
        if ((uint32_t)p >= npix) return;  // out-of-range pixels are not binned
        bad |= !isfinite(v);
        if (p != cur) {
            if (p == old) {  // a <-> o
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    const double x = a[j];
                    a[j] = o[j];
                    o[j] = x;
                }
                old = cur;
                cur = p;
            } else if (p == older) {  // q -> a -> o -> q
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    const double x = q[j];
                    q[j] = o[j];
                    o[j] = a[j];
                    a[j] = x;
                }
                older = old;
                old = cur;
                cur = p;
            } else {  // a new pixel: the least recent one leaves
                if (older >= 0) flush_acc(acc, npt, poff + older, q);
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    q[j] = o[j];
                    o[j] = a[j];
                    a[j] = 0.0;
                }
                older = old;
                old = cur;
                cur = p;
            }
        }
        const cx<double> cs = tr[b & 2047];
        const double wv = w * v;
        a[0] += wv;
        a[1] += wv * cs.x;
        a[2] += wv * cs.y;
        a[3] += gw;
        a[4] += gw * cs.x;
        a[5] += gw * cs.y;
        a[6] += gw * cs.x * cs.x;
        a[7] += gw * cs.x * cs.y;
        a[8] += gw * cs.y * cs.y;
        a[9] += 1.0;
    };
    for (int gi = 0; gi < ngrp; ++gi) {
        const int2 re = runs[tl.x + gi];
        const int seg = re.x;
        if (Ld.seg_accept && !Ld.seg_accept[seg]) continue;
        const int64_t s0 = Ld.seg_off[seg];
        const int n = (int)(Ld.seg_off[seg + 1] - s0);
        const double g = gain[seg];
        const double s2 = sigma0[seg];
        w = g / (s2 * s2);
        gw = g * w;
        int t = phi - re.y;  // the offset is in [0, S): one wrap at most
        if (t < 0) t += S;
        // eight revisits in flight (with the flushes' atomics on one record
        // each, loads in flight bound the pass: 4.64 ms with two, 4.19 with
        // four, 4.10 with eight on the 70 GHz-like set)
        for (; t + 7 * S < n; t += 8 * S) {
            int p[8], b[8];
            TD dv[8];
            TN nv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = s0 + t + u * S;
                p[u] = pix[i];
                b[u] = psi[i];
                dv[u] = d[i];
                if constexpr (NC) nv[u] = ncorr[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                double v = (double)dv[u];
                if constexpr (NC) v -= (double)nv[u];
                step(p[u], b[u], v);
            }
        }
        for (; t < n; t += S) {
            const int64_t i = s0 + t;
            double v = (double)d[i];
            if constexpr (NC) v -= (double)ncorr[i];
            step(pix[i], psi[i], v);
        }
    }
    if (cur >= 0) flush_acc(acc, npt, poff + cur, a);
    if (old >= 0) flush_acc(acc, npt, poff + old, o);
    if (older >= 0) flush_acc(acc, npt, poff + older, q);
    if (bad && err) atomicOr(err, C3_ERR_NONFINITE);
}

// ---------------------------------------------------------------- projection
// s = g (T + Q cos 2psi + U sin 2psi), or the residual r = d - s, on strided
// tiles; the thread keeps the map values of its current pixel in registers
// across revisits (and across the tile's segments), so the map is read once
// per pixel change instead of once per sample.
// T, Q, U of one pixel in one aligned record (one load per pixel change)
template <typename T>
struct alignas(4 * sizeof(T)) Stokes4 {
    T t, q, u, pad;
};

// [3][npix] maps -> [npix] records
template <typename T>
__global__ __launch_bounds__(C3_NT) void k_interleave(const T *__restrict__ maps, int64_t npt,
                                                      Stokes4<T> *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * C3_NT + threadIdx.x; i < npt; i += (int64_t)gridDim.x * C3_NT)
        out[i] = Stokes4<T>{maps[i], maps[npt + i], maps[2 * npt + i], (T)0};
}

// SUB: write d - s (d, of type TD, read per sample); otherwise s (d unused).
// A residual of a few noise units is the difference of two numbers a hundred
// times larger (d and g T), so its rounding is ordered by size.  FP32: the
// gain as a sum of two floats g_hi + g_lo, then r = d - g_hi T - g_lo T -
// g_hi (Q cos 2psi + U sin 2psi), each step one fused multiply-add whose
// result is already residual-sized (about 2e-6 of r against 2e-5 for r =
// d - g (T + Q c + U s) in float).  FP64: the plain sum.  With SUB a lane
// that meets a non-finite d - s at an in-range pixel raises C3_ERR_NONFINITE.
template <typename T, typename TD, bool SUB>
__global__ __launch_bounds__(C3_NT) void k_resid(LayoutDev Ld, const int4 *__restrict__ tiles,
                                                 const int32_t *__restrict__ pix,
                                                 const uint16_t *__restrict__ psi,
                                                 const TD *__restrict__ d,
                                                 const Stokes4<T> *__restrict__ maps,
                                                 const double *__restrict__ gain,
                                                 const cx<T> *__restrict__ trig,
                                                 T *__restrict__ r_out, uint32_t *__restrict__ err) {
    __shared__ cx<T> tr[2048];
    const int4 tl = tiles[blockIdx.x];
    for (int b = threadIdx.x; b < 2048; b += C3_NT) tr[b] = trig[b];
    __syncthreads();
    const int S = tl.z;
    const int nph = tl.w & 0xFFFF, ngrp = tl.w >> 16;
    const int phi = tl.y + threadIdx.x;
    if ((int)threadIdx.x >= nph) return;
    const int band = Ld.seg_band[tl.x];
    const int64_t poff = Ld.band[band].pix_off;
    const uint32_t npix = (uint32_t)Ld.band[band].npix;
    int cur = -1;
    T mT = 0, mQ = 0, mU = 0;
    T ghi = 0, glo = 0;
    bool bad = false;
    auto step = [&](int64_t i, int p, int b, T dv) {
        if (p != cur) {
            cur = p;
            if ((uint32_t)p < npix) {
                const Stokes4<T> m = maps[poff + p];
                mT = m.t;
                mQ = m.q;
                mU = m.u;
            } else {
                mT = mQ = mU = (T)NAN;
            }
        }
        const cx<T> cs = tr[b & 2047];
        if constexpr (SUB) {
            T rv;
            if constexpr (sizeof(T) == 4) {
                const float pu = fmaf(mQ, cs.x, mU * cs.y);
                rv = fmaf(-ghi, mT, dv);
                rv = fmaf(-glo, mT, rv);
                rv = fmaf(-ghi, pu, rv);
            } else {
                rv = dv - ghi * (mT + mQ * cs.x + mU * cs.y);
            }
            bad |= (uint32_t)p < npix && !isfinite(rv);
            r_out[i] = rv;
        } else {
            r_out[i] = ghi * (mT + mQ * cs.x + mU * cs.y);
        }
    };
    for (int gi = 0; gi < ngrp; ++gi) {
        const int seg = tl.x + gi;
        const int64_t s0 = Ld.seg_off[seg];
        const int n = (int)(Ld.seg_off[seg + 1] - s0);
        const double g = gain[seg];
        ghi = (T)g;
        glo = (T)(g - (double)ghi);
        int t = phi;
        for (; t + 3 * S < n; t += 4 * S) {
            int p[4], b[4];
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t i = s0 + t + u * S;
                p[u] = pix[i];
                b[u] = psi[i];
                v[u] = SUB ? (T)d[i] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) step(s0 + t + u * S, p[u], b[u], v[u]);
        }
        for (; t < n; t += S) {
            const int64_t i = s0 + t;
            step(i, pix[i], psi[i], SUB ? (T)d[i] : (T)0);
        }
    }
    if (SUB && bad && err) atomicOr(err, C3_ERR_NONFINITE);
}

// the map gradient from its pixel-major accumulation records (T, Q, U,
// unused) into the [3][npt] layout of the maps
__global__ __launch_bounds__(C3_NT) void k_gmap_out(int64_t npt, const double4 *__restrict__ g4,
                                                    double *__restrict__ gm) {
    for (int64_t p = (int64_t)blockIdx.x * C3_NT + threadIdx.x; p < npt; p += (int64_t)gridDim.x * C3_NT) {
        const double4 r = g4[p];
        gm[p] = r.x;
        gm[npt + p] = r.y;
        gm[2 * npt + p] = r.z;
    }
}

// per non-empty segment: the noise parameters the draws and weights divide by
__global__ __launch_bounds__(C3_NT) void k_check_params(LayoutDev Ld, const double *__restrict__ sigma0,
                                                        const double *__restrict__ fknee,
                                                        const double *__restrict__ alpha,
                                                        uint32_t *__restrict__ err) {
    const int s = blockIdx.x * C3_NT + threadIdx.x;
    if (s >= Ld.nseg || Ld.seg_off[s + 1] <= Ld.seg_off[s]) return;
    uint32_t e = 0;
    if (sigma0) {
        const double v = sigma0[s];
        if (!(v > 0.0) || !isfinite(v)) e |= C3_ERR_SIGMA0;
    }
    if (fknee) {
        const double v = fknee[s];
        if (!(v > 0.0) || !isfinite(v)) e |= C3_ERR_FKNEE;
    }
    if (alpha) {
        const double v = alpha[s];
        if (!(v < 0.0) || !isfinite(v)) e |= C3_ERR_ALPHA;
    }
    if (e) atomicOr(err, e);
}

// ---------------------------------------------------------------- solve
// Extreme eigenvalues of a symmetric 3x3 by cyclic Jacobi rotations: each
// rotation zeroes one off-diagonal pair; eigenvalues come out with absolute
// accuracy ~eps ||A|| even when two of them coincide (1- and 2-hit pixels).
__device__ void eig3_minmax(const double A[3][3], double &lmin, double &lmax) {
    double a[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = A[i][j];
    const double scale = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
    for (int sweep = 0; sweep < 8; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        if (off <= 1e-40 * scale * scale) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2, r = 3 - p - q;
            const double apq = a[p][q];
            if (apq == 0.0) continue;
            const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
            double t;
            if (fabs(th) > 1e150)
                t = 0.5 / th;
            else
                t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            a[p][p] -= t * apq;
            a[q][q] += t * apq;
            a[p][q] = a[q][p] = 0.0;
            const double arp = a[r][p], arq = a[r][q];
            a[r][p] = a[p][r] = c * arp - s * arq;
            a[r][q] = a[q][r] = s * arp + c * arq;
        }
    }
    lmin = fmin(a[0][0], fmin(a[1][1], a[2][2]));
    lmax = fmax(a[0][0], fmax(a[1][1], a[2][2]));
}

template <typename TM>
__global__ __launch_bounds__(C3_NT) void k_solve(int64_t npix, const double *__restrict__ acc,
                                                 double rcmin, TM *__restrict__ map,
                                                 double *__restrict__ rc_out) {
    const int64_t p = (int64_t)blockIdx.x * C3_NT + threadIdx.x;
    if (p >= npix) return;
    double a[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) a[j] = acc[p * 10 + j];
    const double b0 = a[0], b1 = a[1], b2 = a[2];
    double A[3][3] = {{a[3], a[4], a[5]}, {a[4], a[6], a[7]}, {a[5], a[7], a[8]}};
    const double hits = a[9];
    double lmin, lmax;
    eig3_minmax(A, lmin, lmax);
    const double rc = lmax > 0.0 ? lmin / lmax : 0.0;
    if (rc_out) rc_out[p] = rc;
    double m0 = NAN, m1 = NAN, m2 = NAN;
    if (hits >= 3.0 && rc >= rcmin) {
        // Cholesky A = L L^T
        const double l00 = sqrt(A[0][0]);
        const double l10 = A[1][0] / l00, l20 = A[2][0] / l00;
        const double l11 = sqrt(A[1][1] - l10 * l10);
        const double l21 = (A[2][1] - l20 * l10) / l11;
        const double l22 = sqrt(A[2][2] - l20 * l20 - l21 * l21);
        const double y0 = b0 / l00;
        const double y1 = (b1 - l10 * y0) / l11;
        const double y2 = (b2 - l20 * y0 - l21 * y1) / l22;
        m2 = y2 / l22;
        m1 = (y1 - l21 * m2) / l11;
        m0 = (y0 - l10 * m1 - l20 * m2) / l00;
    }
    map[p] = (TM)m0;
    map[npix + p] = (TM)m1;
    map[2 * npix + p] = (TM)m2;
}

// ---------------------------------------------------------------- zero / set
__global__ void k_zero(uint64_t *p, int64_t nwords) {
    for (int64_t i = (int64_t)blockIdx.x * C3_NT + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * C3_NT)
        p[i] = 0;
}
__global__ void k_zero_bytes(uint8_t *p, int64_t nbytes) {
    const int64_t i = threadIdx.x;
    if (i < nbytes) p[i] = 0;
}
__global__ void k_set2(uint64_t *p, uint64_t a, uint64_t b) {
    if (threadIdx.x == 0) {
        p[0] = a;
        p[1] = b;
    }
}

// ---------------------------------------------------------------- repeat probe
// counts[L] += #{t : pix[t] == pix[t + L]} for L in [1, maxlag], t < tmax
__global__ __launch_bounds__(C3_NT) void k_probe(const int32_t *__restrict__ pix, int64_t off,
                                                 int n, int maxlag,
                                                 unsigned long long *counts) {
    const int L = blockIdx.x * C3_NT + threadIdx.x + 1;
    if (L > maxlag) return;
    const int tmax = min(n - L, 8192);
    unsigned long long c = 0;
    for (int t = 0; t < tmax; ++t) c += (pix[off + t] == pix[off + t + L]);
    atomicAdd(counts + L, c);
}

// ---------------------------------------------------------------- chi^2 time part
// chi^2 time-domain terms on strided tiles, r = d - g P m - n_corr: per
// segment sum r^2/sigma0^2, sum (P m) r and sum r^2 (block sums, one atomic
// each); with GRAD the map adjoint -2 g r / sigma0^2 (1, c, s) summed per
// pixel in registers and added with FP64 atomics when the lane's pixel
// changes, into gmap4: one 32-byte record (T, Q, U, unused) per pixel, so a
// flush's three atomics fall on one cache line.  The thread keeps its
// pixel's T, Q, U (interleaved records) in registers across revisits, and
// keeps eight revisits' loads in flight (d of type TD; both types
// compile-time, so the loads issue with no branch between).
template <typename T, typename TD, bool GRAD>
__global__ __launch_bounds__(C3_NT) void k_chisq_time(
    LayoutDev Ld, const int4 *__restrict__ tiles, const int32_t *__restrict__ pix,
    const uint16_t *__restrict__ psi, const TD *__restrict__ d, const T *__restrict__ ncorr,
    const Stokes4<T> *__restrict__ maps, const double *__restrict__ gain,
    const double *__restrict__ sigma0, const cx<double> *__restrict__ trig,
    double *__restrict__ seg_sums, double *__restrict__ gmap4, double gscale0,
    const double *__restrict__ gscale_dev) {
    // dL/dJ: a host factor times an optional device scalar (read here, so the
    // caller's autograd never waits for it)
    const double gscale = gscale_dev ? gscale0 * *gscale_dev : gscale0;
    __shared__ cx<double> tr[2048];
    __shared__ double red[3][C3_NT / 64];
    const int4 tl = tiles[blockIdx.x];
    for (int b = threadIdx.x; b < 2048; b += C3_NT) tr[b] = trig[b];
    __syncthreads();
    const int S = tl.z;
    const int nph = tl.w & 0xFFFF, ngrp = tl.w >> 16;
    const int phi = tl.y + threadIdx.x;
    const bool act = (int)threadIdx.x < nph;
    const int band = Ld.seg_band[tl.x];
    const int64_t poff = Ld.band[band].pix_off;
    const uint32_t npix = (uint32_t)Ld.band[band].npix;
    // map-adjoint sums of the current pixel and the two before it (most
    // recent first), flushed when a fourth pixel arrives or the tile ends (as
    // in the binning: a flush inside the loop also delays the next loads)
    int cur = -1, old = -1, older = -1;
    double mT = 0, mQ = 0, mU = 0;  // map values of pixel cur
    double a[3] = {0, 0, 0}, o[3] = {0, 0, 0}, q[3] = {0, 0, 0};
    double g = 0, cfac = 0, sr2 = 0, spr = 0;
    auto flush = [&](int pp, const double *x) {
        double *rec = gmap4 + (poff + pp) * 4;
        atomicAdd(rec, x[0]);
        atomicAdd(rec + 1, x[1]);
        atomicAdd(rec + 2, x[2]);
    };
    auto step = [&](int p, int b, double dv, double nc) {
        if ((uint32_t)p >= npix) return;  // out-of-range pixels are not in the likelihood
        if (p != cur) {
            if constexpr (GRAD) {
                if (p == old) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const double x = a[j];
                        a[j] = o[j];
                        o[j] = x;
                    }
                    old = cur;
                } else if (p == older) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const double x = q[j];
                        q[j] = o[j];
                        o[j] = a[j];
                        a[j] = x;
                    }
                    older = old;
                    old = cur;
                } else {
                    if (older >= 0) flush(older, q);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        q[j] = o[j];
                        o[j] = a[j];
                        a[j] = 0.0;
                    }
                    older = old;
                    old = cur;
                }
            }
            cur = p;
            const Stokes4<T> m = maps[poff + p];
            mT = m.t;
            mQ = m.q;
            mU = m.u;
        }
        const cx<double> cs = tr[b & 2047];
        const double Pm = mT + mQ * cs.x + mU * cs.y;
        const double r = dv - g * Pm - nc;
        sr2 += r * r;
        spr += Pm * r;
        if constexpr (GRAD) {
            const double cr = cfac * r;
            a[0] += cr;
            a[1] += cr * cs.x;
            a[2] += cr * cs.y;
        }
    };
    for (int gi = 0; gi < ngrp; ++gi) {
        const int seg = tl.x + gi;
        if (Ld.seg_accept && !Ld.seg_accept[seg]) continue;  // uniform over the block
        const int64_t s0 = Ld.seg_off[seg];
        const int n = (int)(Ld.seg_off[seg + 1] - s0);
        g = gain[seg];
        const double sg = sigma0[seg];
        const double is2 = 1.0 / (sg * sg);
        cfac = -2.0 * g * is2 * gscale;
        sr2 = spr = 0;
        int t = act ? phi : n;
        for (; t + 7 * S < n; t += 8 * S) {  // eight revisits' loads in flight
            int p[8], b[8];
            TD v[8];
            T c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = s0 + t + u * S;
                p[u] = pix[i];
                b[u] = psi[i];
                v[u] = d[i];
                c[u] = ncorr[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) step(p[u], b[u], (double)v[u], (double)c[u]);
        }
        for (; t < n; t += S) {
            const int64_t i = s0 + t;
            step(pix[i], psi[i], (double)d[i], (double)ncorr[i]);
        }
        // per-segment sums: block reduction, one atomic per sum
        double v[3] = {sr2 * is2, spr, sr2};
        for (int j = 0; j < 3; ++j) {
            double x = v[j];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = x;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double x = 0;
            for (int w = 0; w < C3_NT / 64; ++w) x += red[threadIdx.x][w];
            atomicAdd(seg_sums + (int64_t)seg * 4 + threadIdx.x, x);
        }
        __syncthreads();
    }
    if constexpr (GRAD) {
        if (cur >= 0) flush(cur, a);
        if (old >= 0) flush(old, o);
        if (older >= 0) flush(older, q);
    }
}

__global__ __launch_bounds__(C3_NT) void k_chisq_finish(
    LayoutDev Ld, const double *__restrict__ st, const double *__restrict__ sw,
    const double *__restrict__ gain, const double *__restrict__ sigma0,
    const double *__restrict__ fknee, const double *__restrict__ alpha, double gscale0,
    const double *__restrict__ gscale_dev, double *chisq, double *ggain, double *gsig, double *gfk,
    double *galpha) {
    const double gscale = gscale_dev ? gscale0 * *gscale_dev : gscale0;
    const int s = blockIdx.x * C3_NT + threadIdx.x;
    if (s >= Ld.nseg) return;
    const bool ok = !Ld.seg_accept || Ld.seg_accept[s];
    const double sg = sigma0[s];
    const double *t = st + (int64_t)s * 4;
    const double *w = sw + (int64_t)s * 4;
    if (chisq) chisq[s] = ok ? t[0] + w[0] : 0.0;
    if (ggain) ggain[s] = ok ? -2.0 * t[1] / (sg * sg) * gscale : 0.0;
    if (!ok) return;
    const int det = Ld.seg_det[s];
    if (gsig) atomicAdd(gsig + det, gscale * (-2.0 * t[2] / (sg * sg * sg) + 2.0 / sg * w[1]));
    if (gfk) atomicAdd(gfk + det, gscale * (-alpha[s] / fknee[s]) * w[1]);
    if (galpha) atomicAdd(galpha + det, gscale * w[2]);
}

// ---------------------------------------------------------------- launch helpers
// the strided kernels are compiled per element type of d (and of n_corr), so
// the launchers pick the instantiation here

template <typename TN>
void launch_bin_typed(hipStream_t st, const LayoutDev &L, const int4 *tiles, int ntile, const int2 *runs,
                      const int32_t *pix,
                      const uint16_t *psi, const void *d, int d_f64, const TN *nc, const double *gain,
                      const double *sigma0, const cx<double> *tr, double *acc, uint32_t *err) {
    const dim3 g(ntile), b(C3_NT);
    if (d_f64) {
        const double *dd = (const double *)d;
        if (nc)
            hipLaunchKernelGGL((k_bin<TN, double, true>), g, b, 0, st, L, tiles, runs, pix, psi, dd, nc, gain, sigma0,
                               tr, acc, err);
        else
            hipLaunchKernelGGL((k_bin<TN, double, false>), g, b, 0, st, L, tiles, runs, pix, psi, dd, nc, gain, sigma0,
                               tr, acc, err);
    } else {
        const float *df = (const float *)d;
        if (nc)
            hipLaunchKernelGGL((k_bin<TN, float, true>), g, b, 0, st, L, tiles, runs, pix, psi, df, nc, gain, sigma0,
                               tr, acc, err);
        else
            hipLaunchKernelGGL((k_bin<TN, float, false>), g, b, 0, st, L, tiles, runs, pix, psi, df, nc, gain, sigma0,
                               tr, acc, err);
    }
}

// maps -> interleaved records, then s = g P m (d == NULL) or r = d - g P m
template <typename T>
void launch_resid_typed(hipStream_t st, const LayoutDev &L, const int4 *tiles, int ntile, const int32_t *pix,
                        const uint16_t *psi, const void *d, int d_f64, const void *maps, void *maps4,
                        const double *gain, const void *trig, void *r_out, uint32_t *err) {
    const int64_t npt = L.npix_total;
    const int gi = (int)std::min<int64_t>((npt + C3_NT - 1) / C3_NT, 65536);
    hipLaunchKernelGGL(k_interleave<T>, dim3(gi), dim3(C3_NT), 0, st, (const T *)maps, npt, (Stokes4<T> *)maps4);
    const Stokes4<T> *m4 = (const Stokes4<T> *)maps4;
    const cx<T> *tr = (const cx<T> *)trig;
    T *out = (T *)r_out;
    const dim3 g(ntile), b(C3_NT);
    if (!d)
        hipLaunchKernelGGL((k_resid<T, T, false>), g, b, 0, st, L, tiles, pix, psi, (const T *)nullptr, m4, gain,
                           tr, out, err);
    else if (d_f64)
        hipLaunchKernelGGL((k_resid<T, double, true>), g, b, 0, st, L, tiles, pix, psi, (const double *)d, m4,
                           gain, tr, out, err);
    else
        hipLaunchKernelGGL((k_resid<T, float, true>), g, b, 0, st, L, tiles, pix, psi, (const float *)d, m4,
                           gain, tr, out, err);
}

template <typename T>
void launch_chisq_typed(hipStream_t st, const LayoutDev &L, const int4 *tiles, int ntile, const int32_t *pix,
                        const uint16_t *psi, const void *d, int d_f64, const void *ncorr, const void *maps,
                        void *maps4, const double *gain, const double *sigma0, const void *trig64,
                        double *seg_sums, double *grad_maps4, double grad_scale, const double *gscale_dev) {
    const int64_t npt = L.npix_total;
    const int gi = (int)std::min<int64_t>((npt + C3_NT - 1) / C3_NT, 65536);
    hipLaunchKernelGGL(k_interleave<T>, dim3(gi), dim3(C3_NT), 0, st, (const T *)maps, npt, (Stokes4<T> *)maps4);
    const Stokes4<T> *m4 = (const Stokes4<T> *)maps4;
    const T *nc = (const T *)ncorr;
    const cx<double> *tr = (const cx<double> *)trig64;
    const dim3 g(ntile), b(C3_NT);
#define C3_CHISQ(TD, GRAD)                                                                              \
    hipLaunchKernelGGL((k_chisq_time<T, TD, GRAD>), g, b, 0, st, L, tiles, pix, psi, (const TD *)d, nc, m4, \
                       gain, sigma0, tr, seg_sums, grad_maps4, grad_scale, gscale_dev)
    if (d_f64) {
        if (grad_maps4)
            C3_CHISQ(double, true);
        else
            C3_CHISQ(double, false);
    } else {
        if (grad_maps4)
            C3_CHISQ(float, true);
        else
            C3_CHISQ(float, false);
    }
#undef C3_CHISQ
}

}  // namespace

namespace c3 {

hipError_t launch_bin_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                            int ntile, const int2 *runs, const int32_t *pix, const uint16_t *psi,
                            const void *d, int d_f64, const void *ncorr, const double *gain,
                            const double *sigma0, const void *trig64, double *acc, uint32_t *err) {
    if (ntile <= 0) return hipSuccess;
    if (mixed)
        launch_bin_typed(st, L, tiles, ntile, runs, pix, psi, d, d_f64, (const float *)ncorr, gain, sigma0,
                         (const cx<double> *)trig64, acc, err);
    else
        launch_bin_typed(st, L, tiles, ntile, runs, pix, psi, d, d_f64, (const double *)ncorr, gain, sigma0,
                         (const cx<double> *)trig64, acc, err);
    return hipGetLastError();
}

hipError_t launch_resid_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                              int ntile, const int32_t *pix, const uint16_t *psi, const void *d,
                              int d_f64, const void *maps, void *maps4, const double *gain,
                              const void *trig, void *r_out, uint32_t *err) {
    if (ntile <= 0) return hipSuccess;
    if (mixed)
        launch_resid_typed<float>(st, L, tiles, ntile, pix, psi, d, d_f64, maps, maps4, gain, trig, r_out, err);
    else
        launch_resid_typed<double>(st, L, tiles, ntile, pix, psi, d, d_f64, maps, maps4, gain, trig, r_out, err);
    return hipGetLastError();
}

hipError_t launch_check_params(hipStream_t st, const LayoutDev &L, const double *sigma0, const double *fknee,
                               const double *alpha, uint32_t *err) {
    if (L.nseg <= 0 || (!sigma0 && !fknee && !alpha)) return hipSuccess;
    const int nb = (L.nseg + C3_NT - 1) / C3_NT;
    hipLaunchKernelGGL(k_check_params, dim3(nb), dim3(C3_NT), 0, st, L, sigma0, fknee, alpha, err);
    return hipGetLastError();
}

hipError_t launch_zero(hipStream_t st, void *p, int64_t bytes) {
    if (bytes <= 0) return hipSuccess;
    const int64_t nw = bytes / 8;
    if (nw > 0) {
        int64_t nb = (nw + C3_NT - 1) / C3_NT;
        if (nb > 65536) nb = 65536;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)nb), dim3(C3_NT), 0, st, (uint64_t *)p, nw);
    }
    const int64_t rem = bytes - nw * 8;
    if (rem > 0)
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(C3_NT), 0, st, (uint8_t *)p + nw * 8, rem);
    return hipGetLastError();
}

hipError_t launch_set_u64(hipStream_t st, uint64_t *p, uint64_t a, uint64_t b) {
    hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, st, p, a, b);
    return hipGetLastError();
}

hipError_t launch_solve(hipStream_t st, int64_t npix, const double *acc, double rcond_min,
                        void *map_out, int map_f64, double *rcond_out) {
    if (npix <= 0) return hipSuccess;
    const int64_t nb = (npix + C3_NT - 1) / C3_NT;
    if (map_f64)
        hipLaunchKernelGGL(k_solve<double>, dim3((unsigned)nb), dim3(C3_NT), 0, st, npix, acc,
                           rcond_min, (double *)map_out, rcond_out);
    else
        hipLaunchKernelGGL(k_solve<float>, dim3((unsigned)nb), dim3(C3_NT), 0, st, npix, acc,
                           rcond_min, (float *)map_out, rcond_out);
    return hipGetLastError();
}

hipError_t launch_repeat_probe(hipStream_t st, const int32_t *pix, int64_t off, int n, int maxlag,
                               unsigned long long *counts) {
    const int nb = (maxlag + C3_NT - 1) / C3_NT;
    hipLaunchKernelGGL(k_probe, dim3(nb), dim3(C3_NT), 0, st, pix, off, n, maxlag, counts);
    return hipGetLastError();
}

hipError_t launch_chisq_time_tiles(hipStream_t st, const LayoutDev &L, int mixed, const int4 *tiles,
                                   int ntile, const int32_t *pix, const uint16_t *psi,
                                   const void *d, int d_f64, const void *ncorr, const void *maps,
                                   void *maps4, const double *gain, const double *sigma0,
                                   const void *trig64, double *seg_sums, double *grad_maps4,
                                   double grad_scale, const double *gscale_dev) {
    if (ntile <= 0) return hipSuccess;
    if (mixed)
        launch_chisq_typed<float>(st, L, tiles, ntile, pix, psi, d, d_f64, ncorr, maps, maps4, gain, sigma0,
                                  trig64, seg_sums, grad_maps4, grad_scale, gscale_dev);
    else
        launch_chisq_typed<double>(st, L, tiles, ntile, pix, psi, d, d_f64, ncorr, maps, maps4, gain, sigma0,
                                   trig64, seg_sums, grad_maps4, grad_scale, gscale_dev);
    return hipGetLastError();
}

hipError_t launch_gmap_out(hipStream_t st, int64_t npt, const double *grad_maps4, double *grad_maps) {
    if (npt <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>((npt + C3_NT - 1) / C3_NT, 65536);
    hipLaunchKernelGGL(k_gmap_out, dim3(g), dim3(C3_NT), 0, st, npt, (const double4 *)grad_maps4, grad_maps);
    return hipGetLastError();
}

hipError_t launch_chisq_finish(hipStream_t st, const LayoutDev &L, const double *seg_time,
                               const double *seg_whittle, const double *gain, const double *sigma0,
                               const double *fknee, const double *alpha, double grad_scale,
                               const double *gscale_dev, double *chisq_seg, double *grad_gain, double *grad_sigma0,
                               double *grad_fknee, double *grad_alpha) {
    if (L.nseg <= 0) return hipSuccess;
    const int nb = (L.nseg + C3_NT - 1) / C3_NT;
    hipLaunchKernelGGL(k_chisq_finish, dim3(nb), dim3(C3_NT), 0, st, L, seg_time, seg_whittle,
                       gain, sigma0, fknee, alpha, grad_scale, gscale_dev, chisq_seg, grad_gain, grad_sigma0,
                       grad_fknee, grad_alpha);
    return hipGetLastError();
}

}  // namespace c3
