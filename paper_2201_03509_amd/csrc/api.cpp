// C-ABI of c3tod: context, host-side validation, planning and launch order.
//
// Planning turns the segment table into device-resident work lists once per
// distinct layout (keyed by a hash of the host mirrors) and caches them:
//   * one FFT plan per distinct complex length M (split M = M1 x M2, radix
//     orders, twiddle tables computed in extended precision on the host);
//   * column and row task lists for the three FFT passes, ordered longest
//     segment first (LPT) so the tail of every launch is short;
//   * decode tasks (blocks of up to 256 chunks of one segment);
//   * strided bin tiles per segment (revisit period per band).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "rowc.h"
#include "tune.h"
#include "validate.h"

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= n && p) return hipSuccess;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            n = 0;
        }
        if (bytes == 0) bytes = 8;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        return e;
    }
    template <typename T>
    hipError_t upload(const std::vector<T> &v, hipStream_t st) {
        hipError_t e = ensure(v.size() * sizeof(T));
        if (e != hipSuccess || v.empty()) return e;
        e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    }
};

uint64_t fnv(uint64_t h, const void *data, size_t n) {
    const uint8_t *b = (const uint8_t *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

int64_t next_5smooth(int64_t n) {
    if (n <= 1) return 1;
    for (int64_t m = n;; ++m) {
        int64_t x = m;
        while (x % 2 == 0) x /= 2;
        while (x % 3 == 0) x /= 3;
        while (x % 5 == 0) x /= 5;
        if (x == 1) return m;
    }
}

struct Plan {
    uint64_t key = 0;
    uint64_t gen = 0;                     // context-unique; renewed when bin tiles change
    int mixed = 0;
    std::vector<SegInfo> h_segs;
    std::vector<int32_t> seg_order;       // LPT order
    std::vector<FftPlan> h_plans;
    std::map<int64_t, int> plan_of_M;
    DevBuf segs, plans, twpool, col_tasks, row_tasks, fsamp;
    int ncol = 0, nrow = 0;
    // FFT batches: contiguous ranges of the column/row task lists whose
    // segments share one workspace region (sized to stay cache resident)
    struct ColGroup {
        int m1reg;                        // register column length, 0: LDS tiles
        int t0, nt;                       // range of the column task list
    };
    struct RowGroup {
        int lds;                          // dynamic LDS bytes of the launch
        int t0, nt;                       // range of the row task list
        int rowc;                         // row length of a compiled row kernel, 0: generic
        bool pair_rows = false;           // rows the compiled kernel's pair tasks cover (not mode 3)
    };
    struct Batch {
        int col0, ncol, row0, nrow;
        std::vector<ColGroup> groups;     // column tasks of the batch, by kernel
        std::vector<RowGroup> rgroups;    // row tasks of the batch, by blocks per CU
    };
    std::vector<Batch> batches;
    int col_lds = 0, row_lds = 0;         // dynamic LDS bytes per FFT pass
    int64_t work_elems = 0;
    int64_t ext_elems = 0;                // complex elements of all extended vectors (ext_off)
    DevBuf sample_tiles;
    DevBuf sample_seg_tiles;              // per segment (first sample tile, count)
    // masked n_corr solver: tiles over the extended vectors, per-segment tile ranges
    DevBuf cg_tiles, cg_seg_tiles;
    int ncg = 0;
    int nsample_tiles = 0;
    // decode tasks per chunk length
    std::map<int, std::unique_ptr<DevBuf>> dec_tasks;
    std::map<int, int> ndec;
    // bin tiles, rebuilt when strides change
    DevBuf bin_tiles;
    int nbin = 0;
    std::vector<int> bin_stride;          // per band, as used for bin_tiles
    // binning runs: tiles over chains of one detector pair's segments across
    // consecutive scans, and the (segment, phase offset) list they index
    DevBuf run_tiles, run_segs;
    int nrun_tiles = 0;
    int run_want = -1;                    // tod_set_bin_runs value the runs were built for
    std::vector<int> run_stride;          // strides the runs were built for
};

}  // namespace

struct tod_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t *d_err = nullptr;
    uint64_t *d_seed_iter = nullptr;
    DevBuf trig32, trig64, work, seg_sums, seg_whittle, probe_counts, resid;
    DevBuf gmap4;                         // map-gradient records (T, Q, U, unused) per pixel
    DevBuf dec_tabs;                      // decoding tables, rebuilt by every decode
    DevBuf dec_tabs2;                     // the TOD stream's decoding tables (tod_sweep_stream)
    DevBuf maps4;                         // the sweep's maps as (T, Q, U, 0) records
    // masked n_corr solver: Krylov vectors and the transform output (the
    // precision's type), partial sums, per-segment state, active flags and the
    // active-segment count
    DevBuf cg_x, cg_res, cg_fin, cg_fout, cg_part, cg_state, cg_act, cg_count, cg_has_gap;
    DevBuf cg_cnt, cg_base, cg_gap_idx, cg_y, cg_rho, cg_p, cg_gap_tiles, cg_seg_gap_tiles;
    // gain draw: filtered template and data (per sample), per-tile partial sums
    DevBuf gain_kt, gain_kd, gain_part;
    // noise-parameter draw: periodogram bins per segment, white-residual partials
    DevBuf xi_bins, xi_part;
    std::map<uint64_t, std::unique_ptr<Plan>> plans;
    std::map<int, int> band_stride;       // band index -> stride (tuned or set)
    std::map<std::string, int> stride_by_key;  // "nside:fsamp" -> stride (cache file)
    int64_t fft_batch = 0;                // complex elements per FFT batch (0: all segments)
    int bin_runs = 0;                     // scans per binning run (0: chosen per layout)
    c3tune::Table tuned;                  // FFT choices
    std::string last_error;
    uint32_t last_err_bits = 0;
    bool timing = false;
    hipEvent_t ev[8] = {};                 // scratch events (autotuning)
    std::vector<hipEvent_t> ev_pool;       // recycled timing events
    struct Rec {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;                 // launches timed since the last read
    struct GraphEntry {
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
    };
    std::map<uint64_t, GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;     // capture-only stream (default priority)
    uint64_t gen_counter = 0;             // source of Plan::gen
    void *noalloc = nullptr;              // this device's static scratch (decode_pointing_noalloc)
};

namespace {

std::string band_key(const tod_band &b);

tod_status fail(tod_ctx c, tod_status s, const std::string &msg) {
    if (c) c->last_error = msg;
    return s;
}

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t _e = (call);                                                           \
        if (_e != hipSuccess)                                                             \
            return fail(ctx, TOD_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

tod_status check_layout(tod_ctx ctx, const tod_layout *L) {
    std::string m;
    const tod_status r = c3val::check_layout(L, m);
    return r == TOD_OK ? r : fail(ctx, r, m);
}

tod_status check_huff(tod_ctx ctx, const tod_huff *h, const char *what) {
    std::string m;
    const tod_status r = c3val::check_huff(h, what, m);
    return r == TOD_OK ? r : fail(ctx, r, m);
}

LayoutDev make_layout_dev(const tod_layout *L) {
    LayoutDev d;
    memset(&d, 0, sizeof(d));
    d.seg_off = L->seg_off;
    d.seg_band = L->seg_band;
    d.seg_det = L->seg_det;
    d.seg_accept = L->seg_accept;
    d.nseg = L->nseg;
    d.nband = L->nband;
    d.ndet = L->ndet;
    d.nsamp = L->nsamp;
    d.npix_total = L->npix_total;
    for (int b = 0; b < L->nband; ++b) {
        d.band[b].npix = L->bands[b].npix;
        d.band[b].pix_off = L->bands[b].pix_off;
        d.band[b].fsamp = L->bands[b].fsamp;
        d.band[b].npsi = L->bands[b].npsi;
        d.band[b].nside = L->bands[b].nside;
    }
    return d;
}

HuffDev make_huff_dev(const tod_huff *h) {
    HuffDev d;
    memset(&d, 0, sizeof(d));
    d.words = h->words;
    d.seg_word_off = h->seg_word_off;
    d.seg_table = h->seg_table;
    d.tables = h->tables;
    d.table_off = h->table_off;
    d.chunk_bit = h->chunk_bit;
    d.chunk_prev = h->chunk_prev;
    d.seg_chunk_off = h->seg_chunk_off;
    d.chunk_len = h->chunk_len;
    d.ntable = h->ntable;
    return d;
}

// ------------------------------------------------------------- twiddles
struct Pool {
    std::vector<long double> re, im;
    std::map<int64_t, int64_t> sub_tab;  // L -> offset of w_L^m
    int64_t add_sub(int64_t L) {
        auto it = sub_tab.find(L);
        if (it != sub_tab.end()) return it->second;
        const int64_t off = (int64_t)re.size();
        for (int64_t m = 0; m < L; ++m) push(m, L);
        sub_tab[L] = off;
        return off;
    }
    void push(int64_t m, int64_t L) {  // e^{-2 pi i m / L}
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
        re.push_back(cosl(a));
        im.push_back(sinl(a));
    }
};

// Work order of one launch.  The chip dispatches a launch's blocks to its
// XCDs round-robin (block b to XCD b mod kXcd), each XCD with its own L2.
// Position kXcd j + x takes the j-th item of XCD x's list, so all the items
// of one group (consecutive items of v with equal key: a segment's columns or
// rows, a tile group's phases) run on one XCD.  In the column pass the two
// reads of each residual sample (at its place and at its mirror image) then
// meet in that L2, and in every pass an XCD streams through its own
// segments.  Groups go to the XCD with the fewest items so far, in the order
// of v (longest first); shorter lists are padded with `empty`, an item its
// kernel returns on at once.  Only speed depends on the order, never results.
constexpr int kXcd = 8;
template <typename T, typename Key>
std::vector<T> xcd_order(const std::vector<T> &v, Key key, const T &empty) {
    if (v.size() <= (size_t)kXcd) return v;
    std::vector<std::vector<T>> lists(kXcd);
    for (size_t i = 0; i < v.size();) {
        size_t j = i;
        while (j < v.size() && key(v[j]) == key(v[i])) ++j;
        size_t x = 0;
        for (size_t y = 1; y < lists.size(); ++y)
            if (lists[y].size() < lists[x].size()) x = y;
        lists[x].insert(lists[x].end(), v.begin() + (std::ptrdiff_t)i, v.begin() + (std::ptrdiff_t)j);
        i = j;
    }
    size_t len = 0;
    for (const auto &l : lists) len = std::max(len, l.size());
    std::vector<T> out;
    out.reserve(len * kXcd);
    for (size_t j = 0; j < len; ++j)
        for (int x = 0; x < kXcd; ++x) out.push_back(j < lists[x].size() ? lists[x][j] : empty);
    return out;
}

// empty items: a column task of no columns, a row task of no segment, a
// strided tile of no phases and no segments
ColTask empty_col(const ColTask &like) {
    ColTask e = like;
    e.c0 = 0;
    e.n = 0;
    e.M2 = 0;
    return e;
}
RowTask empty_row() {
    RowTask e;
    memset(&e, 0, sizeof(e));
    e.seg = -1;
    return e;
}
std::vector<int4> xcd_order_tiles(const std::vector<int4> &v) {
    if (v.empty()) return v;
    return xcd_order(v, [](const int4 &t) { return t.x; }, make_int4(v[0].x, 0, 1, 0));
}

tod_status build_plan(tod_ctx ctx, const tod_layout *L, int mixed, uint64_t key, Plan **out) {
    auto P = std::make_unique<Plan>();
    P->key = key;
    P->gen = ++ctx->gen_counter;
    P->mixed = mixed;
    const int nseg = L->nseg;
    P->h_segs.resize(nseg);
    Pool pool;
    int64_t scr = 0, ext = 0;
    for (int s = 0; s < nseg; ++s) {
        SegInfo &g = P->h_segs[s];
        g.samp_off = L->h_seg_off[s];
        g.n = (int32_t)(L->h_seg_off[s + 1] - L->h_seg_off[s]);
        g.band = L->h_seg_band[s];
        g.det = 0;
        g.accept = 1;
        g.pad = 0;
        g.scr_off = scr;
        g.ext_off = ext;
        g.plan = -1;
        if (g.n <= 0) continue;
        const int64_t M = next_5smooth(g.n);
        ext += M;
        auto it = P->plan_of_M.find(M);
        if (it == P->plan_of_M.end()) {
            c3tune::FftChoice ch;
            // a tuned choice is used only if the kernels here can run it
            const bool tuned = ctx->tuned.get(mixed, M, ch) && c3tune::choice_ok(ch, M, mixed);
            if (!tuned && !c3tune::default_choice(M, mixed, ch))
                return fail(ctx, TOD_ENOTSUP, "no FFT plan for M = " + std::to_string(M));
            FftPlan fp;
            memset(&fp, 0, sizeof(fp));
            fp.M = (int32_t)M;
            fp.M1 = ch.M1;
            fp.M2 = ch.M2;
            fp.B = ch.colreg ? C3_COL_NT : ch.B;
            fp.colreg = ch.colreg;
            fp.nr1 = (int)ch.r1.size();
            fp.nr2 = (int)ch.r2.size();
            for (size_t i = 0; i < ch.r1.size(); ++i) fp.r1[i] = (int8_t)ch.r1[i];
            for (size_t i = 0; i < ch.r2.size(); ++i) fp.r2[i] = (int8_t)ch.r2[i];
            fp.tw1 = pool.add_sub(ch.M1);
            fp.tw2 = pool.add_sub(ch.M2);
            const int64_t N = 2 * M;
            fp.twlo = (int64_t)pool.re.size();
            for (int64_t m = 0; m < 1024; ++m) pool.push(m, N);
            fp.twhi = (int64_t)pool.re.size();
            for (int64_t h = 0; h <= N / 1024 + 1; ++h) pool.push(h * 1024, N);
            fp.twr = fp.twh = -1;
            if (mixed && c3rowc::compiled(ch.M2)) {
                // the compiled row kernel's stage twiddles (rowc.h layout) and w_2L^j
                const int L = ch.M2;
                const c3rowc::Plan3 rp = c3rowc::plan(L);
                fp.twr = (int64_t)pool.re.size();
                for (int st = 1; st < 3; ++st) {
                    const int R = rp.r[st], NS = c3rowc::row_ns(L, st);
                    for (int k = 0; k < NS; ++k)
                        for (int t = 1; t < R; ++t) pool.push((int64_t)t * k, (int64_t)NS * R);
                }
                fp.twh = (int64_t)pool.re.size();
                for (int j = 0; j < L; ++j) pool.push(j, 2 * (int64_t)L);
            }
            P->plan_of_M[M] = (int)P->h_plans.size();
            P->h_plans.push_back(fp);
            it = P->plan_of_M.find(M);
        }
        g.plan = it->second;
    }
    P->ext_elems = ext;
    // LPT order: longest FFT first
    P->seg_order.resize(nseg);
    for (int s = 0; s < nseg; ++s) P->seg_order[s] = s;
    std::stable_sort(P->seg_order.begin(), P->seg_order.end(), [&](int a, int b) {
        return P->h_segs[a].n > P->h_segs[b].n;
    });
    // batches in LPT order; each batch reuses the workspace from offset 0.
    // Column tasks of a batch are grouped by column kernel (one launch each).
    // Row tasks are grouped by how many row blocks fit on a CU (their LDS is
    // two rows of M2), each launch sized to its own longest row.
    const int esz = mixed ? (int)sizeof(cx<float>) : (int)sizeof(cx<double>);
    std::vector<ColTask> col;
    std::vector<RowTask> row;
    std::map<int, std::vector<ColTask>> bcol;            // m1reg -> column tasks of the open batch
    std::map<int, std::pair<int, std::vector<RowTask>>> brow;  // -blocks per CU -> (lds, row tasks)
    std::map<int, std::vector<RowTask>> browc;           // compiled row length -> two-row tasks
    std::map<int, std::vector<RowTask>> bself;           // compiled row length -> rows k1 = 0, M1/2
    Plan::Batch cur{0, 0, 0, 0, {}, {}};
    auto close_batch = [&]() {
        cur.col0 = (int)col.size();
        for (auto &kv : bcol) {
            // register column kernels (kv.first = M1 > 0) return on an empty task
            if (kv.first > 0 && !kv.second.empty())
                kv.second = xcd_order(kv.second, [](const ColTask &t) { return t.seg; }, empty_col(kv.second[0]));
            cur.groups.push_back({kv.first, (int)col.size(), (int)kv.second.size()});
            col.insert(col.end(), kv.second.begin(), kv.second.end());
        }
        cur.row0 = (int)row.size();
        auto row_seg = [](const RowTask &t) { return t.seg; };
        // rows that hold their own mirror modes (k1 = 0, M1/2) of a compiled
        // row length: two of them share a task of the compiled kernel
        // (pad[0] = 1 + the second row's segment, pad[1] = its k1); mode 3,
        // which has no compiled kernel, takes them one per task on the
        // generic kernel (which skips the pair tasks).  An odd one out takes
        // the generic kernel in every mode.
        std::vector<RowTask> singles;
        for (auto &kv : bself) {
            std::vector<RowTask> &v = kv.second;
            if (v.size() % 2) {
                const int rl = 2 * kv.first * esz;
                auto &rg = brow[-std::max(1, (C3_LDS_MAX - 1024) / rl)];
                rg.first = std::max(rg.first, rl);
                rg.second.push_back(v.back());
                v.pop_back();
            }
            for (size_t i = 0; i + 1 < v.size(); i += 2) {
                RowTask t = v[i];
                t.pad[0] = 1 + v[i + 1].seg;
                t.pad[1] = v[i + 1].k1;
                t.off_b = v[i + 1].off_a;
                browc[kv.first].push_back(t);
            }
            singles.insert(singles.end(), v.begin(), v.end());
        }
        for (auto &kv : browc) {
            kv.second = xcd_order(kv.second, row_seg, empty_row());
            cur.rgroups.push_back({2 * kv.first * esz, (int)row.size(), (int)kv.second.size(), kv.first});
            row.insert(row.end(), kv.second.begin(), kv.second.end());
        }
        for (auto &kv : brow) {
            kv.second.second = xcd_order(kv.second.second, row_seg, empty_row());
            cur.rgroups.push_back({kv.second.first, (int)row.size(), (int)kv.second.second.size(), 0});
            row.insert(row.end(), kv.second.second.begin(), kv.second.second.end());
        }
        if (!singles.empty()) {
            int lds = 0;
            for (const auto &kv : bself) lds = std::max(lds, 2 * kv.first * esz);
            singles = xcd_order(singles, row_seg, empty_row());
            cur.rgroups.push_back({lds, (int)row.size(), (int)singles.size(), 0, true});
            row.insert(row.end(), singles.begin(), singles.end());
        }
        cur.ncol = (int)col.size() - cur.col0;
        cur.nrow = (int)row.size() - cur.row0;
        if (cur.ncol > 0 || cur.nrow > 0) P->batches.push_back(cur);
        bcol.clear();
        brow.clear();
        browc.clear();
        bself.clear();
        cur = Plan::Batch{(int)col.size(), 0, (int)row.size(), 0, {}, {}};
    };
    for (int s : P->seg_order) {
        SegInfo &g = P->h_segs[s];
        if (g.plan < 0) continue;
        const FftPlan &fp = P->h_plans[g.plan];
        if (ctx->fft_batch > 0 && scr > 0 && scr + fp.M > ctx->fft_batch) {
            close_batch();
            scr = 0;
        }
        g.scr_off = scr;
        scr += fp.M;
        P->work_elems = std::max(P->work_elems, scr);
        std::vector<ColTask> &cv = bcol[fp.colreg ? fp.M1 : 0];
        for (int c0 = 0; c0 < fp.M2; c0 += fp.B) {
            ColTask ct;
            memset(&ct, 0, sizeof(ct));
            ct.samp_off = g.samp_off;
            ct.scr_off = g.scr_off;
            ct.ext_off = g.ext_off;
            ct.seg = s;
            ct.c0 = c0;
            ct.n = g.n;
            ct.M2 = fp.M2;
            cv.push_back(ct);
        }
        const int rl = 2 * fp.M2 * esz;
        const int per_cu = std::max(1, (C3_LDS_MAX - 1024) / std::max(rl, 1));
        auto &rg = brow[-per_cu];
        for (int k1 = 0; k1 <= fp.M1 / 2; ++k1) {
            RowTask rt;
            memset(&rt, 0, sizeof(rt));
            rt.off_a = g.scr_off + (int64_t)k1 * fp.M2;
            rt.off_b = g.scr_off + (int64_t)((fp.M1 - k1) % fp.M1) * fp.M2;
            rt.seg = s;
            rt.k1 = k1;
            // rows k1 and M1 - k1 distinct: the compiled kernel of the row length
            if (fp.twr >= 0 && k1 > 0 && 2 * k1 != fp.M1) {
                browc[fp.M2].push_back(rt);
            } else if (fp.twr >= 0) {
                bself[fp.M2].push_back(rt);
            } else {
                rg.first = std::max(rg.first, rl);
                rg.second.push_back(rt);
            }
        }
    }
    close_batch();
    P->ncol = (int)col.size();
    P->nrow = (int)row.size();
    for (const FftPlan &fp : P->h_plans) {
        if (!fp.colreg) P->col_lds = std::max(P->col_lds, fp.M1 * fp.B * esz);  // one in-place buffer
        P->row_lds = std::max(P->row_lds, 2 * fp.M2 * esz);  // one in-place buffer, two rows
    }
    std::vector<double> fs(L->nband);
    for (int b = 0; b < L->nband; ++b) fs[b] = L->bands[b].fsamp;
    // sample tiles (projection): 4096 samples per block
    std::vector<int4> tiles;
    std::vector<int2> seg_tiles(nseg);
    for (int s = 0; s < nseg; ++s) {
        const int n = P->h_segs[s].n;
        seg_tiles[s].x = (int)tiles.size();
        for (int t0 = 0; t0 < n; t0 += 4096) tiles.push_back(make_int4(s, t0, std::min(4096, n - t0), 0));
        seg_tiles[s].y = (int)tiles.size() - seg_tiles[s].x;
    }
    P->nsample_tiles = (int)tiles.size();
    hipStream_t st = ctx->stream;
    HIPCHK(P->segs.upload(P->h_segs, st));
    HIPCHK(P->plans.upload(P->h_plans, st));
    HIPCHK(P->col_tasks.upload(col, st));
    HIPCHK(P->row_tasks.upload(row, st));
    HIPCHK(P->fsamp.upload(fs, st));
    HIPCHK(P->sample_tiles.upload(tiles, st));
    HIPCHK(P->sample_seg_tiles.upload(seg_tiles, st));
    if (mixed) {
        std::vector<cx<float>> tw(pool.re.size());
        for (size_t i = 0; i < tw.size(); ++i) tw[i] = {(float)pool.re[i], (float)pool.im[i]};
        HIPCHK(P->twpool.upload(tw, st));
    } else {
        std::vector<cx<double>> tw(pool.re.size());
        for (size_t i = 0; i < tw.size(); ++i) tw[i] = {(double)pool.re[i], (double)pool.im[i]};
        HIPCHK(P->twpool.upload(tw, st));
    }
    *out = P.get();
    ctx->plans[key] = std::move(P);
    return TOD_OK;
}

void drop_graphs(tod_ctx ctx) {
    for (auto &kv : ctx->graphs) {
        if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
        if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
    ctx->graphs.clear();
}

uint64_t layout_key(const tod_layout *L, int mixed, uint64_t salt) {
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &salt, sizeof(salt));
    h = fnv(h, &mixed, sizeof(mixed));
    h = fnv(h, &salt, sizeof(salt));
    h = fnv(h, &L->nseg, sizeof(L->nseg));
    h = fnv(h, L->h_seg_off, sizeof(int64_t) * (L->nseg + 1));
    h = fnv(h, L->h_seg_band, sizeof(int32_t) * L->nseg);
    h = fnv(h, L->bands, sizeof(tod_band) * L->nband);
    if (L->h_seg_det) h = fnv(h, L->h_seg_det, sizeof(int32_t) * L->nseg);  // binning runs
    return h;
}

tod_status get_plan(tod_ctx ctx, const tod_layout *L, int mixed, Plan **out) {
    const uint64_t key = layout_key(L, mixed, ctx->tuned.version * 1000003ull + (uint64_t)ctx->fft_batch);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = it->second.get();
        return TOD_OK;
    }
    if (ctx->plans.size() > 16) {
        // captured sweeps bake in the plans' buffers: they go with them
        drop_graphs(ctx);
        ctx->plans.clear();
    }
    return build_plan(ctx, L, mixed, key, out);
}

tod_status get_decode_tasks(tod_ctx ctx, Plan *P, int C, const DecodeTask **tasks, int *ntask) {
    auto it = P->dec_tasks.find(C);
    if (it == P->dec_tasks.end()) {
        std::vector<DecodeTask> v;
        for (int s : P->seg_order) {
            const int n = P->h_segs[s].n;
            const int nch = (n + C - 1) / C;
            for (int c0 = 0; c0 < nch; c0 += C3_DEC_NT) {
                DecodeTask t;
                t.seg = s;
                t.chunk0 = c0;
                t.nchunk = std::min(C3_DEC_NT, nch - c0);
                t.pad = 0;
                v.push_back(t);
            }
        }
        auto b = std::make_unique<DevBuf>();
        HIPCHK(b->upload(v, ctx->stream));
        P->ndec[C] = (int)v.size();
        it = P->dec_tasks.emplace(C, std::move(b)).first;
    }
    *tasks = (const DecodeTask *)it->second->p;
    *ntask = P->ndec[C];
    return TOD_OK;
}

// Revisit period of the pixel stream of a band: the lag with the most equal
// pixels, probed on up to three of the band's segments.
tod_status probe_stride(tod_ctx ctx, const tod_layout *L, Plan *P, const int32_t *pix, int band,
                        int *stride) {
    const int maxlag = 16384;
    HIPCHK(ctx->probe_counts.ensure(sizeof(unsigned long long) * (maxlag + 1)));
    HIPCHK(c3::launch_zero(ctx->stream, ctx->probe_counts.p, sizeof(unsigned long long) * (maxlag + 1)));
    int used = 0;
    for (int s = 0; s < L->nseg && used < 3; ++s) {
        if (L->h_seg_band[s] != band) continue;
        const SegInfo &g = P->h_segs[s];
        if (g.n < 2 * 64) continue;
        HIPCHK(c3::launch_repeat_probe(ctx->stream, pix, g.samp_off, g.n, std::min(maxlag, g.n - 1),
                                       (unsigned long long *)ctx->probe_counts.p));
        ++used;
    }
    std::vector<unsigned long long> cnt(maxlag + 1);
    HIPCHK(hipMemcpyAsync(cnt.data(), ctx->probe_counts.p, cnt.size() * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int best = 0;
    unsigned long long bc = 0;
    for (int l = 64; l <= maxlag; ++l)
        if (cnt[l] > bc) {
            bc = cnt[l];
            best = l;
        }
    *stride = best > 0 ? best : 256;
    return TOD_OK;
}

tod_status get_bin_tiles(tod_ctx ctx, const tod_layout *L, Plan *P, const int32_t *pix,
                         const int4 **tiles, int *ntile) {
    std::vector<int> st(L->nband, 0);
    for (int b = 0; b < L->nband; ++b) {
        auto it = ctx->band_stride.find(b);
        auto kt = ctx->stride_by_key.find(band_key(L->bands[b]));
        if (it != ctx->band_stride.end() && it->second > 0) {
            st[b] = it->second;
        } else if (kt != ctx->stride_by_key.end() && kt->second > 0) {
            st[b] = kt->second;
        } else if ((int)P->bin_stride.size() == L->nband && P->bin_stride[b] > 0) {
            st[b] = P->bin_stride[b];  // the one this plan's tiles already use
        } else if (pix) {
            tod_status r = probe_stride(ctx, L, P, pix, b, &st[b]);
            if (r != TOD_OK) return r;
            ctx->band_stride[b] = st[b];
        } else {
            st[b] = 256;
        }
    }
    if (st != P->bin_stride || P->nbin == 0) {
        // tiles over groups of up to two consecutive segments of equal length
        // and band (one horn's radiometers share pointing); phases in the low
        // 16 bits of .w, the group size above them
        std::vector<int4> v;
        std::vector<char> done(L->nseg, 0);
        for (int s : P->seg_order) {
            if (done[s]) continue;
            int grp = 1;
            const int base = (s % 2 == 0) ? s : s - 1;
            int first = s;
            if (base + 1 < L->nseg && !done[base] && !done[base + 1] &&
                P->h_segs[base].n == P->h_segs[base + 1].n && P->h_segs[base].band == P->h_segs[base + 1].band) {
                first = base;
                grp = 2;
            }
            for (int g = 0; g < grp; ++g) done[first + g] = 1;
            const int n = P->h_segs[first].n;
            // a period beyond the segment visits each sample once, as S = n does
            const int S = std::max(1, std::min(st[P->h_segs[first].band], std::max(n, 1)));
            const int nph = std::min(S, n);
            for (int p0 = 0; p0 < nph; p0 += C3_NT)
                v.push_back(make_int4(first, p0, S, std::min(C3_NT, nph - p0) | (grp << 16)));
        }
        v = xcd_order_tiles(v);
        HIPCHK(P->bin_tiles.upload(v, ctx->stream));
        P->nbin = (int)v.size();
        P->bin_stride = st;
        P->gen = ++ctx->gen_counter;  // graphs captured with the old tiles no longer match
    }
    *tiles = (const int4 *)P->bin_tiles.p;
    *ntile = P->nbin;
    return TOD_OK;
}

// Binning runs.  Segments pair as in get_bin_tiles (a horn's two radiometers,
// equal neighbours in index order); a detector pair's pairs, in index order,
// are taken as consecutive scans contiguous in time, and G of them form a run
// that one tile's lanes walk in turn.  Lane phase Phi of a multi-pair run
// visits t = (Phi - A_s) mod S, phi + S, ... of each segment s, A_s being the
// samples of the detector's earlier segments in the band: the same spin phase
// in every scan, so a lane meets nearly the same pixels scan after scan (the
// spin axis drifts by less than a pixel per scan) and its register sums are
// flushed once per run.  Every residue mod S is one lane's, so every sample is
// binned once whatever the pointing does.  Pairs shorter than the stride, and
// every pair when the layout has no detector mirror, are runs of one pair with
// phases [0, min(S, n)), as before.
tod_status get_bin_runs(tod_ctx ctx, const tod_layout *L, Plan *P, const int32_t *pix,
                        const int4 **tiles, int *ntile, const int2 **runs) {
    const int4 *pt;
    int np;
    tod_status r = get_bin_tiles(ctx, L, P, pix, &pt, &np);
    if (r != TOD_OK) return r;
    if (P->run_want != ctx->bin_runs || P->run_stride != P->bin_stride || (P->nrun_tiles == 0 && np > 0)) {
        const int nseg = L->nseg;
        const std::vector<int> &st = P->bin_stride;
        auto n_of = [&](int s) { return P->h_segs[s].n; };
        auto band_of = [&](int s) { return P->h_segs[s].band; };
        auto det_of = [&](int s) { return L->h_seg_det ? L->h_seg_det[s] : -1; };
        struct Pr {
            int first, grp;
        };
        std::vector<Pr> pairs;
        for (int s = 0; s < nseg;) {
            if (s % 2 == 0 && s + 1 < nseg && n_of(s) == n_of(s + 1) && band_of(s) == band_of(s + 1)) {
                pairs.push_back({s, 2});
                s += 2;
            } else {
                pairs.push_back({s, 1});
                s += 1;
            }
        }
        // samples of each detector's earlier segments in its band
        std::vector<int64_t> A(nseg, 0);
        {
            std::map<std::pair<int, int>, int64_t> tsum;
            for (int s = 0; s < nseg; ++s) {
                int64_t &t = tsum[{band_of(s), det_of(s)}];
                A[s] = t;
                t += n_of(s);
            }
        }
        auto S_of = [&](int s) { return std::max(1, std::min(st[band_of(s)], std::max(n_of(s), 1))); };
        int G = ctx->bin_runs;
        if (!L->h_seg_det) {
            G = 1;
        } else if (G <= 0) {
            int64_t t1 = 0;
            for (const Pr &q : pairs) t1 += (std::min(S_of(q.first), std::max(n_of(q.first), 0)) + C3_NT - 1) / C3_NT;
            G = (int)std::max<int64_t>(1, std::min<int64_t>(16, t1 / 4096));
        }
        // chains of pairs of one detector pair (long pairs only), in index order
        std::map<std::tuple<int, int, int>, std::vector<int>> chains;
        std::vector<std::vector<int>> runs_of_pairs;
        for (int i = 0; i < (int)pairs.size(); ++i) {
            const Pr &q = pairs[i];
            const int s = q.first;
            if (G > 1 && n_of(s) >= st[band_of(s)])
                chains[{band_of(s), det_of(s), q.grp == 2 ? det_of(s + 1) : -1}].push_back(i);
            else
                runs_of_pairs.push_back({i});
        }
        for (auto &kv : chains)
            for (size_t a = 0; a < kv.second.size(); a += G)
                runs_of_pairs.emplace_back(kv.second.begin() + a,
                                           kv.second.begin() + std::min(kv.second.size(), a + G));
        // longest runs first
        auto run_samples = [&](const std::vector<int> &rp) {
            int64_t t = 0;
            for (int i : rp) t += (int64_t)pairs[i].grp * n_of(pairs[i].first);
            return t;
        };
        std::stable_sort(runs_of_pairs.begin(), runs_of_pairs.end(),
                         [&](const std::vector<int> &a, const std::vector<int> &b) {
                             return run_samples(a) > run_samples(b);
                         });
        std::vector<int2> segs;
        std::vector<int4> tl;
        for (const std::vector<int> &rp : runs_of_pairs) {
            const int first = (int)segs.size();
            const int s0 = pairs[rp[0]].first;
            const int S = S_of(s0);
            const bool multi = rp.size() > 1;
            int nph = multi ? S : std::min(S, n_of(s0));
            for (int i : rp)
                for (int g = 0; g < pairs[i].grp; ++g) {
                    const int sg = pairs[i].first + g;
                    segs.push_back(make_int2(sg, multi ? (int)(A[sg] % S) : 0));
                }
            const int nsg = (int)segs.size() - first;
            for (int p0 = 0; p0 < nph; p0 += C3_NT)
                tl.push_back(make_int4(first, p0, S, std::min(C3_NT, nph - p0) | (nsg << 16)));
        }
        tl = xcd_order_tiles(tl);
        HIPCHK(P->run_tiles.upload(tl, ctx->stream));
        HIPCHK(P->run_segs.upload(segs, ctx->stream));
        P->nrun_tiles = (int)tl.size();
        P->run_want = ctx->bin_runs;
        P->run_stride = st;
        P->gen = ++ctx->gen_counter;
    }
    *tiles = (const int4 *)P->run_tiles.p;
    *ntile = P->nrun_tiles;
    *runs = (const int2 *)P->run_segs.p;
    return TOD_OK;
}

c3::FftArgs fft_args(tod_ctx ctx, Plan *P, const tod_layout *L) {
    c3::FftArgs a;
    memset(&a, 0, sizeof(a));
    a.segs = (const SegInfo *)P->segs.p;
    a.plans = (const FftPlan *)P->plans.p;
    a.twpool = P->twpool.p;
    a.work = ctx->work.p;
    a.col_tasks = (const ColTask *)P->col_tasks.p;
    a.ncol_tasks = P->ncol;
    a.row_tasks = (const RowTask *)P->row_tasks.p;
    a.nrow_tasks = P->nrow;
    a.fsamp_band = (const double *)P->fsamp.p;
    a.seed_iter = ctx->d_seed_iter;
    a.col_lds = P->col_lds;
    a.row_lds = P->row_lds;
    (void)L;
    return a;
}

tod_status ensure_work(tod_ctx ctx, Plan *P) {
    const size_t elt = P->mixed ? sizeof(cx<float>) : sizeof(cx<double>);
    HIPCHK(ctx->work.ensure((size_t)P->work_elems * elt + 64));
    return TOD_OK;
}

// kernel ids of tod_kernel_times
enum { K_DECODE = 0, K_PROJECT, K_COLF, K_ROW, K_COLI, K_BIN, K_SOLVE, K_CHISQ, K_CG, K_GAIN, K_NOISE, K_NKERNEL };

hipEvent_t pool_event(tod_ctx c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// brackets one launch with events on `st` when timing is on (never in capture)
struct KTimer {
    tod_ctx c;
    int kid;
    hipStream_t st;
    hipEvent_t a = nullptr;
    KTimer(tod_ctx ctx, int k, hipStream_t s) : c(ctx), kid(k), st(s) {
        if (c->timing) {
            a = pool_event(c);
            (void)hipEventRecord(a, st);
        }
    }
    ~KTimer() {
        if (a) {
            hipEvent_t b = pool_event(c);
            (void)hipEventRecord(b, st);
            c->recs.push_back({kid, a, b});
        }
    }
};

// the FFT passes over every batch: per batch forward columns, rows, inverse columns
tod_status run_fft(tod_ctx ctx, hipStream_t st, Plan *P, int mixed, const c3::FftArgs &a0, int npass,
                   int first = 0) {
    for (const Plan::Batch &b : P->batches) {
        c3::FftArgs a = a0;
        a.col_tasks = (const ColTask *)P->col_tasks.p + b.col0;
        a.ncol_tasks = b.ncol;
        a.row_tasks = (const RowTask *)P->row_tasks.p + b.row0;
        a.nrow_tasks = b.nrow;
        for (int pass = first; pass < npass; ++pass) {
            if (pass == 1) {
                for (const Plan::RowGroup &g : b.rgroups) {
                    if (g.nt <= 0 || (g.pair_rows && a.mode != 3)) continue;
                    c3::FftArgs ag = a;
                    ag.row_tasks = (const RowTask *)P->row_tasks.p + g.t0;
                    ag.nrow_tasks = g.nt;
                    ag.row_lds = g.lds;
                    KTimer kt(ctx, K_ROW, st);
                    if (g.rowc && c3::rowc_supported(mixed, g.rowc, a.mode))
                        HIPCHK(c3::launch_rowc(st, ag, g.rowc));
                    else
                        HIPCHK(c3::launch_fft_pass(st, mixed, ag, pass, 0));
                }
                continue;
            }
            for (const Plan::ColGroup &g : b.groups) {
                c3::FftArgs ag = a;
                ag.col_tasks = (const ColTask *)P->col_tasks.p + g.t0;
                ag.ncol_tasks = g.nt;
                KTimer kt(ctx, K_COLF + pass, st);
                HIPCHK(c3::launch_fft_pass(st, mixed, ag, pass, g.m1reg));
            }
        }
    }
    return TOD_OK;
}


}  // namespace

// ============================================================== C-ABI
extern "C" {

tod_status tod_ctx_create(tod_ctx *out, int device, void *hip_stream) {
    if (!out) return TOD_EINVAL;
    *out = nullptr;
    tod_ctx ctx = new tod_ctx_s();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return TOD_EHIP;
    }
    if (hipMalloc(&ctx->d_err, 64) != hipSuccess || hipMalloc(&ctx->d_seed_iter, 64) != hipSuccess) {
        delete ctx;
        return TOD_ENOMEM;
    }
    (void)hipMemset(ctx->d_err, 0, 64);
    (void)hipMemset(ctx->d_seed_iter, 0, 64);
    // cos 2psi / sin 2psi at the centres of the 4096 psi bins, 2 psi = pi (2b+1)/2048
    std::vector<cx<float>> t32(4096);
    std::vector<cx<double>> t64(4096);
    for (int b = 0; b < 4096; ++b) {
        const long double a = 3.14159265358979323846264338327950288L * (2.0L * b + 1.0L) / 2048.0L;
        t64[b] = {(double)cosl(a), (double)sinl(a)};
        t32[b] = {(float)t64[b].x, (float)t64[b].y};
    }
    if (ctx->trig32.ensure(sizeof(cx<float>) * 4096) != hipSuccess ||
        ctx->trig64.ensure(sizeof(cx<double>) * 4096) != hipSuccess ||
        hipMemcpy(ctx->trig32.p, t32.data(), sizeof(cx<float>) * 4096, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->trig64.p, t64.data(), sizeof(cx<double>) * 4096, hipMemcpyHostToDevice) != hipSuccess) {
        delete ctx;
        return TOD_EHIP;
    }
    for (auto &e : ctx->ev) (void)hipEventCreate(&e);
    if (c3::noalloc_scratch(&ctx->noalloc) != hipSuccess) {  // device is current here
        delete ctx;
        return TOD_EHIP;
    }
    if (c3::fft_init_attributes() != hipSuccess) {
        delete ctx;
        return TOD_EHIP;
    }
    (void)hipDeviceSynchronize();
    *out = ctx;
    return TOD_OK;
}

tod_status tod_ctx_destroy(tod_ctx ctx) {
    if (!ctx) return TOD_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->graphs) {
        if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
        if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto &e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->d_err) (void)hipFree(ctx->d_err);
    if (ctx->d_seed_iter) (void)hipFree(ctx->d_seed_iter);
    delete ctx;
    return TOD_OK;
}

tod_status tod_sync(tod_ctx ctx) {
    if (!ctx) return TOD_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    uint32_t e = 0;
    HIPCHK(hipMemcpy(&e, ctx->d_err, sizeof(e), hipMemcpyDeviceToHost));
    ctx->last_err_bits = e;
    if (e) {
        char buf[256];
        snprintf(buf, sizeof(buf),
                 "device error bits 0x%x (1 invalid code, 2 chunk mismatch, 4 pixel range, 8 psi range, "
                 "16 sigma0, 32 f_knee, 64 alpha, 128 non-finite data)", e);
        return fail(ctx, TOD_ECORRUPT, buf);
    }
    return TOD_OK;
}

tod_status tod_clear_error(tod_ctx ctx) {
    if (!ctx) return TOD_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(c3::launch_zero(ctx->stream, ctx->d_err, 8));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->last_err_bits = 0;
    ctx->last_error.clear();
    return TOD_OK;
}

const char *tod_last_error(tod_ctx ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

uint32_t tod_device_error_bits(tod_ctx ctx) { return ctx ? ctx->last_err_bits : 0u; }

tod_status decode_pointing(tod_ctx ctx, const tod_layout *lay, const tod_huff *pix,
                           const tod_huff *psi, int32_t *pix_out, uint16_t *psi_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if ((r = check_huff(ctx, pix, "pix")) != TOD_OK) return r;
    if ((r = check_huff(ctx, psi, "psi")) != TOD_OK) return r;
    if (pix->chunk_len != psi->chunk_len) return fail(ctx, TOD_EINVAL, "pix and psi chunk_len differ");
    if (!pix_out || !psi_out) return fail(ctx, TOD_EINVAL, "NULL output");
    Plan *P;
    if ((r = get_plan(ctx, lay, 1, &P)) != TOD_OK) return r;
    const DecodeTask *tasks;
    int nt;
    if ((r = get_decode_tasks(ctx, P, pix->chunk_len, &tasks, &nt)) != TOD_OK) return r;
    HIPCHK(ctx->dec_tabs.ensure(sizeof(DecTab) * (size_t)(pix->ntable + psi->ntable)));
    KTimer kt(ctx, K_DECODE, ctx->stream);
    HIPCHK(c3::launch_decode(ctx->stream, make_layout_dev(lay), make_huff_dev(pix), make_huff_dev(psi),
                             (DecTab *)ctx->dec_tabs.p, tasks, nt, pix_out, psi_out, ctx->d_err));
    return TOD_OK;
}

tod_status decode_pointing_noalloc(tod_ctx ctx, const tod_layout *lay, const tod_huff *pix,
                                   const tod_huff *psi, int32_t *pix_out, uint16_t *psi_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if ((r = check_huff(ctx, pix, "pix")) != TOD_OK) return r;
    if ((r = check_huff(ctx, psi, "psi")) != TOD_OK) return r;
    if (pix->chunk_len != psi->chunk_len) return fail(ctx, TOD_EINVAL, "pix and psi chunk_len differ");
    if (!pix_out || !psi_out) return fail(ctx, TOD_EINVAL, "NULL output");
    if (!ctx->noalloc) return fail(ctx, TOD_EHIP, "no static scratch on this device");
    // the work list is counted from the host mirror and built on the device:
    // no plan, no device allocation
    const int C = pix->chunk_len;
    int64_t ntask = 0;
    for (int s = 0; s < lay->nseg; ++s) {
        const int64_t n = lay->h_seg_off[s + 1] - lay->h_seg_off[s];
        const int64_t nch = n > 0 ? (n + C - 1) / C : 0;
        ntask += (nch + C3_DEC_NT - 1) / C3_DEC_NT;
    }
    const int64_t need = c3::noalloc_task_offset((int64_t)pix->ntable + psi->ntable) +
                         ntask * (int64_t)sizeof(DecodeTask);
    if (need > (int64_t)C3_NOALLOC_BYTES || ntask > INT32_MAX) {
        char buf[160];
        snprintf(buf, sizeof(buf), "decode_pointing_noalloc needs %lld bytes of its %u-byte static scratch",
                 (long long)need, (unsigned)C3_NOALLOC_BYTES);
        return fail(ctx, TOD_ENOTSUP, buf);
    }
    KTimer kt(ctx, K_DECODE, ctx->stream);
    HIPCHK(c3::launch_decode_noalloc(ctx->stream, make_layout_dev(lay), make_huff_dev(pix), make_huff_dev(psi),
                                     ctx->noalloc, (int)ntask, pix_out, psi_out, ctx->d_err));
    return TOD_OK;
}

// one TOD or flag stream: kind 0/1 TOD in FP32/FP64, 2 flags
static tod_status decode_stream(tod_ctx ctx, const tod_layout *lay, const tod_huff *h, const char *what,
                                int kind, double quantum, uint32_t flag_mask, void *out, uint8_t *mask_out) {
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if ((r = check_huff(ctx, h, what)) != TOD_OK) return r;
    Plan *P;
    if ((r = get_plan(ctx, lay, 1, &P)) != TOD_OK) return r;
    const DecodeTask *tasks;
    int nt;
    if ((r = get_decode_tasks(ctx, P, h->chunk_len, &tasks, &nt)) != TOD_OK) return r;
    HIPCHK(ctx->dec_tabs.ensure(sizeof(DecTab) * (size_t)std::max(h->ntable, 1)));
    KTimer kt(ctx, K_DECODE, ctx->stream);
    HIPCHK(c3::launch_decode_stream(ctx->stream, make_layout_dev(lay), make_huff_dev(h), (DecTab *)ctx->dec_tabs.p,
                                    tasks, nt, kind, quantum, flag_mask, out, mask_out, ctx->d_err));
    return TOD_OK;
}

tod_status decode_tod(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const tod_huff *tod, double quantum,
                      void *d_out) {
    if (!ctx) return TOD_EINVAL;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (!d_out) return fail(ctx, TOD_EINVAL, "NULL output");
    if (!(quantum > 0.0)) return fail(ctx, TOD_EINVAL, "quantum must be > 0");
    return decode_stream(ctx, lay, tod, "tod", prec == TOD_MIXED ? 0 : 1, quantum, 0, d_out, nullptr);
}

tod_status decode_flags(tod_ctx ctx, const tod_layout *lay, const tod_huff *flags, uint32_t flag_mask,
                        uint32_t *flags_out, uint8_t *mask_out) {
    if (!ctx) return TOD_EINVAL;
    if (!flags_out && !mask_out) return fail(ctx, TOD_EINVAL, "no output");
    return decode_stream(ctx, lay, flags, "flag", 2, 1.0, flag_mask, flags_out, mask_out);
}

tod_status project_sky(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const int32_t *pix,
                       const uint16_t *psi, const void *maps, const double *gain, void *s_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (!pix || !psi || !maps || !gain || !s_out) return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    // strided tiles (the revisit period is probed from pix on first use)
    const int4 *tiles;
    int nt;
    if ((r = get_bin_tiles(ctx, lay, P, pix, &tiles, &nt)) != TOD_OK) return r;
    HIPCHK(ctx->maps4.ensure((size_t)lay->npix_total * 4 * (mixed ? 4 : 8)));
    KTimer kt(ctx, K_PROJECT, ctx->stream);
    HIPCHK(c3::launch_resid_tiles(ctx->stream, make_layout_dev(lay), mixed, tiles, nt, pix, psi, nullptr, 0,
                                  maps, ctx->maps4.p, gain, mixed ? ctx->trig32.p : ctx->trig64.p, s_out,
                                  nullptr));
    return TOD_OK;
}

static tod_status ncorr_impl(tod_ctx ctx, const tod_layout *lay, int mixed, Plan *P, const void *d,
                             tod_dtype d_dtype, const void *s, int s_f64, const double *sigma0,
                             const double *fknee, const double *alpha, int mean_only, void *out) {
    tod_status r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    c3::FftArgs a = fft_args(ctx, P, lay);
    a.in_a = d;
    a.in_a_f64 = d_dtype == TOD_F64;
    a.in_b = s;
    a.in_b_f64 = s_f64;
    a.out = out;
    a.sigma0 = sigma0;
    a.fknee = fknee;
    a.alpha = alpha;
    a.mean_only = mean_only;
    a.mode = 0;
    return run_fft(ctx, ctx->stream, P, mixed, a, 3);
}

tod_status sample_ncorr(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const void *d,
                        tod_dtype d_dtype, const void *s, const double *sigma0, const double *fknee,
                        const double *alpha, uint64_t seed, uint64_t iter, int mean_only,
                        void *ncorr_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!d || !sigma0 || !fknee || !alpha || !ncorr_out) return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    HIPCHK(c3::launch_set_u64(ctx->stream, ctx->d_seed_iter, seed, iter));
    HIPCHK(c3::launch_check_params(ctx->stream, make_layout_dev(lay), sigma0, fknee, alpha, ctx->d_err));
    return ncorr_impl(ctx, lay, mixed, P, d, d_dtype, s, !mixed, sigma0, fknee, alpha, mean_only,
                      ncorr_out);
}

// tiles of C3_CG_TILE reals over every segment's extended vector, built once per plan
static tod_status cg_tiles(tod_ctx ctx, Plan *P) {
    if (P->cg_seg_tiles.p) return TOD_OK;
    std::vector<int4> t;
    std::vector<int2> st(P->h_segs.size(), make_int2(0, 0));
    for (size_t s = 0; s < P->h_segs.size(); ++s) {
        const SegInfo &g = P->h_segs[s];
        if (g.plan < 0) continue;
        const int64_t N = 2 * (int64_t)P->h_plans[g.plan].M;
        st[s].x = (int)t.size();
        for (int64_t t0 = 0; t0 < N; t0 += C3_CG_TILE)
            t.push_back(make_int4((int)s, (int)t0, (int)std::min<int64_t>(C3_CG_TILE, N - t0), 0));
        st[s].y = (int)t.size() - st[s].x;
    }
    if (t.size() > (size_t)INT32_MAX / 2) return fail(ctx, TOD_ENOTSUP, "too many solver tiles");
    HIPCHK(P->cg_tiles.upload(t, ctx->stream));
    HIPCHK(P->cg_seg_tiles.upload(st, ctx->stream));
    P->ncg = (int)t.size();
    return TOD_OK;
}

tod_status sample_ncorr_masked(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const void *d,
                               tod_dtype d_dtype, const void *s, const uint8_t *mask,
                               const double *sigma0, const double *fknee, const double *alpha,
                               uint64_t seed, uint64_t iter, int mean_only, double tol, int max_iter,
                               void *ncorr_out, int32_t *iters_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!d || !s || !mask || !sigma0 || !fknee || !alpha || !ncorr_out)
        return fail(ctx, TOD_EINVAL, "NULL argument");
    if (!(tol >= 0.0) || max_iter < 1) return fail(ctx, TOD_EINVAL, "tol must be >= 0 and max_iter >= 1");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    if ((r = cg_tiles(ctx, P)) != TOD_OK) return r;
    const int nseg = lay->nseg;
    const size_t NR = 2 * (size_t)P->ext_elems + 64, esz = mixed ? 4 : 8;
    HIPCHK(ctx->cg_x.ensure(NR * esz));
    HIPCHK(ctx->cg_res.ensure(NR * esz));
    HIPCHK(ctx->cg_fin.ensure(NR * esz));
    HIPCHK(ctx->cg_fout.ensure(NR * esz));
    HIPCHK(ctx->cg_cnt.ensure((size_t)P->ncg * 4 + 64));
    HIPCHK(ctx->cg_base.ensure((size_t)P->ncg * 8 + 64));
    HIPCHK(ctx->cg_state.ensure((size_t)nseg * sizeof(c3::CgState) + 64));
    HIPCHK(ctx->cg_act.ensure((size_t)nseg * 4 + 64));
    HIPCHK(ctx->cg_count.ensure(64));
    hipStream_t st = ctx->stream;
    HIPCHK(c3::launch_set_u64(st, ctx->d_seed_iter, seed, iter));
    HIPCHK(c3::launch_check_params(st, make_layout_dev(lay), sigma0, fknee, alpha, ctx->d_err));
    int32_t *act = (int32_t *)ctx->cg_act.p, *count = (int32_t *)ctx->cg_count.p;
    c3::CgState *cs = (c3::CgState *)ctx->cg_state.p;
    const double tol2 = tol * tol;
    auto fin = [&](int step, const int2 *seg_tiles) -> hipError_t {
        KTimer kt(ctx, K_CG, st);
        return c3::launch_cg_finish(st, nseg, seg_tiles, (const double *)ctx->cg_part.p, cs, act, step, tol2,
                                    max_iter, count);
    };
    auto vec = [&](int op, const c3::CgVecArgs &va) -> hipError_t {
        KTimer kt(ctx, K_CG, st);
        return c3::launch_cg_vec(st, mixed, op, va);
    };
    HIPCHK(ctx->cg_part.ensure((size_t)P->ncg * 8 + 64));

    c3::FftArgs a = fft_args(ctx, P, lay);
    a.sigma0 = sigma0;
    a.fknee = fknee;
    a.alpha = alpha;
    a.full_io = 1;
    if (!mean_only) {  // F^H W1 -> fout: rows and inverse columns only
        a.mode = 3;
        a.which = 0;
        a.out = ctx->cg_fout.p;
        if ((r = run_fft(ctx, st, P, mixed, a, 3, 1)) != TOD_OK) return r;
    }
    // mu u -> res
    c3::CgVecArgs v;
    memset(&v, 0, sizeof(v));
    v.tiles = (const int4 *)P->cg_tiles.p;
    v.ntile = P->ncg;
    v.segs = (const SegInfo *)P->segs.p;
    v.act = act;
    v.cs = cs;
    v.d = d;
    v.d_f64 = d_dtype == TOD_F64;
    v.s = s;
    v.s_f64 = !mixed;
    v.mask = mask;
    v.sigma0 = sigma0;
    v.w1 = ctx->cg_fout.p;
    v.have_draw = !mean_only;
    v.x = ctx->cg_x.p;
    v.res = ctx->cg_res.p;
    v.fin = ctx->cg_fin.p;
    v.fout = ctx->cg_fout.p;
    v.part = (double *)ctx->cg_part.p;
    HIPCHK(vec(c3::CG_OP_INIT, v));
    // x0 = M b = M (mu u) + M F^H (W2 sqrt(1/P)) over every segment
    a.mode = 2;
    a.which = 3;
    a.mean_only = mean_only;
    a.in_a = ctx->cg_res.p;
    a.in_a_f64 = !mixed;
    a.out = ctx->cg_x.p;
    if ((r = run_fft(ctx, st, P, mixed, a, 3)) != TOD_OK) return r;

    // the masked extended positions: counts per extended tile, their offsets
    // and the gap tiles laid out on the host, indices filled on the device
    v.cnt = (int32_t *)ctx->cg_cnt.p;
    HIPCHK(vec(c3::CG_OP_GAP_COUNT, v));
    std::vector<int32_t> cnt(P->ncg);
    if (P->ncg) {
        HIPCHK(hipMemcpyAsync(cnt.data(), ctx->cg_cnt.p, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    std::vector<int64_t> base(P->ncg);
    {
        int64_t acc = 0;
        for (int t = 0; t < P->ncg; ++t) {
            base[t] = acc;
            acc += cnt[t];
        }
    }
    std::vector<int4> gt;
    std::vector<int2> seg_gt(nseg, make_int2(0, 0));
    std::vector<int32_t> has_gap(nseg, 0);
    int64_t total = 0;
    {
        // extended tiles are laid out segment by segment (cg_tiles), so a
        // segment's masked entries are contiguous from base[first tile]
        int t = 0;
        for (int sgi = 0; sgi < nseg; ++sgi) {
            const SegInfo &g = P->h_segs[sgi];
            if (g.plan < 0) continue;
            const int64_t N = 2 * (int64_t)P->h_plans[g.plan].M;
            const int nt = (int)((N + C3_CG_TILE - 1) / C3_CG_TILE);
            int64_t m = 0;
            for (int k = 0; k < nt; ++k) m += cnt[t + k];
            const int64_t j0 = nt ? base[t] : 0;
            t += nt;
            seg_gt[sgi].x = (int)gt.size();
            for (int64_t o = 0; o < m; o += C3_CG_TILE) {
                const int64_t j = j0 + o;
                gt.push_back(make_int4(sgi, (int)(j & 0x7FFFFFFF), (int)std::min<int64_t>(C3_CG_TILE, m - o),
                                       (int)(j >> 31)));
            }
            seg_gt[sgi].y = (int)gt.size() - seg_gt[sgi].x;
            has_gap[sgi] = m > 0;
            total += m;
        }
        if (t != P->ncg) return fail(ctx, TOD_EHIP, "extended tile layout mismatch");
    }
    if (gt.size() > (size_t)INT32_MAX / 2) return fail(ctx, TOD_ENOTSUP, "too many masked samples");
    HIPCHK(ctx->cg_gap_idx.ensure((size_t)total * 8 + 64));
    HIPCHK(ctx->cg_y.ensure((size_t)total * 8 + 64));
    HIPCHK(ctx->cg_rho.ensure((size_t)total * 8 + 64));
    HIPCHK(ctx->cg_p.ensure((size_t)total * 8 + 64));
    HIPCHK(ctx->cg_part.ensure(std::max<size_t>(P->ncg, gt.size()) * 8 + 64));
    v.part = (double *)ctx->cg_part.p;
    HIPCHK(ctx->cg_gap_tiles.upload(gt, st));
    HIPCHK(ctx->cg_seg_gap_tiles.upload(seg_gt, st));
    HIPCHK(ctx->cg_base.upload(base, st));
    HIPCHK(ctx->cg_has_gap.upload(has_gap, st));
    v.gap_base = (const int64_t *)ctx->cg_base.p;
    v.gap_idx = (int64_t *)ctx->cg_gap_idx.p;
    HIPCHK(vec(c3::CG_OP_GAP_FILL, v));
    HIPCHK(c3::launch_cg_zero(st, mixed, ctx->cg_fin.p, (int64_t)(2 * P->ext_elems)));

    // CG on the masked positions
    c3::CgVecArgs gv = v;
    gv.tiles = (const int4 *)ctx->cg_gap_tiles.p;
    gv.ntile = (int)gt.size();
    gv.y = (double *)ctx->cg_y.p;
    gv.rho = (double *)ctx->cg_rho.p;
    gv.p = (double *)ctx->cg_p.p;
    const int2 *gseg = (const int2 *)ctx->cg_seg_gap_tiles.p;
    HIPCHK(vec(c3::CG_OP_GAP_START, gv));
    HIPCHK(fin(c3::CG_RZ0, gseg));
    gv.scatter_src = gv.p;
    HIPCHK(vec(c3::CG_OP_GAP_SCATTER, gv));
    a.which = 1;  // M
    a.in_a = ctx->cg_fin.p;
    a.out = ctx->cg_fout.p;
    a.active = act;
    for (int it = 1; it <= max_iter; ++it) {
        if ((r = run_fft(ctx, st, P, mixed, a, 3)) != TOD_OK) return r;  // M S p
        HIPCHK(vec(c3::CG_OP_GAP_PQ, gv));
        HIPCHK(fin(c3::CG_ALPHA, gseg));
        HIPCHK(vec(c3::CG_OP_GAP_UPDATE, gv));
        HIPCHK(fin(c3::CG_RES, gseg));
        int32_t h = 0;
        HIPCHK(hipMemcpyAsync(&h, count, sizeof(h), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h == 0) break;
        HIPCHK(vec(c3::CG_OP_GAP_DIR, gv));
    }
    // x = x0 + M S y where the segment has masked samples
    c3::CgVecArgs fv = gv;
    fv.act = nullptr;
    fv.scatter_src = gv.y;
    HIPCHK(vec(c3::CG_OP_GAP_SCATTER, fv));
    a.active = (const int32_t *)ctx->cg_has_gap.p;
    if ((r = run_fft(ctx, st, P, mixed, a, 3)) != TOD_OK) return r;
    c3::CgVecArgs c = v;
    c.tiles = (const int4 *)P->sample_tiles.p;
    c.ntile = P->nsample_tiles;
    c.has_gap = (const int32_t *)ctx->cg_has_gap.p;
    c.out = ncorr_out;
    HIPCHK(vec(c3::CG_OP_CROP, c));
    if (iters_out) HIPCHK(c3::launch_cg_iters(st, nseg, cs, iters_out));
    return TOD_OK;
}

tod_status sample_gain(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const void *d,
                       tod_dtype d_dtype, const void *t, const double *sigma0, const double *fknee,
                       const double *alpha, uint64_t seed, uint64_t iter, int mean_only,
                       double *gain_out, double *sigma_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!d || !t || !sigma0 || !fknee || !alpha || !gain_out) return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    const size_t esz = mixed ? 4 : 8;
    HIPCHK(ctx->gain_kt.ensure((size_t)lay->nsamp * esz + 64));
    HIPCHK(ctx->gain_kd.ensure((size_t)lay->nsamp * esz + 64));
    HIPCHK(ctx->gain_part.ensure((size_t)P->nsample_tiles * sizeof(double2) + 64));
    hipStream_t st = ctx->stream;
    HIPCHK(c3::launch_set_u64(st, ctx->d_seed_iter, seed, iter));
    HIPCHK(c3::launch_check_params(st, make_layout_dev(lay), sigma0, fknee, alpha, ctx->d_err));
    c3::FftArgs a = fft_args(ctx, P, lay);
    a.sigma0 = sigma0;
    a.fknee = fknee;
    a.alpha = alpha;
    a.mode = 2;
    a.which = 2;  // 1 / (sigma0^2 + P)
    a.in_a = t;
    a.in_a_f64 = !mixed;
    a.out = ctx->gain_kt.p;
    if ((r = run_fft(ctx, st, P, mixed, a, 3)) != TOD_OK) return r;
    a.in_a = d;
    a.in_a_f64 = d_dtype == TOD_F64;
    a.out = ctx->gain_kd.p;
    if ((r = run_fft(ctx, st, P, mixed, a, 3)) != TOD_OK) return r;
    {
        KTimer kt(ctx, K_GAIN, st);
        HIPCHK(c3::launch_gain_dots(st, mixed, (const int4 *)P->sample_tiles.p, P->nsample_tiles, lay->seg_off, t,
                                    ctx->gain_kt.p, ctx->gain_kd.p, (double2 *)ctx->gain_part.p));
    }
    {
        KTimer kt(ctx, K_GAIN, st);
        HIPCHK(c3::launch_gain_finish(st, lay->nseg, (const int2 *)P->sample_seg_tiles.p,
                                      (const double2 *)ctx->gain_part.p, ctx->d_seed_iter, mean_only, gain_out,
                                      sigma_out));
    }
    return TOD_OK;
}

tod_status sample_noise(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const void *d,
                        tod_dtype d_dtype, const void *t, const double *gain, const void *ncorr,
                        const double *fknee_in, uint64_t seed, uint64_t iter, int mean_only,
                        double *sigma0_out, double *fknee_out, double *alpha_out) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!d || !t || !gain || !ncorr || !fknee_in || !sigma0_out || !fknee_out || !alpha_out)
        return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    const size_t nbin = (size_t)lay->nseg * C3_XI_NBIN;
    HIPCHK(ctx->xi_bins.ensure(nbin * 8 + 64));
    HIPCHK(ctx->xi_part.ensure((size_t)P->nsample_tiles * 8 + 64));
    hipStream_t st = ctx->stream;
    HIPCHK(c3::launch_set_u64(st, ctx->d_seed_iter, seed, iter));
    HIPCHK(c3::launch_check_params(st, make_layout_dev(lay), nullptr, fknee_in, nullptr, ctx->d_err));
    {
        KTimer kt(ctx, K_NOISE, st);
        HIPCHK(c3::launch_zero(st, ctx->xi_bins.p, (int64_t)(nbin * 8)));
    }
    {
        KTimer kt(ctx, K_NOISE, st);
        HIPCHK(c3::launch_xi_white(st, mixed, (const int4 *)P->sample_tiles.p, P->nsample_tiles, lay->seg_off, d,
                                   d_dtype == TOD_F64, t, gain, ncorr, (double *)ctx->xi_part.p));
    }
    c3::FftArgs a = fft_args(ctx, P, lay);
    a.mode = 4;  // periodogram bins: forward passes only
    a.in_a = ncorr;
    a.in_a_f64 = !mixed;
    a.bins = (double *)ctx->xi_bins.p;
    if ((r = run_fft(ctx, st, P, mixed, a, 2)) != TOD_OK) return r;
    {
        KTimer kt(ctx, K_NOISE, st);
        HIPCHK(c3::launch_xi_sample(st, lay->nseg, (const SegInfo *)P->segs.p, (const FftPlan *)P->plans.p,
                                    lay->seg_band, (const double *)P->fsamp.p,
                                    (const int2 *)P->sample_seg_tiles.p, (const double *)ctx->xi_part.p,
                                    (const double *)ctx->xi_bins.p, fknee_in, ctx->d_seed_iter, mean_only,
                                    sigma0_out, fknee_out, alpha_out));
    }
    return TOD_OK;
}

tod_status bin_tod(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const int32_t *pix,
                   const uint16_t *psi, const void *d, tod_dtype d_dtype, const void *ncorr,
                   const double *gain, const double *sigma0, double *acc, int accumulate) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!pix || !psi || !d || !gain || !sigma0 || !acc) return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    const int4 *tiles;
    const int2 *runs;
    int nt;
    if ((r = get_bin_runs(ctx, lay, P, pix, &tiles, &nt, &runs)) != TOD_OK) return r;
    const LayoutDev Ld = make_layout_dev(lay);
    HIPCHK(c3::launch_check_params(ctx->stream, Ld, sigma0, nullptr, nullptr, ctx->d_err));
    if (!accumulate) HIPCHK(c3::launch_zero(ctx->stream, acc, lay->npix_total * 10 * sizeof(double)));
    KTimer kt(ctx, K_BIN, ctx->stream);
    HIPCHK(c3::launch_bin_tiles(ctx->stream, Ld, mixed, tiles, nt, runs, pix, psi, d, d_dtype == TOD_F64, ncorr,
                                gain, sigma0, ctx->trig64.p, acc, ctx->d_err));
    return TOD_OK;
}

tod_status solve_maps(tod_ctx ctx, int64_t npix, const double *acc, double rcond_min,
                      void *map_out, tod_dtype map_dtype, double *rcond_out) {
    if (!ctx) return TOD_EINVAL;
    if (npix < 0 || !acc || !map_out) return fail(ctx, TOD_EINVAL, "bad argument");
    if (map_dtype != TOD_F32 && map_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad map dtype");
    KTimer kt(ctx, K_SOLVE, ctx->stream);
    HIPCHK(c3::launch_solve(ctx->stream, npix, acc, rcond_min, map_out, map_dtype == TOD_F64, rcond_out));
    return TOD_OK;
}

static tod_status chisq_common(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const int32_t *pix,
                               const uint16_t *psi, const void *d, tod_dtype d_dtype,
                               const void *ncorr, const void *maps, const double *gain,
                               const double *sigma0, const double *fknee, const double *alpha,
                               double gscale, const double *gscale_dev, double *grad_maps, double *chisq_seg,
                               double *grad_gain, double *gsig, double *gfk, double *galpha) {
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (!pix || !psi || !d || !ncorr || !maps || !gain || !sigma0 || !fknee || !alpha)
        return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    const int4 *tiles;
    int nt;
    if ((r = get_bin_tiles(ctx, lay, P, pix, &tiles, &nt)) != TOD_OK) return r;
    const size_t ssz = sizeof(double) * 4 * (size_t)std::max(1, lay->nseg);
    HIPCHK(ctx->seg_sums.ensure(ssz));
    HIPCHK(ctx->seg_whittle.ensure(ssz));
    hipStream_t st = ctx->stream;
    HIPCHK(c3::launch_zero(st, ctx->seg_sums.p, ssz));
    HIPCHK(c3::launch_zero(st, ctx->seg_whittle.p, ssz));
    if (grad_maps) {
        HIPCHK(ctx->gmap4.ensure(sizeof(double) * 4 * (size_t)std::max<int64_t>(1, lay->npix_total)));
        HIPCHK(c3::launch_zero(st, ctx->gmap4.p, sizeof(double) * 4 * lay->npix_total));
    }
    if (gsig) HIPCHK(c3::launch_zero(st, gsig, sizeof(double) * lay->ndet));
    if (gfk) HIPCHK(c3::launch_zero(st, gfk, sizeof(double) * lay->ndet));
    if (galpha) HIPCHK(c3::launch_zero(st, galpha, sizeof(double) * lay->ndet));
    HIPCHK(ctx->maps4.ensure((size_t)lay->npix_total * 4 * (mixed ? 4 : 8)));
    const LayoutDev Ld = make_layout_dev(lay);
    HIPCHK(c3::launch_check_params(st, Ld, sigma0, fknee, alpha, ctx->d_err));
    {
        KTimer kt(ctx, K_CHISQ, st);
        double *g4 = grad_maps ? (double *)ctx->gmap4.p : nullptr;
        HIPCHK(c3::launch_chisq_time_tiles(st, Ld, mixed, tiles, nt, pix, psi, d, d_dtype == TOD_F64,
                                           ncorr, maps, ctx->maps4.p, gain, sigma0, ctx->trig64.p,
                                           (double *)ctx->seg_sums.p, g4, gscale, gscale_dev));
        if (grad_maps) HIPCHK(c3::launch_gmap_out(st, lay->npix_total, g4, grad_maps));
    }
    c3::FftArgs a = fft_args(ctx, P, lay);
    a.in_a = ncorr;
    a.in_a_f64 = !mixed;
    a.in_b = nullptr;
    a.sigma0 = sigma0;
    a.fknee = fknee;
    a.alpha = alpha;
    a.mode = 1;
    a.whittle = (double *)ctx->seg_whittle.p;
    {
        tod_status rr = run_fft(ctx, st, P, mixed, a, 2);
        if (rr != TOD_OK) return rr;
    }
    HIPCHK(c3::launch_chisq_finish(st, Ld, (const double *)ctx->seg_sums.p,
                                   (const double *)ctx->seg_whittle.p, gain, sigma0, fknee, alpha,
                                   gscale, gscale_dev, chisq_seg, grad_gain, gsig, gfk, galpha));
    return TOD_OK;
}

tod_status tod_chisq(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const int32_t *pix,
                     const uint16_t *psi, const void *d, tod_dtype d_dtype, const void *ncorr,
                     const void *maps, const double *gain, const double *sigma0,
                     const double *fknee, const double *alpha, double *chisq_seg) {
    if (!ctx) return TOD_EINVAL;
    if (!chisq_seg) return fail(ctx, TOD_EINVAL, "NULL chisq_seg");
    return chisq_common(ctx, lay, prec, pix, psi, d, d_dtype, ncorr, maps, gain, sigma0, fknee, alpha,
                        1.0, nullptr, nullptr, chisq_seg, nullptr, nullptr, nullptr, nullptr);
}

tod_status tod_chisq_backward(tod_ctx ctx, const tod_layout *lay, tod_prec prec,
                              const int32_t *pix, const uint16_t *psi, const void *d,
                              tod_dtype d_dtype, const void *ncorr, const void *maps,
                              const double *gain, const double *sigma0, const double *fknee,
                              const double *alpha, double grad_scale, const double *grad_scale_dev,
                              double *grad_maps,
                              double *grad_gain, double *grad_sigma0, double *grad_fknee,
                              double *grad_alpha) {
    if (!ctx) return TOD_EINVAL;
    return chisq_common(ctx, lay, prec, pix, psi, d, d_dtype, ncorr, maps, gain, sigma0, fknee, alpha,
                        grad_scale, grad_scale_dev, grad_maps, nullptr, grad_gain, grad_sigma0, grad_fknee,
                        grad_alpha);
}

// The fused sweep; with tod != NULL the TOD comes from its compressed stream,
// decoded into d_work (the precision's type) right after the pointing.
static tod_status sweep_impl(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const tod_huff *pix,
                             const tod_huff *psi, const tod_huff *tod, double quantum, void *d_work,
                             const void *d, tod_dtype d_dtype, const void *maps, const double *gain,
                             const double *sigma0, const double *fknee, const double *alpha, uint64_t seed,
                             uint64_t iter, void *ncorr_out, double *acc, int32_t *pix_work,
                             uint16_t *psi_work, int use_graph) {
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if ((r = check_huff(ctx, pix, "pix")) != TOD_OK) return r;
    if ((r = check_huff(ctx, psi, "psi")) != TOD_OK) return r;
    if (pix->chunk_len != psi->chunk_len) return fail(ctx, TOD_EINVAL, "pix and psi chunk_len differ");
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (d_dtype != TOD_F32 && d_dtype != TOD_F64) return fail(ctx, TOD_EINVAL, "bad d dtype");
    if (tod) {
        if ((r = check_huff(ctx, tod, "tod")) != TOD_OK) return r;
        if (!(quantum > 0.0)) return fail(ctx, TOD_EINVAL, "quantum must be > 0");
        if (!d_work) return fail(ctx, TOD_EINVAL, "NULL d_work");
        d = d_work;
        d_dtype = prec == TOD_MIXED ? TOD_F32 : TOD_F64;
    }
    if (!d || !maps || !gain || !sigma0 || !fknee || !alpha || !ncorr_out || !acc || !pix_work || !psi_work)
        return fail(ctx, TOD_EINVAL, "NULL argument");
    const int mixed = prec == TOD_MIXED;
    Plan *P;
    if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
    if ((r = ensure_work(ctx, P)) != TOD_OK) return r;
    const size_t rsz = (size_t)lay->nsamp * (mixed ? 4 : 8);
    HIPCHK(ctx->resid.ensure(rsz + 64));
    const DecodeTask *dt;
    int ndt;
    if ((r = get_decode_tasks(ctx, P, pix->chunk_len, &dt, &ndt)) != TOD_OK) return r;
    HIPCHK(ctx->dec_tabs.ensure(sizeof(DecTab) * (size_t)(pix->ntable + psi->ntable)));
    const DecodeTask *dtt = nullptr;
    int ndtt = 0;
    if (tod) {
        if ((r = get_decode_tasks(ctx, P, tod->chunk_len, &dtt, &ndtt)) != TOD_OK) return r;
        HIPCHK(ctx->dec_tabs2.ensure(sizeof(DecTab) * (size_t)tod->ntable));
    }
    HIPCHK(ctx->maps4.ensure((size_t)lay->npix_total * 4 * (mixed ? 4 : 8)));
    hipStream_t st = ctx->stream;
    const LayoutDev Ld = make_layout_dev(lay);
    if (P->nbin > 0) {
        // tiles exist: rebuild them if a band's stride or the run length has
        // been set or tuned since (no probe: the pointing of this call is not
        // decoded yet)
        const int4 *t0;
        const int2 *r0;
        int n0;
        if ((r = get_bin_runs(ctx, lay, P, nullptr, &t0, &n0, &r0)) != TOD_OK) return r;
    }

    // graph key: every pointer and size the captured kernels bake in -- the
    // layout and stream structs as the kernels receive them, the caller's
    // buffers, the context's scratch and the plan (its generation changes
    // whenever its task lists or tiles are rebuilt)
    const HuffDev Hp = make_huff_dev(pix), Hs = make_huff_dev(psi);
    HuffDev Ht;
    memset(&Ht, 0, sizeof(Ht));
    if (tod) Ht = make_huff_dev(tod);
    uint64_t gk = 1469598103934665603ull;
    gk = fnv(gk, &Ld, sizeof(Ld));
    gk = fnv(gk, &Hp, sizeof(Hp));
    gk = fnv(gk, &Hs, sizeof(Hs));
    gk = fnv(gk, &Ht, sizeof(Ht));
    gk = fnv(gk, &quantum, sizeof(quantum));
    const void *ptrs[] = {d, maps, gain, sigma0, fknee, alpha, ncorr_out, acc, pix_work, psi_work,
                          ctx->work.p, ctx->resid.p, ctx->dec_tabs.p, ctx->maps4.p, ctx->trig32.p,
                          ctx->trig64.p, ctx->d_err, ctx->d_seed_iter, dt, P->bin_tiles.p, P->run_tiles.p,
                          P->run_segs.p, ctx->dec_tabs2.p, dtt};
    gk = fnv(gk, ptrs, sizeof(ptrs));
    gk = fnv(gk, &ndt, sizeof(ndt));
    gk = fnv(gk, &P->key, sizeof(P->key));
    gk = fnv(gk, &P->gen, sizeof(P->gen));
    gk = fnv(gk, &d_dtype, sizeof(d_dtype));
    gk = fnv(gk, &mixed, sizeof(mixed));

    HIPCHK(c3::launch_set_u64(st, ctx->d_seed_iter, seed, iter));
    const bool have_tiles = P->nbin > 0;
    if (use_graph && have_tiles) {
        auto it = ctx->graphs.find(gk);
        if (it != ctx->graphs.end()) {
            HIPCHK(hipGraphLaunch(it->second.ex, st));
            return TOD_OK;
        }
    }
    // eager (or capture) sequence
    auto run = [&](bool capture) -> tod_status {
        HIPCHK(c3::launch_check_params(st, Ld, sigma0, fknee, alpha, ctx->d_err));
        {
            KTimer kt(ctx, K_DECODE, st);
            HIPCHK(c3::launch_decode(st, Ld, make_huff_dev(pix), make_huff_dev(psi),
                                     (DecTab *)ctx->dec_tabs.p, dt, ndt, pix_work, psi_work,
                                     ctx->d_err));
        }
        if (tod) {  // d = quantum x (the undifferenced integers), bit-exact as decode_tod
            KTimer kt(ctx, K_DECODE, st);
            HIPCHK(c3::launch_decode_stream(st, Ld, Ht, (DecTab *)ctx->dec_tabs2.p, dtt, ndtt, mixed ? 0 : 1,
                                            quantum, 0, d_work, nullptr, ctx->d_err));
        }
        const int4 *tiles = (const int4 *)P->bin_tiles.p;
        int nt = P->nbin;
        const int4 *rtiles = (const int4 *)P->run_tiles.p;
        const int2 *runs = (const int2 *)P->run_segs.p;
        int nrt = P->nrun_tiles;
        if (!capture && !have_tiles) {
            tod_status rr = get_bin_runs(ctx, lay, P, pix_work, &rtiles, &nrt, &runs);
            if (rr != TOD_OK) return rr;
            tiles = (const int4 *)P->bin_tiles.p;
            nt = P->nbin;
        }
        {
            KTimer kt(ctx, K_PROJECT, st);
            HIPCHK(c3::launch_resid_tiles(st, Ld, mixed, tiles, nt, pix_work, psi_work, d,
                                          d_dtype == TOD_F64, maps, ctx->maps4.p, gain,
                                          mixed ? ctx->trig32.p : ctx->trig64.p, ctx->resid.p, ctx->d_err));
        }
        {
            c3::FftArgs a = fft_args(ctx, P, lay);
            a.in_a = ctx->resid.p;
            a.in_a_f64 = !mixed;
            a.in_b = nullptr;
            a.out = ncorr_out;
            a.sigma0 = sigma0;
            a.fknee = fknee;
            a.alpha = alpha;
            a.mean_only = 0;
            tod_status rr = run_fft(ctx, st, P, mixed, a, 3);
            if (rr != TOD_OK) return rr;
        }
        {
            HIPCHK(c3::launch_zero(st, acc, lay->npix_total * 10 * sizeof(double)));
            KTimer kt(ctx, K_BIN, st);
            HIPCHK(c3::launch_bin_tiles(st, Ld, mixed, rtiles, nrt, runs, pix_work, psi_work, d,
                                        d_dtype == TOD_F64, ncorr_out, gain, sigma0, ctx->trig64.p, acc,
                                        ctx->d_err));
        }
        return TOD_OK;
    };
    if (!(use_graph && have_tiles) || ctx->timing) return run(false);
    // capture on a context-owned stream (the caller's may be the null stream),
    // then launch the graph on the caller's stream
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    tod_ctx_s::GraphEntry ge;
    st = ctx->cap_stream;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    tod_status rr = run(true);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(st, &g);
    st = ctx->stream;
    if (rr != TOD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rr;
    }
    HIPCHK(e2);
    ge.g = g;
    HIPCHK(hipGraphInstantiate(&ge.ex, g, nullptr, nullptr, 0));
    ctx->graphs[gk] = ge;
    HIPCHK(hipGraphLaunch(ge.ex, st));
    return TOD_OK;
}

tod_status tod_sweep(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const tod_huff *pix,
                     const tod_huff *psi, const void *d, tod_dtype d_dtype, const void *maps,
                     const double *gain, const double *sigma0, const double *fknee,
                     const double *alpha, uint64_t seed, uint64_t iter, void *ncorr_out,
                     double *acc, int32_t *pix_work, uint16_t *psi_work, int use_graph) {
    if (!ctx) return TOD_EINVAL;
    return sweep_impl(ctx, lay, prec, pix, psi, nullptr, 0.0, nullptr, d, d_dtype, maps, gain, sigma0, fknee,
                      alpha, seed, iter, ncorr_out, acc, pix_work, psi_work, use_graph);
}

tod_status tod_sweep_stream(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const tod_huff *pix,
                            const tod_huff *psi, const tod_huff *tod, double quantum, void *d_work,
                            const void *maps, const double *gain, const double *sigma0,
                            const double *fknee, const double *alpha, uint64_t seed, uint64_t iter,
                            void *ncorr_out, double *acc, int32_t *pix_work, uint16_t *psi_work,
                            int use_graph) {
    if (!ctx) return TOD_EINVAL;
    if (!tod) return fail(ctx, TOD_EINVAL, "NULL tod stream");
    return sweep_impl(ctx, lay, prec, pix, psi, tod, quantum, d_work, nullptr, TOD_F32, maps, gain, sigma0,
                      fknee, alpha, seed, iter, ncorr_out, acc, pix_work, psi_work, use_graph);
}

tod_status tod_set_bin_stride(tod_ctx ctx, int32_t band, int32_t stride) {
    if (!ctx) return TOD_EINVAL;
    if (band < 0 || band >= C3_MAXBAND || stride < 0 || stride > c3tune::kMaxStride)
        return fail(ctx, TOD_EINVAL, "bad band/stride (stride must be in [0, 2^26])");
    if (stride == 0)
        ctx->band_stride.erase(band);
    else
        ctx->band_stride[band] = stride;
    return TOD_OK;
}

tod_status tod_set_bin_runs(tod_ctx ctx, int32_t scans) {
    if (!ctx) return TOD_EINVAL;
    if (scans < 0 || scans > 16) return fail(ctx, TOD_EINVAL, "scans per binning run must be in [0, 16]");
    ctx->bin_runs = scans;
    return TOD_OK;
}

tod_status tod_set_fft_batch(tod_ctx ctx, int64_t complex_elems) {
    if (!ctx) return TOD_EINVAL;
    if (complex_elems < 0) return fail(ctx, TOD_EINVAL, "negative batch size");
    ctx->fft_batch = complex_elems;
    return TOD_OK;
}

tod_status tod_enable_timing(tod_ctx ctx, int enable) {
    if (!ctx) return TOD_EINVAL;
    ctx->timing = enable != 0;
    return TOD_OK;
}

tod_status tod_kernel_times(tod_ctx ctx, double *total_ms, int32_t *launches) {
    if (!ctx || !total_ms || !launches) return TOD_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < K_NKERNEL; ++i) {
        total_ms[i] = 0;
        launches[i] = 0;
    }
    for (auto &r : ctx->recs) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        total_ms[r.kid] += ms;
        launches[r.kid] += 1;
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->recs.clear();
    return TOD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuning
namespace {

std::string band_key(const tod_band &b) {
    char buf[64];
    snprintf(buf, sizeof(buf), "%d:%.6g", b.nside, b.fsamp);
    return buf;
}

// Mean time (ms) of the three n_corr FFT passes for K segments of length M
// with the FFT split `ch`.
tod_status time_fft_choice(tod_ctx ctx, int mixed, int64_t M, const c3tune::FftChoice &ch, int K,
                           float *ms_out) {
    c3tune::Table saved = ctx->tuned;
    ctx->tuned.put(mixed, M, ch);
    std::vector<int64_t> off(K + 1);
    std::vector<int32_t> band(K, 0);
    for (int i = 0; i <= K; ++i) off[i] = (int64_t)i * M;
    tod_band b;
    b.nside = 1;
    b.npsi = 4096;
    b.npix = 12;
    b.pix_off = 0;
    b.fsamp = 1.0;
    tod_layout L;
    memset(&L, 0, sizeof(L));
    L.nseg = K;
    L.nband = 1;
    L.ndet = 1;
    L.nsamp = off[K];
    L.npix_total = 12;
    L.h_seg_off = off.data();
    L.h_seg_band = band.data();
    L.bands = &b;
    const uint64_t key = layout_key(&L, mixed, 0x7475ull ^ ctx->tuned.version);
    Plan *P = nullptr;
    tod_status r = build_plan(ctx, &L, mixed, key, &P);
    ctx->tuned = saved;
    if (r != TOD_OK) return r;
    r = ensure_work(ctx, P);
    if (r != TOD_OK) return r;
    const size_t esz = mixed ? 4 : 8;
    DevBuf din, dout, prm;
    HIPCHK(din.ensure(off[K] * esz));
    HIPCHK(dout.ensure(off[K] * esz));
    HIPCHK(prm.ensure(3 * K * sizeof(double)));
    std::vector<double> hp(3 * K);
    for (int i = 0; i < K; ++i) {
        hp[i] = 1.0;
        hp[K + i] = 0.1;
        hp[2 * K + i] = -1.5;
    }
    HIPCHK(hipMemcpy(prm.p, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c3::launch_zero(ctx->stream, din.p, off[K] * esz));
    c3::FftArgs a = fft_args(ctx, P, &L);
    a.in_a = din.p;
    a.in_a_f64 = !mixed;
    a.out = dout.p;
    a.sigma0 = (const double *)prm.p;
    a.fknee = (const double *)prm.p + K;
    a.alpha = (const double *)prm.p + 2 * K;
    {
        tod_status rr = run_fft(ctx, ctx->stream, P, mixed, a, 3);
        if (rr != TOD_OK) return rr;
    }
    HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));
    const int reps = 3;
    for (int i = 0; i < reps; ++i) {
        tod_status rr = run_fft(ctx, ctx->stream, P, mixed, a, 3);
        if (rr != TOD_OK) return rr;
    }
    HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[3]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
    *ms_out = ms / reps;
    ctx->plans.erase(key);
    return TOD_OK;
}

}  // namespace

extern "C" {

tod_status tod_load_tuning(tod_ctx ctx, const char *cache_path) {
    if (!ctx) return TOD_EINVAL;
    if (!cache_path) return fail(ctx, TOD_EINVAL, "NULL path");
    FILE *f = fopen(cache_path, "rb");
    if (!f) return TOD_OK;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    fclose(f);
    std::map<std::string, int> strides;
    if (!c3tune::from_json(s, ctx->tuned, strides)) return fail(ctx, TOD_EINVAL, "unreadable tuning cache");
    for (auto &kv : strides) ctx->stride_by_key[kv.first] = kv.second;
    return TOD_OK;
}

tod_status tod_autotune(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const int32_t *pix,
                        const char *cache_path) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    const int mixed = prec == TOD_MIXED;
    if (cache_path) {
        if ((r = tod_load_tuning(ctx, cache_path)) != TOD_OK) return r;
    }
    std::map<int64_t, int> count;
    for (int s = 0; s < lay->nseg; ++s) {
        const int64_t n = lay->h_seg_off[s + 1] - lay->h_seg_off[s];
        if (n > 0) count[next_5smooth(n)]++;
    }
    for (auto &kv : count) {
        const int64_t M = kv.first;
        c3tune::FftChoice have;
        if (ctx->tuned.get(mixed, M, have)) continue;
        const int K = (int)std::max<int64_t>(2, std::min<int64_t>(32, (int64_t)(64ll << 20) / (8 * M)));
        // each candidate's time is the better of two measurements, and a
        // later candidate must beat the best so far by 3 %: near-equal
        // splits would otherwise trade places from run to run on timing
        // noise, and with them the kernels a sweep launches
        float best = 1e30f;
        c3tune::FftChoice bc;
        for (const c3tune::FftChoice &c : c3tune::candidates(M, mixed)) {
            float ms, ms2;
            if ((r = time_fft_choice(ctx, mixed, M, c, K, &ms)) != TOD_OK) return r;
            if ((r = time_fft_choice(ctx, mixed, M, c, K, &ms2)) != TOD_OK) return r;
            ms = std::min(ms, ms2);
            if (ms < 0.97f * best) {
                best = ms;
                bc = c;
            }
        }
        if (best < 1e30f) ctx->tuned.put(mixed, M, bc);
    }
    if (pix) {
        Plan *P;
        if ((r = get_plan(ctx, lay, mixed, &P)) != TOD_OK) return r;
        for (int b = 0; b < lay->nband; ++b) {
            int st = 0;
            if ((r = probe_stride(ctx, lay, P, pix, b, &st)) != TOD_OK) return r;
            ctx->band_stride[b] = st;
            ctx->stride_by_key[band_key(lay->bands[b])] = st;
        }
    }
    if (cache_path) {
        FILE *f = fopen(cache_path, "wb");
        if (!f) return fail(ctx, TOD_EINVAL, std::string("cannot write ") + cache_path);
        const std::string js = c3tune::to_json(ctx->tuned, ctx->stride_by_key);
        fwrite(js.data(), 1, js.size(), f);
        fclose(f);
    }
    return TOD_OK;
}

tod_status tod_plan(tod_ctx ctx, const tod_layout *lay, tod_prec prec, const char *tune_cache) {
    if (!ctx) return TOD_EINVAL;
    tod_status r;
    if ((r = check_layout(ctx, lay)) != TOD_OK) return r;
    if (prec != TOD_MIXED && prec != TOD_PLAIN_FP64) return fail(ctx, TOD_EINVAL, "bad precision");
    if (tune_cache && (r = tod_load_tuning(ctx, tune_cache)) != TOD_OK) return r;
    Plan *P;
    if ((r = get_plan(ctx, lay, prec == TOD_MIXED, &P)) != TOD_OK) return r;
    return ensure_work(ctx, P);
}

}  // extern "C"
