// Host-side validation of the layout and stream descriptions every entry
// point takes (the checks made before any device work is queued).  Host code
// only: it reads the host mirrors and the struct fields, never device memory.
#pragma once
#include <stdint.h>

#include <string>

#include "../../include/c3tod.h"

#define C3_MAXBAND_HOST 16   // bands a layout may have (C3_MAXBAND of the kernels)

namespace c3val {

inline tod_status err(std::string &msg, tod_status s, const std::string &m) {
    msg = m;
    return s;
}

inline tod_status check_layout(const tod_layout *L, std::string &msg) {
    if (!L) return err(msg, TOD_EINVAL, "layout is NULL");
    if (L->nseg < 0 || L->nband < 1 || L->nband > C3_MAXBAND_HOST || L->ndet < 1)
        return err(msg, TOD_EINVAL, "nseg/nband/ndet out of range");
    if (!L->seg_off || !L->seg_band || !L->seg_det || !L->h_seg_off || !L->h_seg_band || !L->bands)
        return err(msg, TOD_EINVAL, "layout has a NULL array");
    if (L->h_seg_off[0] != 0) return err(msg, TOD_EINVAL, "seg_off[0] != 0");
    for (int s = 0; s < L->nseg; ++s) {
        // compared before subtracting: from seg_off[0] = 0 up, every offset is
        // then >= 0 and the difference cannot overflow
        if (L->h_seg_off[s + 1] < L->h_seg_off[s]) return err(msg, TOD_EINVAL, "seg_off is not non-decreasing");
        const int64_t n = L->h_seg_off[s + 1] - L->h_seg_off[s];
        // the strided kernels step t + 4 S with t, S <= n in 32-bit arithmetic
        if (n > (1 << 28)) return err(msg, TOD_ENOTSUP, "segment longer than 2^28 samples");
        if (L->h_seg_band[s] < 0 || L->h_seg_band[s] >= L->nband)
            return err(msg, TOD_EINVAL, "seg_band out of range");
    }
    if (L->h_seg_off[L->nseg] != L->nsamp) return err(msg, TOD_EINVAL, "nsamp != seg_off[nseg]");
    int64_t off = 0;
    for (int b = 0; b < L->nband; ++b) {
        const tod_band &B = L->bands[b];
        if (B.npsi != 4096) return err(msg, TOD_EINVAL, "npsi must be 4096");
        // pixel indices are 32-bit on the device: nside <= 8192 (12 nside^2 < 2^31)
        if (B.nside < 1 || B.nside > 8192) return err(msg, TOD_EINVAL, "nside must be in [1, 8192]");
        if (B.npix != 12ll * B.nside * B.nside) return err(msg, TOD_EINVAL, "npix != 12 nside^2");
        if (B.pix_off != off) return err(msg, TOD_EINVAL, "band pix_off not contiguous");
        if (!(B.fsamp > 0)) return err(msg, TOD_EINVAL, "fsamp must be > 0");
        off += B.npix;
    }
    if (off != L->npix_total) return err(msg, TOD_EINVAL, "npix_total != sum of band npix");
    return TOD_OK;
}

inline tod_status check_huff(const tod_huff *h, const char *what, std::string &msg) {
    if (!h || !h->words || !h->seg_word_off || !h->seg_table || !h->tables || !h->table_off ||
        !h->chunk_bit || !h->chunk_prev || !h->seg_chunk_off)
        return err(msg, TOD_EINVAL, std::string(what) + " stream has a NULL array");
    if (h->chunk_len < 32 || h->chunk_len > 4096 || (h->chunk_len % 32))
        return err(msg, TOD_EINVAL, std::string(what) + " chunk_len must be a multiple of 32 in [32, 4096]");
    if (h->ntable < 1) return err(msg, TOD_EINVAL, std::string(what) + " has no tables");
    return TOD_OK;
}

}  // namespace c3val
