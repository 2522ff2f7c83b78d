// Launch schedules of the apply kernels.  See schedule.hpp.
#include "schedule.hpp"

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>

namespace napspmv {

void row_blocks(const int32_t *rowptr, int64_t n, int cap, int max_rows,
                std::vector<int32_t> &rowblk, std::vector<int32_t> &blkptr) {
    rowblk.clear();
    blkptr.clear();
    int64_t r = 0;
    while (r < n) {
        rowblk.push_back((int32_t)r);
        blkptr.push_back(rowptr[r]);
        const int64_t start = r;
        if (rowptr[r + 1] - rowptr[r] > cap) {
            ++r;                                   // a long row alone
            continue;
        }
        while (r < n && r - start < max_rows && rowptr[r + 1] - rowptr[start] <= cap) ++r;
    }
    rowblk.push_back((int32_t)n);
    blkptr.push_back(rowptr[n]);
}

void row_blocks_per_process(const int32_t *rowptr, const std::vector<int64_t> &starts, int cap,
                            int max_rows, std::vector<int32_t> &rowblk,
                            std::vector<int32_t> &blkptr) {
    rowblk.clear();
    blkptr.clear();
    const int64_t n_p = (int64_t)starts.size() - 1;
    std::vector<int32_t> rb, bp;
    for (int64_t t = 0; t < n_p; ++t) {
        const int64_t r0 = starts[t], r1 = starts[t + 1];
        row_blocks(rowptr + r0, r1 - r0, cap, max_rows, rb, bp);
        for (size_t b = 0; b + 1 < rb.size(); ++b) {
            rowblk.push_back(rb[b] + (int32_t)r0);
            blkptr.push_back(bp[b]);
        }
    }
    rowblk.push_back((int32_t)starts[n_p]);
    blkptr.push_back(rowptr[starts[n_p]]);
}

void sort_blocks(const std::vector<int32_t> &blkptr, int cap, const int32_t *col,
                 const uint8_t *val, int vs, int32_t *col_out, uint8_t *val_out,
                 uint16_t *slot_out, int run, const uint8_t *keep) {
    const int64_t nb = (int64_t)blkptr.size() - 1;
#pragma omp parallel
    {
        std::vector<int32_t> ord, at;
#pragma omp for schedule(dynamic, 64)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t k0 = blkptr[b], len = blkptr[b + 1] - k0;
            ord.resize((size_t)len);
            std::iota(ord.begin(), ord.end(), 0);
            const int64_t a = k0 & -(int64_t)run, lo = k0 - a, hi = lo + len;
            const bool tiled = run > 1 && cap % (run * kLanes) == 0 && hi <= cap;
            const bool sorted = len <= cap && !(keep && keep[b]) && (run == 1 || tiled);
            if (sorted)
                std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
                    return col[k0 + x] < col[k0 + y];
                });
            // at[q]: the position, from k0, of the q-th entry of gather order
            at.resize((size_t)len);
            if (sorted && tiled) {
                int64_t q = 0;
                for (int u = 0; u < cap / (run * kLanes); ++u)
                    for (int j = 0; j < run; ++j)
                        for (int t = 0; t < kLanes; ++t) {
                            const int64_t d = run_offset(run, u, t, j);
                            if (d >= lo && d < hi) at[(size_t)q++] = (int32_t)(d - lo);
                        }
            } else {
                std::iota(at.begin(), at.end(), 0);
            }
            for (int64_t q = 0; q < len; ++q) {
                const int64_t from = k0 + ord[q], to = k0 + at[q];
                col_out[to] = col[from];
                std::memcpy(val_out + to * vs, val + from * vs, (size_t)vs);
                slot_out[to] = (uint16_t)(sorted ? ord[q] : 0);
            }
        }
    }
}

bool pack_block(int64_t k0, int64_t k1, int cap, int run, const int32_t *pos,
                const uint16_t *slot, uint32_t *word, int32_t *base) {
    const int64_t a = k0 & -(int64_t)run;
    if (run < 1 || cap % (run * kLanes) != 0 || k1 - a > cap || cap > (1 << kPackSlotBits))
        return false;
    const int nbase = cap / kPackLanes;
    std::vector<int32_t> lo((size_t)nbase, INT32_MAX), hi((size_t)nbase, -1);
    for (int u = 0; u < cap / (run * kLanes); ++u)
        for (int t = 0; t < kLanes; ++t)
            for (int j = 0; j < run; ++j) {
                const int64_t k = a + run_offset(run, u, t, j);
                if (k < k0 || k >= k1) continue;
                const int32_t i = pack_base_index(cap, run, u, t, j);
                lo[(size_t)i] = std::min(lo[(size_t)i], pos[k]);
                hi[(size_t)i] = std::max(hi[(size_t)i], pos[k]);
            }
    for (int i = 0; i < nbase; ++i)
        if (hi[(size_t)i] >= 0 && (int64_t)hi[(size_t)i] - lo[(size_t)i] >= (int64_t(1) << kPackPosBits))
            return false;
    for (int i = 0; i < nbase; ++i) base[i] = hi[(size_t)i] >= 0 ? lo[(size_t)i] : 0;
    for (int u = 0; u < cap / (run * kLanes); ++u)
        for (int t = 0; t < kLanes; ++t)
            for (int j = 0; j < run; ++j) {
                const int64_t k = a + run_offset(run, u, t, j);
                if (k < k0 || k >= k1) continue;
                const int32_t i = pack_base_index(cap, run, u, t, j);
                word[k] = ((uint32_t)slot[k] << kPackPosBits) | (uint32_t)(pos[k] - base[i]);
            }
    return true;
}

void row_block_windows(const std::vector<int32_t> &rowblk, const std::vector<int32_t> &on_lo,
                       const std::vector<int32_t> &on_hi, int64_t n, int window,
                       std::vector<int32_t> &win) {
    const int64_t nb = (int64_t)rowblk.size() - 1;
    win.assign(2 * nb, 0);
    for (int64_t b = 0; b < nb; ++b) {
        int64_t lo = INT64_MAX, hi = -1;
        for (int64_t r = rowblk[b]; r < rowblk[b + 1]; ++r) {
            if (on_lo[r] <= on_hi[r]) {
                lo = std::min<int64_t>(lo, on_lo[r]);
                hi = std::max<int64_t>(hi, on_hi[r]);
            }
        }
        int64_t s = 0, len = 0;
        if (hi >= lo) {
            if (hi - lo + 1 <= window) {
                s = lo;
                len = hi - lo + 1;
            } else {
                s = std::min(std::max<int64_t>(((int64_t)rowblk[b] + rowblk[b + 1]) / 2 - window / 2, lo),
                             hi - window + 1);
                len = window;
            }
        }
        s = std::max<int64_t>(0, std::min<int64_t>(s, n - len));
        win[2 * b] = (int32_t)s;
        win[2 * b + 1] = (int32_t)len;
    }
}

void merge_tasks(int64_t n_items, int64_t n_blocks, std::vector<int32_t> &tasks, int64_t tail) {
    tasks.clear();
    tasks.reserve((size_t)(n_items + n_blocks));
    // the launch's XCD ranges (see xcd_block): 8 contiguous stretches of the
    // task list, each dispatched in order on one XCD
    const int64_t n = n_items + n_blocks, q = n / 8, r = n % 8;
    int64_t i = 0, b = 0, start = 0;
    for (int64_t x = 0; x < 8 && n > 0; ++x) {
        const int64_t len = q + (x < r ? 1 : 0);
        const int64_t ni = n_items * (start + len) / n - i;     // this range's share of items
        // items go in proportion over the range but the last `tail` tasks,
        // so that no item (several times a row block's bytes) is left
        // running alone at the end of the launch
        const int64_t span = std::max(ni, len - tail), sb = span - ni;
        int64_t il = 0, bl = 0;
        for (int64_t s = 0; s < len; ++s) {
            if (il < ni && (bl >= sb || il * sb <= bl * ni))
                tasks.push_back(~(int32_t)(i + il++));
            else
                tasks.push_back((int32_t)(b + bl++));
        }
        i += ni;
        b += bl;
        start += len;
    }
}

void flat_items(int64_t total, int max_len, std::vector<int32_t> &items) {
    items.clear();
    for (int64_t a = 0; a < total; a += max_len) {
        items.push_back((int32_t)a);
        items.push_back((int32_t)std::min<int64_t>(max_len, total - a));
    }
}

}  // namespace napspmv
