// Host checks of the launch schedules (paper_1612_08060_amd/csrc/schedule.cpp):
// every task, row block and sorted entry is accounted for exactly once, and
// each schedule keeps the properties the kernels rely on.  Prints "ok" and
// returns 0, or prints the first failure and returns 1.
#include "schedule.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

static int fail(const char *what, long long a, long long b) {
    std::printf("FAIL %s (%lld, %lld)\n", what, a, b);
    return 1;
}

static int check_merge(int64_t tail) {
    for (int64_t ni = 0; ni < 400; ni += 13)
        for (int64_t nb = 0; nb < 6000; nb += 41) {
            std::vector<int32_t> t;
            napspmv::merge_tasks(ni, nb, t, tail);
            if ((int64_t)t.size() != ni + nb) return fail("merge size", ni, nb);
            int64_t ei = 0, eb = 0;
            for (int32_t x : t) {
                if (x < 0) {
                    if (~x != ei++) return fail("item order", ni, nb);
                } else if (x != eb++) {
                    return fail("block order", ni, nb);
                }
            }
            if (ei != ni || eb != nb) return fail("merge counts", ni, nb);
            // the XCD ranges of the launch (xcd_block): proportional shares,
            // and no item in a range's last `tail` tasks unless the items
            // do not fit before them (then they lead the range)
            const int64_t n = ni + nb, q = n / 8, r = n % 8;
            int64_t start = 0, seen = 0;
            for (int64_t x = 0; x < 8; ++x) {
                const int64_t len = q + (x < r ? 1 : 0);
                const int64_t share = (n ? ni * (start + len) / n : 0) - seen;
                int64_t cnt = 0, last = -1;
                for (int64_t s = 0; s < len; ++s)
                    if (t[start + s] < 0) { ++cnt; last = s; }
                if (cnt != share) return fail("range share", x, cnt);
                const int64_t limit = std::max(share, len - tail);
                if (last >= limit) return fail("item in the tail", x, last);
                seen += cnt;
                start += len;
            }
        }
    return 0;
}

// Gather-order sort of the blocks `bp` of a random column pattern: every
// block of at most `cap` entries holds a permutation of its entries with
// slots pointing at their stored positions; read in the order the kernel's
// load instructions visit positions (plain order, or for a run layout the
// order of run_offset restricted to the block), columns ascend; longer
// blocks, and with `with_keep` a random third of the blocks flagged to
// keep their order, stay in stored order with slot 0.
static int check_sort(std::mt19937 &rng, const std::vector<int32_t> &rowptr,
                      const std::vector<int32_t> &bp, int cap, int run, int trial,
                      bool with_keep = false) {
    const int nnz = rowptr.back();
    std::vector<int32_t> col(nnz), col_out(nnz);
    std::vector<double> val(nnz), val_out(nnz);
    std::vector<uint16_t> slot(nnz);
    for (int k = 0; k < nnz; ++k) { col[k] = (int32_t)(rng() % 1000); val[k] = k + 0.5; }
    std::vector<uint8_t> keep(bp.size(), 0);
    if (with_keep)
        for (auto &f : keep) f = rng() % 3 == 0;
    napspmv::sort_blocks(bp, cap, col.data(), reinterpret_cast<const uint8_t *>(val.data()), 8,
                         col_out.data(), reinterpret_cast<uint8_t *>(val_out.data()), slot.data(),
                         run, with_keep ? keep.data() : nullptr);
    int64_t tiled = 0;
    for (size_t b = 0; b + 1 < bp.size(); ++b) {
        const int32_t k0 = bp[b], len = bp[b + 1] - k0;
        if (len > cap || keep[b]) {
            for (int32_t q = 0; q < len; ++q)
                if (slot[k0 + q] != 0 || col_out[k0 + q] != col[k0 + q] ||
                    val_out[k0 + q] != val[k0 + q])
                    return fail("long block moved", trial, q);
            continue;
        }
        // positions in load order
        std::vector<int32_t> order;
        const int32_t a = k0 & -run;
        if (run > 1 && !(cap % (run * napspmv::kLanes) == 0 && k0 - a + len <= cap)) {
            // a single row whose aligned span does not fit: stored order
            for (int32_t q = 0; q < len; ++q)
                if (slot[k0 + q] != 0 || col_out[k0 + q] != col[k0 + q] ||
                    val_out[k0 + q] != val[k0 + q])
                    return fail("unfit run block moved", trial, q);
            continue;
        }
        if (run > 1) {
            ++tiled;
            for (int u = 0; u < cap / (run * napspmv::kLanes); ++u)
                for (int j = 0; j < run; ++j)
                    for (int t = 0; t < napspmv::kLanes; ++t) {
                        const int32_t k = a + napspmv::run_offset(run, u, t, j);
                        if (k >= k0 && k < k0 + len) order.push_back(k);
                    }
        } else {
            for (int32_t q = 0; q < len; ++q) order.push_back(k0 + q);
        }
        if ((int32_t)order.size() != len) return fail("load order size", trial, (long long)b);
        std::vector<char> hit(len, 0);
        for (int32_t q = 0; q < len; ++q) {
            const int32_t k = order[q];
            if (q && col_out[k] < col_out[order[q - 1]]) return fail("not sorted", trial, q);
            const int32_t from = slot[k];
            if (from >= len || hit[from]++) return fail("slot permutation", trial, q);
            if (col_out[k] != col[k0 + from] || val_out[k] != val[k0 + from])
                return fail("slot target", trial, q);
        }
    }
    if (run > 1 && !with_keep && tiled == 0) return fail("no block took the run layout", trial, run);
    return 0;
}

// The loads of the run kernels (local_product_runs, remote_product_runs):
// lane t's u-th vector starts at min(a + run_offset(run, u, t, 0), last
// aligned start) with a = k0 & -run.  Over blocks cut at cap - 7 entries,
// every loaded position lies in [0, nnz + 8) (the arrays' padding), the
// positions inside [k0, k1) are visited exactly once, and each lands at an
// LDS index below cap (its offset from a).
static int check_run_loads() {
    std::mt19937 rng(5);
    for (int trial = 0; trial < 40; ++trial) {
        const int n_p = 1 + trial % 5, n = n_p * (20 + trial * 7 % 60);
        std::vector<int32_t> rowptr(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            const int len = (rng() % 23 == 0) ? 1500 + rng() % 3000 : rng() % 40;
            rowptr[i + 1] = rowptr[i] + len;
        }
        const int nnz = rowptr[n];
        std::vector<int64_t> starts(n_p + 1);
        for (int t = 0; t <= n_p; ++t) starts[t] = (int64_t)n * t / n_p;
        for (int cap : {1024, 2048, 4096, 8192}) {
            std::vector<int32_t> rb, bp;
            napspmv::row_blocks_per_process(rowptr.data(), starts, cap - 7, 1024, rb, bp);
            for (int run : {2, 4, 8}) {
                if (cap < run * napspmv::kLanes) continue;
                for (size_t b = 0; b + 1 < bp.size(); ++b) {
                    const int32_t k0 = bp[b], k1 = bp[b + 1], a = k0 & -run;
                    const bool multi = rb[b + 1] - rb[b] > 1;
                    if (multi && k1 - a > cap) return fail("aligned span over cap", trial, (long long)b);
                    if (k1 == k0 || k1 - a > cap) continue;     // the one-entry-per-lane path
                    const int32_t last = (k1 - 1) & -run;
                    std::vector<char> seen(k1 - k0, 0);
                    for (int u = 0; u < cap / (run * napspmv::kLanes); ++u)
                        for (int t = 0; t < napspmv::kLanes; ++t) {
                            const int32_t e = std::min(a + napspmv::run_offset(run, u, t, 0), last);
                            if (e < 0 || e + run > nnz + 8) return fail("load outside the arrays", trial, e);
                            for (int j = 0; j < run; ++j) {
                                const int32_t k = a + napspmv::run_offset(run, u, t, j);
                                if (k < k0 || k >= k1) continue;
                                if (e != k - j) return fail("used entry from a clamped load", trial, k);
                                if (seen[k - k0]++) return fail("entry loaded twice", trial, k);
                                if (k - a >= cap) return fail("LDS index over cap", trial, k);
                            }
                        }
                    for (char c : seen)
                        if (!c) return fail("entry not loaded", trial, (long long)b);
                }
            }
        }
    }
    return 0;
}

// Packed words (pack_block): decoded the way remote_product_runs decodes
// them (lane t's base for load u * run + j at pack_base_index(cap, run, 0,
// t, 0) + (u * run + j) * pack_base_stride(run)), every entry of a packed
// block gives back its position and slot; a block with a lane group whose
// positions span 2^kPackPosBits or more, a block whose aligned span exceeds
// cap and a cap above 2^kPackSlotBits are refused with nothing written.
static int check_pack() {
    using namespace napspmv;
    std::mt19937 rng(11);
    for (int cap : {1024, 2048, 4096, 8192})
        for (int run : {2, 4, 8})
            for (int u = 0; u < cap / (run * kLanes); ++u)
                for (int t = 0; t < kLanes; ++t)
                    for (int j = 0; j < run; ++j)
                        if (pack_base_index(cap, run, 0, t, 0) + (u * run + j) * pack_base_stride(run) !=
                            pack_base_index(cap, run, u, t, j))
                            return fail("kernel base index", cap, t);
    int64_t packed = 0, refused = 0;
    for (int trial = 0; trial < 60; ++trial) {
        const int cap = 1024 << (trial % 4), run = 2 << (trial % 3);
        if (cap < run * kLanes) continue;
        const int n = 3000 + (int)(rng() % 4000);
        std::vector<int32_t> rowptr(n + 1, 0);
        for (int i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + (int32_t)(rng() % 30);
        const int nnz = rowptr[n];
        std::vector<int64_t> starts = {0, n / 3, n};
        std::vector<int32_t> rb, bp;
        row_blocks_per_process(rowptr.data(), starts, cap - 7, 1024, rb, bp);
        // positions: a few bands of a large buffer (packable), or, in every
        // third trial, some blocks spread over 2^22 (refused)
        std::vector<int32_t> col(nnz), pos(nnz);
        std::vector<double> val(nnz), val2(nnz);
        for (size_t b = 0; b + 1 < bp.size(); ++b) {
            const bool wide = trial % 3 == 2 && b % 2 == 1;
            for (int32_t k = bp[b]; k < bp[b + 1]; ++k) {
                col[k] = wide ? (int32_t)(rng() % (1u << 22))
                              : (int32_t)((rng() % 64) * 40000 + rng() % 9000);
                val[k] = k;
            }
        }
        std::vector<uint16_t> slot(nnz);
        sort_blocks(bp, cap, col.data(), reinterpret_cast<const uint8_t *>(val.data()), 8, pos.data(),
                    reinterpret_cast<uint8_t *>(val2.data()), slot.data(), run);
        std::vector<uint32_t> word(nnz, 0xdeadbeefu);
        std::vector<int32_t> base(cap / kPackLanes);
        for (size_t b = 0; b + 1 < bp.size(); ++b) {
            const int32_t k0 = bp[b], k1 = bp[b + 1], a = k0 & -run;
            if (k1 == k0) continue;
            int32_t span = 0;
            for (int u = 0; u < cap / (run * kLanes); ++u)
                for (int t = 0; t < kLanes; t += kPackLanes)
                    for (int j = 0; j < run; ++j) {
                        int32_t lo = INT32_MAX, hi = -1;
                        for (int l = t; l < t + kPackLanes; ++l) {
                            const int32_t k = a + run_offset(run, u, l, j);
                            if (k >= k0 && k < k1) { lo = std::min(lo, pos[k]); hi = std::max(hi, pos[k]); }
                        }
                        if (hi >= 0) span = std::max(span, hi - lo);
                    }
            std::fill(base.begin(), base.end(), -7);
            const bool fits = k1 - a <= cap;
            const bool ok = pack_block(k0, k1, cap, run, pos.data(), slot.data(), word.data(), base.data());
            if (ok != (fits && span < (1 << kPackPosBits))) return fail("pack decision", trial, (long long)b);
            if (!ok) {
                ++refused;
                for (int32_t k = k0; k < k1; ++k)
                    if (word[k] != 0xdeadbeefu) return fail("refused block written", trial, k);
                for (int32_t x : base)
                    if (x != -7) return fail("refused block wrote bases", trial, (long long)b);
                continue;
            }
            ++packed;
            for (int u = 0; u < cap / (run * kLanes); ++u)
                for (int t = 0; t < kLanes; ++t)
                    for (int j = 0; j < run; ++j) {
                        const int32_t k = a + run_offset(run, u, t, j);
                        if (k < k0 || k >= k1) continue;
                        const int32_t bi = pack_base_index(cap, run, 0, t, 0) + (u * run + j) * pack_base_stride(run);
                        const int32_t p = base[bi] + (int32_t)(word[k] & ((1u << kPackPosBits) - 1));
                        if (p != pos[k]) return fail("packed position", trial, k);
                        if ((word[k] >> kPackPosBits) != slot[k]) return fail("packed slot", trial, k);
                    }
        }
    }
    if (packed == 0 || refused == 0) return fail("pack cases", packed, refused);
    // a cap whose slots need more than kPackSlotBits bits
    std::vector<int32_t> pos(16, 1);
    std::vector<uint16_t> slot(16, 0);
    std::vector<uint32_t> word(16, 0);
    std::vector<int32_t> base(65536 / kPackLanes, 0);
    if (pack_block(0, 16, 65536, 2, pos.data(), slot.data(), word.data(), base.data()))
        return fail("cap over the slot bits packed", 0, 0);
    return 0;
}

static int check_blocks_and_sort() {
    std::mt19937 rng(7);
    for (int trial = 0; trial < 60; ++trial) {
        const int n_p = 1 + trial % 9, n = n_p * (5 + trial * 3 % 40);
        std::vector<int32_t> rowptr(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            // mostly short rows, a few longer than any block
            const int len = (rng() % 17 == 0) ? 300 + rng() % 200 : rng() % 30;
            rowptr[i + 1] = rowptr[i] + len;
        }
        std::vector<int64_t> starts(n_p + 1);
        for (int t = 0; t <= n_p; ++t) starts[t] = (int64_t)n * t / n_p;
        for (int cap : {64, 256}) {
            const int max_rows = 8;
            std::vector<int32_t> rb, bp;
            napspmv::row_blocks_per_process(rowptr.data(), starts, cap, max_rows, rb, bp);
            if (rb.front() != 0 || rb.back() != n) return fail("blocks cover", trial, cap);
            for (size_t b = 0; b + 1 < rb.size(); ++b) {
                const int32_t r0 = rb[b], r1 = rb[b + 1];
                if (r1 <= r0) return fail("empty block", trial, (long long)b);
                if (bp[b] != rowptr[r0]) return fail("block pointer", trial, (long long)b);
                const int64_t t = std::upper_bound(starts.begin(), starts.end(), r0) - starts.begin() - 1;
                if (r1 > starts[t + 1]) return fail("block spans processes", trial, (long long)b);
                const bool single = r1 - r0 == 1;
                if (!single && (rowptr[r1] - rowptr[r0] > cap || r1 - r0 > max_rows))
                    return fail("block too large", trial, (long long)b);
            }
            if (check_sort(rng, rowptr, bp, cap, 1, trial)) return 1;
        }
        // run layouts: blocks of at most cap - 7 entries, as the library
        // cuts them, so that a block of several rows has an aligned span
        // of at most cap
        for (int cap : {1024, 2048}) {
            std::vector<int32_t> rb, bp;
            napspmv::row_blocks_per_process(rowptr.data(), starts, cap - 7, 8, rb, bp);
            for (int run : {2, 4, 8})
                if (cap % (run * napspmv::kLanes) == 0 &&
                    (check_sort(rng, rowptr, bp, cap, run, trial) ||
                     check_sort(rng, rowptr, bp, cap, run, trial, true)))
                    return 1;
        }
        // single rows of cap - 6 .. cap entries: blocks whose aligned span
        // may exceed cap
        for (int cap : {1024, 2048}) {
            std::vector<int32_t> rp2(n + 1, 0);
            for (int i = 0; i < n; ++i)
                rp2[i + 1] = rp2[i] + (i % 7 == 3 ? cap - (int)(rng() % 7) : (int)(rng() % 30));
            std::vector<int32_t> rb, bp;
            napspmv::row_blocks_per_process(rp2.data(), starts, cap - 7, 8, rb, bp);
            for (int run : {2, 4})
                if (check_sort(rng, rp2, bp, cap, run, trial)) return 1;
        }
    }
    return 0;
}

// Saddle-point matrix [[H, B^T], [B, 0]] (H: n1 x n1 banded, B: m x n1, m < n1)
// with a process boundary at row n1: the B rows have no on-process entry, so
// their on-process row blocks are empty.  The runs of a non-empty block may
// load a neighbouring block's entries (another process's 16-bit column
// offsets), but every column the kernel uses to read v must be its own
// process's, so that a 16-bit offset from the block's process stays below
// n.  Returns the empty blocks seen.
static int check_saddle_loads(int64_t &empty_blocks) {
    empty_blocks = 0;
    std::mt19937 rng(11);
    for (int trial = 0; trial < 12; ++trial) {
        const int n1 = 96 + 32 * (trial % 3), m = 40 + 8 * (trial % 4), n = n1 + m;
        // processes: n1 split in 3, then the m B rows in 1 or 2
        std::vector<int64_t> starts = {0, n1 / 3, 2 * n1 / 3, n1};
        if (trial % 2) starts.push_back(n1 + m / 2);
        starts.push_back(n);
        auto owner = [&](int64_t j) {
            return (int64_t)(std::upper_bound(starts.begin(), starts.end(), j) - starts.begin()) - 1;
        };
        std::vector<std::vector<int32_t>> rows(n);
        for (int i = 0; i < n1; ++i) {
            for (int j = std::max(0, i - 3); j <= std::min(n1 - 1, i + 3); ++j) rows[i].push_back(j);
        }
        for (int q = 0; q < m; ++q) {
            for (int e = 0; e < 4; ++e) {
                const int j = (int)(rng() % n1);
                rows[n1 + q].push_back(j);          // B
                rows[j].push_back(n1 + q);          // B^T
            }
        }
        // on-process part in stored order
        std::vector<int32_t> rowptr(n + 1, 0), col;
        for (int i = 0; i < n; ++i) {
            for (int32_t j : rows[i])
                if (owner(j) == owner(i)) col.push_back(j);
            rowptr[i + 1] = (int32_t)col.size();
        }
        // the on-process product's loads: runs of E entries per lane
        // (product_runs), blocks cut at cap - 7 entries and 512 rows;
        // every column it uses to read v is the block's own (a loaded entry
        // outside the block is replaced by the process's first row)
        const int nnz = rowptr[n];
        for (int cap : {1024, 4096}) {
            std::vector<int32_t> rb, bp;
            napspmv::row_blocks_per_process(rowptr.data(), starts, cap - 7, 512, rb, bp);
            for (int run : {2, 4, 8}) {
                for (size_t b = 0; b + 1 < rb.size(); ++b) {
                    const int32_t k0 = bp[b], k1 = bp[b + 1], a = k0 & -run;
                    const int64_t t = owner(rb[b]);
                    if (k1 == k0) {
                        if (run == 2 && cap == 1024) ++empty_blocks;
                        continue;
                    }
                    if (k1 - a > cap) continue;     // a single long row, walked in chunks
                    const int32_t last = (k1 - 1) & -run;
                    for (int u = 0; u < cap / (run * napspmv::kLanes); ++u)
                        for (int l = 0; l < napspmv::kLanes; ++l) {
                            const int32_t e = std::min(a + napspmv::run_offset(run, u, l, 0), last);
                            if (e < 0 || e + run > nnz + 8) return fail("load outside the arrays", trial, e);
                            for (int j = 0; j < run; ++j) {
                                const int32_t k = a + napspmv::run_offset(run, u, l, j);
                                const bool used = k >= k0 && k < k1;
                                const int64_t c = used ? col[k] : starts[t];
                                if (used && owner(col[k]) != t)
                                    return fail("column outside the block's process", trial, k);
                                if (c < 0 || c >= n) return fail("v read outside v", trial, k);
                            }
                        }
                }
            }
        }
    }
    return 0;
}

int main() {
    int64_t empty = 0;
    if (check_merge(napspmv::kItemTail) || check_merge(napspmv::kPackScatterTail) ||
        check_blocks_and_sort() || check_run_loads() || check_pack() || check_saddle_loads(empty))
        return 1;
    if (empty == 0) return fail("saddle matrices produced no empty block", 0, 0);
    std::printf("ok\n");
    return 0;
}
