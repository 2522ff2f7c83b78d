// Launch schedules of the apply kernels, computed on the host from a plan.
#pragma once

#include <cstdint>
#include <vector>

namespace napspmv {

// Row blocks of the stream product: maximal runs of consecutive rows whose
// entries fit in `cap` (at most `max_rows` rows); a row longer than `cap`
// gets a block of its own.  rowblk[b], blkptr[b] = first row and first entry
// of block b; both have nblocks + 1 entries.
void row_blocks(const int32_t *rowptr, int64_t n, int cap, int max_rows,
                std::vector<int32_t> &rowblk, std::vector<int32_t> &blkptr);

// Row blocks of each process's rows [starts[t], starts[t+1]) in turn, so no
// block holds rows of two processes (the per-process launches of a
// partition use exactly these blocks).  Same encoding as row_blocks.
void row_blocks_per_process(const int32_t *rowptr, const std::vector<int64_t> &starts, int cap,
                            int max_rows, std::vector<int32_t> &rowblk,
                            std::vector<int32_t> &blkptr);

// Lanes of a workgroup of the apply kernels.
constexpr int kLanes = 256;

// Columns of v per band of the exchange buffers for row blocks of `cap`
// entries and `vec_bytes`-byte vector elements: cap * 8 bytes of v, the
// slice an exchange item stages in LDS (cap columns of float64, 2 cap of
// float32).  The first launch's LDS holds either such a slice or a row
// block's products and window, so float32 bands take no more LDS than
// float64 ones, and longer bands give each off-process block longer runs
// of ghosts side by side.
constexpr int band_columns(int cap, int vec_bytes) { return cap * 8 / vec_bytes; }

// Entries per lane that the off-process product loads with one vector load
// of columns, values and slots: 16 bytes of values (2 float64, 4 float32, 8
// bfloat16 entries), and no more than cap / kLanes.
constexpr int remote_run(int value_size, int cap) {
    return 16 / value_size <= cap / kLanes ? 16 / value_size : cap / kLanes;
}

// Offset from a = k0 & -run of the entry that lane t loads as component j of
// its u-th vector: the kernels' load order.
constexpr int32_t run_offset(int run, int u, int t, int j) { return run * (u * kLanes + t) + j; }

// Gather order of a block's entries: each block [blkptr[b], blkptr[b+1]) of
// at most `cap` entries is reordered by ascending column (stable), so the
// lanes of a wave read nearby ghost values; slot_out[k] = the stored
// position, inside its block, of the entry now at k.  Longer blocks (a
// single long row) keep stored order (slot 0).  `vs` = bytes of one value.
// With run > 1 (cap a multiple of run * kLanes), a block whose aligned span
// k1 - (k0 & -run) fits in `cap` is laid out for vector loads of `run`
// entries per lane: the gather-ordered entries fill the positions of
// [k0, k1) in the order the kernel's load instructions visit them (vector u,
// component j, lane t; see run_offset), so that each load instruction still
// reads, across its lanes, consecutive entries of gather order; a block
// whose aligned span does not fit (a single row, which the kernel walks in
// chunks) stays in stored order, slot 0, like the long ones.  With run 1,
// every block of at most `cap` entries is in plain gather order.  Blocks
// with keep[b] != 0 (keep may be null) stay in stored order, slot 0.
void sort_blocks(const std::vector<int32_t> &blkptr, int cap, const int32_t *col,
                 const uint8_t *val, int vs, int32_t *col_out, uint8_t *val_out,
                 uint16_t *slot_out, int run = 1, const uint8_t *keep = nullptr);

// Packed off-process words.  An off-process block laid out by runs for the
// gather (sort_blocks with run > 1) can carry each entry's ghost position
// and slot in one 32-bit word instead of an int32 position and a 16-bit
// slot: the slot (below 2^kPackSlotBits) in the high bits, and in the low
// kPackPosBits bits the position's offset from a base shared by the
// kPackLanes consecutive lanes of one wave load instruction (the smallest
// position those lanes read).  In gather order such lanes read positions of
// one or two bands of the ghost buffer, so the offsets stay small.  The
// bases of a block (cap / kPackLanes of them; wave = lane / kWave, group =
// lane % kWave / kPackLanes) sit at [wave][group][u * run + j] for runs of
// 2 (float64), so that a lane loads its bases for one vector of the run
// with one vector load (off-process launch 0.2075 -> 0.2029 ms), and at
// [wave][u * run + j][group] for runs of 4 and 8, whose lanes load them one
// by one, a wave's four groups from one 16-byte piece (float32 and
// bfloat16 lost 2-3% with the vector form).
constexpr int kWave = 64;
constexpr int kPackLanes = 16;
constexpr int kPackPosBits = 19;
constexpr int kPackSlotBits = 32 - kPackPosBits;

// Per-block kinds of the off-process product (a block's base entry; >= 0:
// the first ghost position of a narrow block, kept in stored order).
constexpr int32_t kPlainBlock = -1;
constexpr int32_t kPackedBlock = -2;

// Distance between the bases of consecutive loads of one lane.
constexpr int32_t pack_base_stride(int run) { return run < 4 ? 1 : kWave / kPackLanes; }

// Index of the base that lane t's component j of vector u reads.
constexpr int32_t pack_base_index(int cap, int run, int u, int t, int j) {
    return run < 4 ? ((t / kWave) * (kWave / kPackLanes) + (t % kWave) / kPackLanes) * (cap / kLanes) +
                         u * run + j
                   : ((t / kWave) * (cap / kLanes) + u * run + j) * (kWave / kPackLanes) +
                         (t % kWave) / kPackLanes;
}

// Pack block [k0, k1) of `pos` and `slot` (in load order, as sort_blocks
// wrote them) into word[k0..k1) and base[0 .. cap / kPackLanes).  Returns
// false, writing nothing, when the block is not laid out by runs (its
// aligned span k1 - (k0 & -run) exceeds cap, or cap is not a multiple of
// run * kLanes), when cap exceeds 2^kPackSlotBits, or when the positions of
// some lane group span 2^kPackPosBits or more.  Groups that read no entry
// of the block get base 0.
bool pack_block(int64_t k0, int64_t k1, int cap, int run, const int32_t *pos,
                const uint16_t *slot, uint32_t *word, int32_t *base);

// The window of v (first column, length <= `window`) each row block stages
// in LDS, as interleaved pairs: the block's whole on-process column range if
// it fits, otherwise `window` columns centred on the block's rows inside that
// range.  Windows stay inside [0, n).
void row_block_windows(const std::vector<int32_t> &rowblk, const std::vector<int32_t> &on_lo,
                       const std::vector<int32_t> &on_hi, int64_t n, int window,
                       std::vector<int32_t> &win);

// Launch order of the first apply launch: exchange items (encoded ~i) and
// local row blocks (encoded b >= 0), each list kept in its own order.  Each
// XCD's contiguous share of the launch gets its proportional slice of both,
// interleaved, except that its last `tail` tasks are row blocks only: an
// XCD holds about 128 of these blocks at once (32 CUs, 4 each), and an
// item still running in the final rounds would leave the rest idle.  NAP
// pack-and-scatter items carry about twice an exchange item's bytes, so
// they keep a longer tail.
constexpr int64_t kItemTail = 512;
constexpr int64_t kPackScatterTail = 1024;
void merge_tasks(int64_t n_items, int64_t n_blocks, std::vector<int32_t> &tasks,
                 int64_t tail = kItemTail);

// Work items covering [0, total) in order, pieces of at most `max_len`.
void flat_items(int64_t total, int max_len, std::vector<int32_t> &items);

}  // namespace napspmv
