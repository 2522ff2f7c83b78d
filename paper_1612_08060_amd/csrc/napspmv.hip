// The C ABI of include/napspmv.h: plan creation (host builder + device
// upload), the apply path (exchange kernels + split product), caller-owned
// workspaces, batched and per-partition applies, graph capture, tuning and
// diagnostics.  Nothing here throws across the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <chrono>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "napspmv.h"
#include "plan_build.hpp"
#include "schedule.hpp"

using napspmv::Error;
using napspmv::HostPlan;

namespace {
constexpr int kIndexedItem = 4096;                  // entries of an indexed exchange item
constexpr int kMinItem = 256, kMaxItem = 1 << 24;   // entries of a band exchange item
constexpr int kMaxRowsPerBlock = napspmv::kMaxRows;  // rows of an off-process block
constexpr int kMaxRowsOnBlock = napspmv::kMaxRowsOn;  // rows of an on-process block
constexpr int64_t kAlign = 256;

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Room for the holes the segment packing of the ghost buffer may leave (see
// build_layout): the buffer has G + ghost_slack(G) positions whatever the
// tuning, so workspace sizes never change.
int64_t ghost_slack(int64_t G) { return G / 16 + 64; }
}  // namespace

// Launch schedules of one set of row blocks and exchange items.
struct Schedules {
    int32_t *onblk = nullptr, *onptr = nullptr, *win = nullptr;
    int32_t *offblk = nullptr, *offptr = nullptr, *items = nullptr, *tasks = nullptr;
    int32_t *ndblk = nullptr, *ndptr = nullptr;     // three-way: on_node row blocks
    int32_t *onbase = nullptr;                      // first row of each on-process block's process
    int32_t *sitems = nullptr;                      // NAP: band items of the ghost scatter
    int32_t *gband = nullptr;                       // NAP: ghost band boundaries (pack-and-scatter items)
    int32_t *s1band = nullptr;                      // socket plans: l1x band boundaries
    int64_t n_on = 0, n_off = 0, n_items = 0, n_tasks = 0, n_nd = 0, n_sitems = 0, bytes = 0;
    // per-partition schedules only: each process's range of tasks and of
    // off-process blocks
    std::vector<int64_t> task_ptr, off_ptr;
};

struct napspmv_plan_s {
    HostPlan hp;
    uint32_t flags = 0;
    bool on_device = false;
    int device = 0;
    // tuning (-1 = automatic)
    int block_nnz = -1, item = -1, window = -1, remote_nnz = -1;
    int auto_block_nnz = 4096, auto_item = 65536, auto_window = 1024, auto_remote_nnz = 8192;
    int cur_block_nnz = 0, cur_item = 0, cur_window = -1, cur_remote_nnz = 0;   // on the device
    bool cur_item_auto = true;       // the schedules were built with an automatic item size
    int sorted_remote_nnz = 0;       // block size the off-process entry order was sorted for
    int64_t G = 0, E = 0, H = 0, Gon = 0;
    int64_t E1 = 0;                  // socket plans: entries of the l1x cross-socket buffer
    int64_t Gdev = 0;                // positions of the device ghost buffer (ghosts and holes)
    int32_t *d_rp_on = nullptr, *d_col_on = nullptr, *d_rp_off = nullptr, *d_col_off = nullptr;
    uint16_t *d_col16_on = nullptr;  // on-process columns as offsets from the process's first row
    void *d_val_on = nullptr, *d_val_off = nullptr;
    // Band-ordered exchange buffers (see exchange_item), laid out for bands of
    // `layout_cap` columns: gpos[k] = device position of ghost k of the
    // plan's process-ordered ghost list; d_off = column offset inside its
    // band of every ghost (standard) or send-buffer entry (NAP); d_code = the
    // source of every ghost position for the NAP scatter.
    int layout_cap = 0;
    std::vector<int32_t> gpos;
    std::vector<int32_t> dmap;           // direct reads: source code of every ghost
    std::vector<int64_t> gband, sband;   // band boundaries of the ghost / send buffers
    std::vector<int64_t> s1band;         // socket plans: band boundaries of the l1x buffer
    int32_t *d_s1src = nullptr;          // socket plans: source position of every l1x entry
    uint16_t *d_off = nullptr;
    uint32_t *d_code = nullptr;
    int32_t *d_pgcol = nullptr, *d_pgpos = nullptr;   // per-process indexed gathers
    // three-way plans: the fully local step as an indexed list (device
    // position, column of v) so that it does not walk every ghost position
    int32_t *d_l2pos = nullptr, *d_l2col = nullptr;
    // three-way plans: the on_node block, and the helper stream and events
    // that run the inter-node hop and scatter beside the on_node product
    int32_t *d_rp_nd = nullptr, *d_col_nd = nullptr;
    void *d_val_nd = nullptr;
    // gather order of the off-process (and on_node) blocks; see sort_blocks
    uint16_t *d_slot_off = nullptr, *d_slot_nd = nullptr;
    // off-process blocks whose ghost positions span less than 65536: their
    // positions as 16-bit offsets (d_col16_off) from the block's first one
    // (d_offbase[b]; -1 for a block that keeps 32-bit positions); null when
    // no block qualifies or the plan reads ghosts directly
    uint16_t *d_col16_off = nullptr;
    int32_t *d_offbase = nullptr;
    // off-process blocks in gather order whose d_col_off entries are packed
    // words (d_offbase[b] = kPackedBlock): their lane-group bases, cap /
    // kPackLanes per block (napspmv::pack_block)
    int32_t *d_pbase = nullptr;
    int64_t offbase_bytes = 0;
    int64_t block_kinds[3] = {0, 0, 0};  // off-process blocks: plain, packed, narrow
    int32_t plain_band = 0;          // exchange bands below it use plain stores (plain_bands)
    hipStream_t helper = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    void *d_ws = nullptr;            // the plan's own workspace (ghost, send, receive)
    Schedules sched;                 // all partitions in one launch pair
    Schedules part;                  // per-partition schedules (built on request)
    bool part_ready = false;
    int64_t device_bytes = 0;
    double build_s = 0, upload_s = 0;
};

// A batch object owns a ring of descriptor tables: call k fills table
// k mod kBatchRing, so a call waits for the device only when the call
// kBatchRing before it has not yet been read.
constexpr int kBatchRing = 4;

struct napspmv_batch_s {
    int capacity = 0;
    int device = 0;
    size_t desc_bytes = 0;
    int next = 0;                            // table of the next call
    void *d_desc[kBatchRing] = {};           // device descriptor tables
    void *h_desc[kBatchRing] = {};           // their pinned host staging
    hipEvent_t done[kBatchRing] = {};        // recorded after the launches that read each
    bool pending[kBatchRing] = {};
};

namespace {

thread_local std::string g_last_error;
std::atomic<int64_t> g_in_use{0};
std::atomic<int64_t> g_budget{0};

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw Error(NAPSPMV_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            if (hipSetDevice(dev) != hipSuccess) throw Error(NAPSPMV_EHIP, "hipSetDevice failed");
        } else {
            prev = -1;
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(NAPSPMV_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(NAPSPMV_EINVAL, e.what());
    }
}

int64_t vec_bytes(int dtype) { return dtype == NAPSPMV_F64 ? 8 : 4; }


// Workspace layout: ghost buffer, then the NAP send buffer, then the NAP
// receive buffer (explicit hop only), each 256-byte aligned.
struct WsLayout {
    int64_t ghost = 0, send = 0, recv = 0, total = 0;
};

WsLayout ws_layout(const napspmv_plan_s *p) {
    const int64_t vb = vec_bytes(p->hp.dtype);
    const bool nap = p->hp.mode == NAPSPMV_NAP;
    const bool copy = nap && (p->flags & NAPSPMV_EXCHANGE_COPY);
    WsLayout l;
    // direct reads fill no ghost buffer
    l.send = p->hp.direct ? 0 : align_up((p->G + ghost_slack(p->G)) * vb);
    // the received region: the send buffer (received in place) followed by
    // the cross-socket buffer of a socket plan
    l.total = l.send + (nap ? align_up((p->E + p->E1) * vb) : 0);
    l.recv = copy ? l.total : l.send;
    if (copy) l.total += align_up(p->E * vb);
    return l;
}

struct Ws {
    void *ghost, *send, *recv;
};

Ws ws_ptrs(const napspmv_plan_s *p, void *base) {
    if (!base) return Ws{nullptr, nullptr, nullptr};
    const WsLayout l = ws_layout(p);
    char *b = static_cast<char *>(base);
    return Ws{b + l.ghost, b + l.send, b + l.recv};
}

// Device arrays are never empty and start zeroed: the product kernels read
// clamped dummy entries (index 0 of an empty part) whose values they discard.
constexpr size_t kMinAlloc = 256;
// Entries of zero padding after the entry arrays of the products (columns,
// values, slots): the products load aligned runs of up to 8 entries, up to
// seven entries past a block.
constexpr size_t kQuadPad = 8;
// Row blocks of several rows hold at most block_nnz - 7 (remote_nnz - 7)
// entries, so that the aligned runs over a block stay within block_nnz
// (remote_nnz).
constexpr int kQuadSlack = 7;

template <typename T>
void upload(T *&dst, const std::vector<T> &src, int64_t &total, size_t pad = 0) {
    const size_t bytes = src.size() * sizeof(T), cap = std::max(bytes + pad * sizeof(T), kMinAlloc);
    HIP_OK(hipMalloc(reinterpret_cast<void **>(&dst), cap));
    total += (int64_t)cap;
    if (bytes) HIP_OK(hipMemcpy(dst, src.data(), bytes, hipMemcpyHostToDevice));
    if (cap > bytes) HIP_OK(hipMemset(reinterpret_cast<char *>(dst) + bytes, 0, cap - bytes));
}

void free_ptr(void *p) {
    if (p) (void)hipFree(p);
}

void charge(napspmv_plan_s *p, int64_t bytes) {
    p->device_bytes += bytes;
    g_in_use += bytes;
}

void free_schedules(napspmv_plan_s *p, Schedules &s) {
    void *ptrs[] = {s.onblk, s.onptr, s.win, s.offblk, s.offptr, s.items, s.tasks, s.ndblk, s.ndptr,
                    s.sitems, s.onbase, s.gband, s.s1band};
    for (void *q : ptrs) free_ptr(q);
    charge(p, -s.bytes);
    s = Schedules();
}

void free_device(napspmv_plan_s *p) {
    free_schedules(p, p->sched);
    free_schedules(p, p->part);
    p->part_ready = false;
    void *ptrs[] = {p->d_rp_on, p->d_col_on, p->d_rp_off, p->d_col_off, p->d_val_on,
                    p->d_val_off, p->d_off, p->d_code, p->d_pgcol, p->d_pgpos, p->d_ws,
                    p->d_l2pos, p->d_l2col,
                    p->d_rp_nd, p->d_col_nd, p->d_val_nd, p->d_slot_off, p->d_slot_nd,
                    p->d_col16_on, p->d_s1src, p->d_col16_off, p->d_offbase, p->d_pbase};
    for (void *q : ptrs) free_ptr(q);
    p->d_col16_off = nullptr;
    p->d_offbase = nullptr;
    p->d_pbase = nullptr;
    p->offbase_bytes = 0;
    p->d_rp_nd = p->d_col_nd = nullptr;
    p->d_val_nd = nullptr;
    p->d_slot_off = p->d_slot_nd = nullptr;
    p->d_col16_on = nullptr;
    p->d_s1src = nullptr;
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->helper) (void)hipStreamDestroy(p->helper);
    p->ev_fork = p->ev_join = nullptr;
    p->helper = nullptr;
    p->d_rp_on = p->d_col_on = p->d_rp_off = p->d_col_off = nullptr;
    p->d_val_on = p->d_val_off = p->d_ws = nullptr;
    p->d_off = nullptr;
    p->d_code = nullptr;
    p->d_pgcol = p->d_pgpos = nullptr;
    p->d_l2pos = p->d_l2col = nullptr;
    p->layout_cap = 0;
    p->sorted_remote_nnz = 0;
    g_in_use -= p->device_bytes;
    p->device_bytes = 0;
    p->on_device = false;
}

int64_t planned_device_bytes(const napspmv_plan_s *p) {
    const HostPlan &hp = p->hp;
    int64_t b = (int64_t)(hp.rowptr_on.size() + hp.col_on.size() + hp.rowptr_off.size() +
                          hp.col_off.size()) * 4 + (int64_t)(hp.val_on.size() + hp.val_off.size());
    b += (int64_t)(hp.rowptr_nd.size() + hp.col_nd.size()) * 4 + (int64_t)hp.val_nd.size();
    b += (int64_t)(hp.col_off.size() + hp.col_nd.size()) * 2;   // gather-order slots
    if (!hp.direct) b += (int64_t)hp.col_off.size() * 2;         // 16-bit positions (narrow blocks)
    // lane-group bases of packed blocks: 8192 / 16 per block at most, blocks
    // cut by entries or by 1024 rows
    if (!hp.direct) b += (hp.n_p + hp.n / 1024 + 1) * 2048 + (int64_t)hp.col_off.size() / 2;
    b += (int64_t)kQuadPad * (4 + hp.value_size) * 3;             // padding for vector loads
    // band offsets (ghosts or send entries) and, for NAP, the scatter codes
    const int64_t gd = p->G + ghost_slack(p->G);
    b += hp.mode == NAPSPMV_NAP ? p->E * 2 + gd * 4 : gd * 2;
    b += p->E1 * 4;                                               // l1x sources
    return b + ws_layout(p).total;
}

void upload_schedules(napspmv_plan_s *p, Schedules &s, const std::vector<int32_t> &onblk,
                      const std::vector<int32_t> &onptr, const std::vector<int32_t> &wins,
                      const std::vector<int32_t> &offblk, const std::vector<int32_t> &offptr,
                      const std::vector<int32_t> &items, const std::vector<int32_t> &tasks,
                      const std::vector<int32_t> &ndblk = {}, const std::vector<int32_t> &ndptr = {},
                      const std::vector<int32_t> &sitems = {}, const std::vector<int32_t> &onbase = {},
                      const std::vector<int32_t> &gband = {}, const std::vector<int32_t> &s1band = {}) {
    free_schedules(p, s);
    int64_t total = 0;
    try {
        upload(s.ndblk, ndblk, total);
        upload(s.ndptr, ndptr, total);
        upload(s.onblk, onblk, total);
        upload(s.onptr, onptr, total);
        upload(s.win, wins, total);
        upload(s.offblk, offblk, total);
        upload(s.offptr, offptr, total);
        upload(s.items, items, total);
        upload(s.tasks, tasks, total);
        upload(s.sitems, sitems, total);
        upload(s.onbase, onbase, total);
        upload(s.gband, gband, total);
        if (!s1band.empty()) upload(s.s1band, s1band, total);
    } catch (...) {
        s.bytes = total;
        charge(p, total);
        throw;
    }
    s.bytes = total;
    charge(p, total);
    s.n_on = (int64_t)onblk.size() - 1;
    s.n_off = (int64_t)offblk.size() - 1;
    s.n_items = (int64_t)items.size() / 4;
    s.n_sitems = (int64_t)sitems.size() / 4;
    s.n_tasks = (int64_t)tasks.size();
    s.n_nd = ndblk.empty() ? 0 : (int64_t)ndblk.size() - 1;
}

int cur_cap(const napspmv_plan_s *p) { return p->block_nnz >= 0 ? p->block_nnz : p->auto_block_nnz; }
int cur_rcap(const napspmv_plan_s *p) {
    return p->remote_nnz >= 0 ? p->remote_nnz : p->auto_remote_nnz;
}
bool valid_block(int v) { return v == 1024 || v == 2048 || v == 4096 || v == 8192; }
// remote block sizes, in the order of the batched launch's groups
constexpr int kRemoteSizes = 4;
int remote_size_index(int rcap) { return rcap == 1024 ? 0 : rcap == 2048 ? 1 : rcap == 4096 ? 2 : 3; }
int cur_win(const napspmv_plan_s *p) { return p->window >= 0 ? p->window : p->auto_window; }
int cur_item(const napspmv_plan_s *p) { return p->item >= 0 ? p->item : p->auto_item; }

// Per-partition schedules (standard mode): each process's row blocks and
// indexed gather items for its own ghosts (into their band-ordered
// positions), contiguous per process, so one process's product is one pair
// of launches.
void build_partitions(napspmv_plan_s *p) {
    const HostPlan &hp = p->hp;
    const int cap = cur_cap(p), win = cur_win(p);
    {
        // indexed gathers: source column and device position of every ghost
        int64_t total = 0;
        if (!p->d_pgcol) upload(p->d_pgcol, hp.ghost_col, total);
        if (p->d_pgpos) {
            HIP_OK(hipMemcpy(p->d_pgpos, p->gpos.data(), p->gpos.size() * 4, hipMemcpyHostToDevice));
        } else {
            upload(p->d_pgpos, p->gpos, total);
        }
        charge(p, total);
    }
    std::vector<int32_t> onblk, onptr, wins, offblk, offptr, items, tasks, onbase;
    std::vector<int64_t> task_ptr(hp.n_p + 1, 0), off_ptr(hp.n_p + 1, 0);
    for (int64_t t = 0; t < hp.n_p; ++t) {
        const int64_t r0 = hp.starts[t], r1 = hp.starts[t + 1];
        std::vector<int32_t> ob, op, fb, fp, it, ts, wn;
        napspmv::row_blocks(hp.rowptr_on.data() + r0, r1 - r0, cap - kQuadSlack, kMaxRowsOnBlock,
                            ob, op);
        napspmv::row_blocks(hp.rowptr_off.data() + r0, r1 - r0, cur_rcap(p) - kQuadSlack,
                            kMaxRowsPerBlock, fb, fp);
        for (auto &x : ob) x += (int32_t)r0;
        for (auto &x : fb) x += (int32_t)r0;
        if (win > 0) napspmv::row_block_windows(ob, hp.on_lo, hp.on_hi, hp.n, win, wn);
        std::vector<int32_t> flat;
        napspmv::flat_items(hp.ghost_ptr[t + 1] - hp.ghost_ptr[t], kIndexedItem, flat);
        for (size_t k = 0; k < flat.size(); k += 2) {
            const int32_t q[4] = {-1, flat[k] + (int32_t)hp.ghost_ptr[t], flat[k + 1], 0};
            it.insert(it.end(), q, q + 4);
        }
        const int32_t blk_base = (int32_t)onblk.size();
        const int32_t item_base = (int32_t)(items.size() / 4);
        napspmv::merge_tasks((int64_t)it.size() / 4, (int64_t)ob.size() - 1, ts);
        for (auto &x : ts) x = x < 0 ? ~(~x + item_base) : x + blk_base;
        // concatenate; a process's closing boundary is the next one's first
        onblk.insert(onblk.end(), ob.begin(), ob.end() - 1);
        onptr.insert(onptr.end(), op.begin(), op.end() - 1);
        onbase.insert(onbase.end(), ob.size() - 1, (int32_t)r0);
        wins.insert(wins.end(), wn.begin(), wn.end());
        off_ptr[t] = (int64_t)offblk.size();
        offblk.insert(offblk.end(), fb.begin(), fb.end() - 1);
        offptr.insert(offptr.end(), fp.begin(), fp.end() - 1);
        off_ptr[t + 1] = (int64_t)offblk.size();
        items.insert(items.end(), it.begin(), it.end());
        tasks.insert(tasks.end(), ts.begin(), ts.end());
        task_ptr[t + 1] = (int64_t)tasks.size();
    }
    onblk.push_back((int32_t)hp.n);
    onptr.push_back(hp.rowptr_on[hp.n]);
    offblk.push_back((int32_t)hp.n);
    offptr.push_back(hp.rowptr_off[hp.n]);
    upload_schedules(p, p->part, onblk, onptr, wins, offblk, offptr, items, tasks, {}, {}, {}, onbase);
    p->part.task_ptr = task_ptr;
    p->part.off_ptr = off_ptr;
    p->part_ready = true;
}

// Map the ghost positions of a block list to device positions (`map`),
// reorder the entries of every block into gather order (sort_blocks) and
// copy them, with their slots, over the device arrays (already allocated).
// With `p` (the off-process part of a plan that fills a ghost buffer), the
// blocks whose positions span less than 65536 (stencil-like halos) stay in
// stored order instead, need no slots, and have their positions as 16-bit
// offsets from their first one (p->d_col16_off, p->d_offbase): two bytes
// instead of six per entry.  Their stored order already reads the ghosts
// in short ascending runs (a row's neighbours in each halo plane).  The
// other gather-ordered blocks carry position and slot in one packed word
// where pack_block allows it (p->d_pbase): four bytes instead of six.
void sort_upload(const std::vector<int32_t> &col, const std::vector<int32_t> &map,
                 const std::vector<uint8_t> &val, int vs, const std::vector<int32_t> &blkptr, int cap,
                 int32_t *d_col, void *d_val, uint16_t *d_slot, napspmv_plan_s *p = nullptr) {
    if (p) {
        free_ptr(p->d_offbase);
        free_ptr(p->d_pbase);
        p->d_offbase = nullptr;
        p->d_pbase = nullptr;
        charge(p, -p->offbase_bytes);
        p->offbase_bytes = 0;
    }
    if (col.empty()) return;
    std::vector<int32_t> cm(col.size()), c2(col.size());
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)col.size(); ++k) cm[k] = map[col[k]];
    const int64_t nb = (int64_t)blkptr.size() - 1;
    std::vector<int32_t> base;
    std::vector<uint8_t> keep;
    int64_t narrow = 0;
    if (p) {
        base.assign(nb, napspmv::kPlainBlock);
        keep.assign(nb, 0);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : narrow)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t k0 = blkptr[b], k1 = blkptr[b + 1];
            if (k1 == k0) continue;
            int32_t lo = INT32_MAX, hi = -1;
            for (int64_t k = k0; k < k1; ++k) {
                lo = std::min(lo, cm[k]);
                hi = std::max(hi, cm[k]);
            }
            if (hi - lo > 65535) continue;
            base[b] = lo;
            keep[b] = 1;
            ++narrow;
        }
    }
    std::vector<uint8_t> v2(val.size());
    std::vector<uint16_t> s2(col.size());
    const int run = napspmv::remote_run(vs, cap);
    napspmv::sort_blocks(blkptr, cap, cm.data(), val.data(), vs, c2.data(), v2.data(), s2.data(),
                         run, narrow ? keep.data() : nullptr);
    // packed words, written over the positions of each block that takes them
    int64_t packed = 0;
    std::vector<int32_t> pbase;
    if (p) {
        const int64_t per = cap / napspmv::kPackLanes;
        pbase.assign((size_t)(nb * per), 0);
        uint32_t *words = reinterpret_cast<uint32_t *>(c2.data());
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : packed)
        for (int64_t b = 0; b < nb; ++b)
            if (base[b] == napspmv::kPlainBlock && blkptr[b + 1] > blkptr[b] &&
                napspmv::pack_block(blkptr[b], blkptr[b + 1], cap, run, c2.data(), s2.data(),
                                    words, pbase.data() + b * per)) {
                base[b] = napspmv::kPackedBlock;
                ++packed;
            }
    }
    HIP_OK(hipMemcpy(d_col, c2.data(), c2.size() * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_val, v2.data(), v2.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_slot, s2.data(), s2.size() * 2, hipMemcpyHostToDevice));
    if (p) {
        int64_t empty = 0;
        for (int64_t b = 0; b < nb; ++b) empty += blkptr[b + 1] == blkptr[b];
        p->block_kinds[0] = nb - packed - narrow - empty;
        p->block_kinds[1] = packed;
        p->block_kinds[2] = narrow;
    }
    if (narrow == 0 && packed == 0) return;
    int64_t total = 0;
    if (packed) upload(p->d_pbase, pbase, total);
    if (narrow == 0) {
        upload(p->d_offbase, base, total);
        p->offbase_bytes = total;
        charge(p, total);
        return;
    }
    std::vector<uint16_t> c16(col.size(), 0);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nb; ++b)
        if (base[b] >= 0)
            for (int64_t k = blkptr[b]; k < blkptr[b + 1]; ++k) c16[k] = (uint16_t)(c2[k] - base[b]);
    if (!p->d_col16_off) {
        // kept across re-sorts, like the other entry arrays
        const size_t bytes = (col.size() + kQuadPad) * 2;
        HIP_OK(hipMalloc(reinterpret_cast<void **>(&p->d_col16_off), bytes));
        HIP_OK(hipMemset(p->d_col16_off, 0, bytes));
        charge(p, (int64_t)bytes);
    }
    HIP_OK(hipMemcpy(p->d_col16_off, c16.data(), c16.size() * 2, hipMemcpyHostToDevice));
    upload(p->d_offbase, base, total);
    p->offbase_bytes = total;
    charge(p, total);
}

// Stable sort of entries by the band of their column and then by `group`
// (NULL: none): pos[k] = the device position of entry k, bstart = band
// boundaries (nb + 1).  A counting sort when the key space is small.
void band_order(const int32_t *cols, int64_t m, int cap, int64_t nb, const int32_t *group,
                int64_t ngroups, std::vector<int32_t> &pos, std::vector<int64_t> &bstart) {
    if (!group) ngroups = 1;
    auto key = [&](int64_t k) { return (int64_t)(cols[k] / cap) * ngroups + (group ? group[k] : 0); };
    pos.resize(m);
    bstart.assign(nb + 1, 0);
    for (int64_t k = 0; k < m; ++k) ++bstart[cols[k] / cap + 1];
    for (int64_t b = 0; b < nb; ++b) bstart[b + 1] += bstart[b];
    const int64_t nk = nb * ngroups;
    if (nk <= (int64_t)1 << 26) {
        std::vector<int64_t> next(nk + 1, 0);
        for (int64_t k = 0; k < m; ++k) ++next[key(k) + 1];
        for (int64_t q = 0; q < nk; ++q) next[q + 1] += next[q];
        for (int64_t k = 0; k < m; ++k) pos[k] = (int32_t)next[key(k)]++;
    } else {
        std::vector<int32_t> ord(m);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
        for (int64_t q = 0; q < m; ++q) pos[ord[q]] = (int32_t)q;
    }
}

// Segment packing of the ghost buffer.  On entry gpos/gband hold the order
// (band, first reading block, column) without holes; each block's ghosts of
// a band form one run of a few values (about 6 on the KKT-like matrix),
// which in that order straddles the 64-byte segments of the buffer at
// random, so a block's gather touches about 1.8 segments per run.  Inside
// each band the runs are re-placed group by group, a group being the runs
// of kPackGroup consecutive blocks (blocks that run at the same time on one
// XCD, so their segments still meet in its L2; packing a whole band at once
// spreads each block over the band and loses that): runs of a segment or
// more start on a segment boundary, shorter ones go first-fit (longest
// first) into the segment tails the group left free, and a tail nothing
// fits stays a hole.  Most runs then lie in one segment (8.3 M instead of
// 11.1 M gather requests on the KKT-like matrix).  If the holes would exceed
// ghost_slack(G) the order stays unpacked.  Values inside a run keep column
// order.
constexpr int32_t kPackGroup = 64;

void pack_segments(napspmv_plan_s *p, const int32_t *first_blk, int seg) {
    const int64_t G = p->G, nb = (int64_t)p->gband.size() - 1;
    p->Gdev = G;
    if (G == 0 || seg <= 1) return;
    std::vector<int32_t> ord(G);
    for (int64_t k = 0; k < G; ++k) ord[p->gpos[k]] = (int32_t)k;
    std::vector<int64_t> local(G), bsize(nb, 0);
#pragma omp parallel
    {
        std::vector<int64_t> rs, rl, order;
        std::vector<std::pair<int64_t, int64_t>> freel;   // (offset, room) of segment tails
#pragma omp for schedule(dynamic, 8)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t a0 = p->gband[b], a1 = p->gband[b + 1];
            rs.clear();
            rl.clear();
            for (int64_t q = a0; q < a1;) {
                int64_t e = q + 1;
                while (e < a1 && first_blk[ord[e]] == first_blk[ord[q]]) ++e;
                rs.push_back(q);
                rl.push_back(e - q);
                q = e;
            }
            // groups of runs of kPackGroup consecutive blocks, each packed alone
            order.resize(rs.size());
            std::iota(order.begin(), order.end(), 0);
            auto group = [&](int64_t r) { return first_blk[ord[rs[r]]] / kPackGroup; };
            std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
                const int32_t gx = group(x), gy = group(y);
                return gx != gy ? gx < gy : rl[x] > rl[y];
            });
            int64_t cur = 0;
            int32_t open_group = -1;
            for (int64_t r : order) {
                if (group(r) != open_group) {
                    open_group = group(r);
                    freel.clear();
                }
                const int64_t L = rl[r];
                int64_t at = -1;
                if (L < seg)
                    for (size_t f = 0; f < freel.size(); ++f)
                        if (freel[f].second >= L) {
                            at = freel[f].first;
                            freel[f].first += L;
                            freel[f].second -= L;
                            if (freel[f].second == 0) freel.erase(freel.begin() + f);
                            break;
                        }
                if (at < 0) {
                    at = cur;
                    cur += L;
                    const int64_t tail = (seg - cur % seg) % seg;
                    if (tail) freel.emplace_back(cur, tail);
                    cur += tail;
                }
                for (int64_t i = 0; i < L; ++i) local[rs[r] + i] = at + i;
            }
            bsize[b] = cur;
        }
    }
    std::vector<int64_t> base(nb + 1, 0);
    for (int64_t b = 0; b < nb; ++b) base[b + 1] = base[b] + bsize[b];
    if (base[nb] - G > ghost_slack(G)) return;        // too many holes: keep the unpacked order
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t q = p->gband[b]; q < p->gband[b + 1]; ++q)
            p->gpos[ord[q]] = (int32_t)(base[b] + local[q]);
    p->gband = base;
    p->Gdev = base[nb];
}

// Band layout of the exchange buffers for bands of `cap` columns (the LDS
// tile of the exchange kernels, band_columns of the block size): ghost
// positions, band offsets, NAP send positions and scatter codes; uploaded
// over the plan's device arrays.
void build_layout(napspmv_plan_s *p, int cap, const std::vector<int32_t> &offptr,
                  const std::vector<int32_t> &ndptr) {
    const HostPlan &hp = p->hp;
    const int64_t nb = (hp.n + cap - 1) / cap, G = p->G, E = p->E;
    // Inside a band, ghosts are ordered by the first off-process row block
    // that reads them (then by column): each block's gather then finds most
    // of its ghosts of a band side by side, where in process order they are
    // spread over its process's whole run of the band, which other blocks
    // share (about 35 instead of 23 useful bytes per 64-byte request on the
    // KKT-like matrix).  The exchange writes every band as one range, so
    // any order inside a band costs it nothing.  A three-way plan numbers
    // its on_node blocks after its off_node blocks.
    std::vector<int32_t> first_blk(G, INT32_MAX);
    const int64_t n_off = (int64_t)offptr.size() - 1;
    auto mark = [&](const std::vector<int32_t> &cols, const std::vector<int32_t> &bptr, int64_t base) {
        for (int64_t b = 0; b + 1 < (int64_t)bptr.size(); ++b)
            for (int64_t k = bptr[b]; k < bptr[b + 1]; ++k)
                first_blk[cols[k]] = std::min<int32_t>(first_blk[cols[k]], (int32_t)(base + b));
    };
    mark(hp.col_off, offptr, 0);
    if (hp.three_way) mark(hp.col_nd, ndptr, n_off);
    int32_t nblk = (int32_t)(n_off + (hp.three_way ? (int64_t)ndptr.size() - 1 : 0)) + 1;
    for (int32_t &f : first_blk)
        if (f == INT32_MAX) f = nblk - 1;      // a ghost no block reads (none in a valid plan)
    band_order(hp.ghost_col.data(), G, cap, nb, first_blk.data(), nblk, p->gpos, p->gband);
    pack_segments(p, first_blk.data(), 64 / (int)vec_bytes(hp.dtype));
    const std::vector<int32_t> &gpos = p->gpos;
    const int64_t Gd = p->Gdev;
    if (hp.mode == NAPSPMV_STANDARD) {
        std::vector<uint16_t> off(Gd, 0);      // holes copy the band's first column
        for (int64_t k = 0; k < G; ++k) off[gpos[k]] = (uint16_t)(hp.ghost_col[k] % cap);
        if (Gd) HIP_OK(hipMemcpy(p->d_off, off.data(), Gd * 2, hipMemcpyHostToDevice));
    } else {
        // inside a band, the send buffer is grouped by destination (receiving
        // node, or socket for the cross-socket entries of a socket plan), so
        // the values one destination's ghosts take from a band lie together
        int64_t ngroups = 1;
        for (int32_t g : hp.pack_group) ngroups = std::max<int64_t>(ngroups, (int64_t)g + 1);
        for (int32_t g : hp.l1x_group) ngroups = std::max<int64_t>(ngroups, (int64_t)g + 1);
        std::vector<int32_t> spos;
        band_order(hp.pack_idx.data(), E, cap, nb, hp.pack_group.data(), ngroups, spos, p->sband);
        std::vector<uint16_t> off(E);
        for (int64_t e = 0; e < E; ++e) off[spos[e]] = (uint16_t)(hp.pack_idx[e] % cap);
        // socket plans: the l1x buffer follows the send buffer, band-ordered
        // the same way; each entry copies a received value of its band
        std::vector<int32_t> l1pos;
        if (p->E1 > 0) {
            band_order(hp.l1x_col.data(), p->E1, cap, nb, hp.l1x_group.data(), ngroups, l1pos,
                       p->s1band);
            std::vector<int32_t> src(p->E1);
            for (int64_t k = 0; k < p->E1; ++k) src[l1pos[k]] = spos[hp.l1x_src[k]];
            HIP_OK(hipMemcpy(p->d_s1src, src.data(), p->E1 * 4, hipMemcpyHostToDevice));
        }
        std::vector<uint32_t> code(Gd, napspmv::kFromV);   // holes copy the band's first column
        for (int64_t h = 0; h < p->H; ++h) {
            const int64_t src = hp.scat_src[h];
            code[gpos[hp.scat_dst[h]]] = (uint32_t)(src < E ? spos[src] : E + l1pos[src - E]);
        }
        for (int64_t k = 0; k < p->Gon; ++k)
            code[gpos[hp.l2_dst[k]]] = napspmv::kFromV | (uint32_t)(hp.l2_src[k] % cap);
        if (E) HIP_OK(hipMemcpy(p->d_off, off.data(), E * 2, hipMemcpyHostToDevice));
        if (Gd) HIP_OK(hipMemcpy(p->d_code, code.data(), Gd * 4, hipMemcpyHostToDevice));
        if (hp.direct) {
            // off-node ghosts read the received buffer, on-node ones v (sign bit)
            p->dmap.assign(G, 0);
            for (int64_t h = 0; h < p->H; ++h) p->dmap[hp.scat_dst[h]] = spos[hp.scat_src[h]];
            for (int64_t k = 0; k < p->Gon; ++k)
                p->dmap[hp.l2_dst[k]] = (int32_t)(napspmv::kFromV | (uint32_t)hp.l2_src[k]);
        }
        if (hp.three_way && p->Gon > 0) {
            std::vector<int32_t> l2pos(p->Gon);
            for (int64_t k = 0; k < p->Gon; ++k) l2pos[k] = gpos[hp.l2_dst[k]];
            HIP_OK(hipMemcpy(p->d_l2pos, l2pos.data(), p->Gon * 4, hipMemcpyHostToDevice));
        }
    }
    p->layout_cap = cap;
}

// Band items (band, first, count, 0) over a band-ordered buffer, at most
// `item` entries each.
void band_items(const std::vector<int64_t> &bstart, int item, std::vector<int32_t> &items) {
    items.clear();
    for (int64_t b = 0; b + 1 < (int64_t)bstart.size(); ++b)
        for (int64_t k = bstart[b]; k < bstart[b + 1]; k += item) {
            const int32_t q[4] = {(int32_t)b, (int32_t)k, (int32_t)std::min<int64_t>(item, bstart[b + 1] - k), 0};
            items.insert(items.end(), q, q + 4);
        }
}

// The first launch's exchange buffer and both launches' w are written with
// non-temporal stores when that buffer is larger than the 256 MB Infinity
// Cache: the second launch cannot find it there anyway, and lines left dirty
// in L2 would be written back while the second launch runs.  (Smaller
// buffers are read back from the cache, and plain stores are faster.)
int32_t stream_out(const napspmv_plan_s *p) {
    const int64_t x = (p->hp.mode == NAPSPMV_STANDARD ? p->G : p->E) * vec_bytes(p->hp.dtype);
    return x > ((int64_t)256 << 20) ? 1 : 0;
}

// Except, in a standard plan whose ghost buffer is at most twice that
// cache, the bands of its first 160 MB: those the exchange stores plainly.
// Their write-back then overlaps the end of the first launch and the second
// launch, and the first launch gains more than the second loses (KKT-like
// float64 apply, plain stores for the first 79 / 158 / 237 MB of the 316 MB
// ghost buffer: 0.4565 / 0.452 / 0.4625 ms against 0.458 ms).  With a much
// larger buffer the second launch loses more (the strided partition of the
// same matrix, 996 MB of ghosts: 0.916 -> 0.929 ms).  Returns the first band
// stored non-temporally; computed when the bands are laid out.
int32_t plain_bands(const napspmv_plan_s *p) {
    constexpr int64_t kPlainBytes = (int64_t)160 << 20;
    const int64_t vb = vec_bytes(p->hp.dtype);
    if (p->hp.mode != NAPSPMV_STANDARD || !stream_out(p) || p->G * vb > ((int64_t)512 << 20))
        return 0;
    int32_t b = 0;
    while (b + 1 < (int32_t)p->gband.size() && p->gband[b + 1] * vb <= kPlainBytes) ++b;
    return b;
}

// (Re)build the launch schedules for the current tuning: on-process row
// blocks with their v windows and process bases, off-process row blocks,
// the band items of the exchange (standard: the ghost buffer; NAP: the send
// buffer, plus the scatter items over the ghost buffer) and the task list of
// the first launch; re-lay the bands and re-sort the off-process blocks when
// the block sizes change.  Per-partition schedules follow.
void refresh_schedules(napspmv_plan_s *p) {
    const int cap = cur_cap(p), win = cur_win(p), item = cur_item(p), rcap = cur_rcap(p);
    if (p->sched.onblk && cap == p->cur_block_nnz && win == p->cur_window && item == p->cur_item &&
        rcap == p->cur_remote_nnz && (p->item < 0) == p->cur_item_auto)
        return;
    const HostPlan &hp = p->hp;
    std::vector<int32_t> onblk, onptr, wins, offblk, offptr, items, tasks, sitems, onbase, gbv, s1v;
    int64_t tail = napspmv::kItemTail;
    // on-process blocks never span two processes: each block's columns are
    // offsets from its process's first row
    napspmv::row_blocks_per_process(hp.rowptr_on.data(), hp.starts, cap - kQuadSlack,
                                    kMaxRowsOnBlock, onblk, onptr);
    onbase.resize(onblk.size() - 1);
    for (size_t b = 0; b + 1 < onblk.size(); ++b)
        onbase[b] = (int32_t)hp.starts[(std::upper_bound(hp.starts.begin(), hp.starts.end(), onblk[b]) -
                                        hp.starts.begin()) - 1];
    if (win > 0) napspmv::row_block_windows(onblk, hp.on_lo, hp.on_hi, hp.n, win, wins);
    napspmv::row_blocks_per_process(hp.rowptr_off.data(), hp.starts, rcap - kQuadSlack,
                                    kMaxRowsPerBlock, offblk, offptr);
    std::vector<int32_t> ndblk, ndptr;
    if (hp.three_way)
        napspmv::row_blocks_per_process(hp.rowptr_nd.data(), hp.starts, rcap - kQuadSlack,
                                        kMaxRowsPerBlock, ndblk, ndptr);
    const int band = napspmv::band_columns(cap, (int)vec_bytes(hp.dtype));
    if (band != p->layout_cap || rcap != p->sorted_remote_nnz) {
        // the exchange layout follows the band width and the off-process
        // block cuts; the entry order of the off-process blocks follows the
        // layout and the block cuts
        HIP_OK(hipDeviceSynchronize());
        build_layout(p, band, offptr, ndptr);
        p->plain_band = plain_bands(p);
        sort_upload(hp.col_off, hp.direct ? p->dmap : p->gpos, hp.val_off, (int)hp.value_size,
                    offptr, rcap, p->d_col_off, p->d_val_off, p->d_slot_off,
                    hp.direct ? nullptr : p);
        if (hp.direct) {
            // direct reads keep int32 sources in gather order
            p->block_kinds[0] = p->block_kinds[1] = p->block_kinds[2] = 0;
            for (size_t b = 0; b + 1 < offptr.size(); ++b) p->block_kinds[0] += offptr[b + 1] > offptr[b];
        }
        if (hp.three_way)
            sort_upload(hp.col_nd, p->gpos, hp.val_nd, (int)hp.value_size, ndptr, rcap,
                        p->d_col_nd, p->d_val_nd, p->d_slot_nd);
        p->sorted_remote_nnz = rcap;
    }
    if (hp.mode == NAPSPMV_STANDARD) {
        band_items(p->gband, item, items);
    } else {
        // received in place, each band's send entries in one item: pack and
        // scatter band by band in the first launch (pack_scatter_item)
        int64_t widest = 0;
        for (size_t b = 0; b + 1 < p->sband.size(); ++b)
            widest = std::max(widest, p->sband[b + 1] - p->sband[b]);
        // (an automatic item size always allows it: a band's item is then
        // as wide as the band)
        // (a socket plan always fuses: its l1x copies run inside the items)
        const bool fuse = hp.pps > 0 ||
                          (!hp.three_way && !hp.direct && !(p->flags & NAPSPMV_EXCHANGE_COPY) &&
                           (p->item < 0 || widest <= item));
        if (fuse) {
            tail = napspmv::kPackScatterTail;
            for (size_t b = 0; b + 1 < p->sband.size(); ++b) {
                const int64_t ns = p->sband[b + 1] - p->sband[b], ng = p->gband[b + 1] - p->gband[b];
                if (ns == 0 && ng == 0) continue;
                const int32_t q[4] = {(int32_t)b, (int32_t)p->sband[b], (int32_t)ns, 1};
                items.insert(items.end(), q, q + 4);
            }
            gbv.assign(p->gband.begin(), p->gband.end());
            if (p->E1 > 0) {
                // l1x band boundaries, offset to their place after the send buffer
                s1v.resize(p->s1band.size());
                for (size_t b = 0; b < p->s1band.size(); ++b) s1v[b] = (int32_t)(p->E + p->s1band[b]);
            }
        } else {
            band_items(p->sband, item, items);
            band_items(p->gband, item, sitems);
        }
    }
    napspmv::merge_tasks((int64_t)items.size() / 4, (int64_t)onblk.size() - 1, tasks, tail);
    upload_schedules(p, p->sched, onblk, onptr, wins, offblk, offptr, items, tasks, ndblk, ndptr,
                     sitems, onbase, gbv, s1v);
    p->cur_block_nnz = cap;
    p->cur_window = win;
    p->cur_item = item;
    p->cur_item_auto = p->item < 0;
    p->cur_remote_nnz = rcap;
    if (p->part_ready) build_partitions(p);
}

void to_device(napspmv_plan_s *p) {
    HostPlan &hp = p->hp;
    HIP_OK(hipGetDevice(&p->device));
    const int64_t need = planned_device_bytes(p);
    const int64_t budget = g_budget.load();
    if (budget > 0 && g_in_use.load() + need > budget)
        throw Error(NAPSPMV_ENOMEM, "device budget exceeded: plan needs " + std::to_string(need) +
                                        " bytes, " + std::to_string(g_in_use.load()) +
                                        " in use of " + std::to_string(budget));
    int64_t total = 0;
    try {
        upload(p->d_rp_on, hp.rowptr_on, total);
        int64_t most_rows = 0;
        for (int64_t t = 0; t < hp.n_p; ++t) most_rows = std::max(most_rows, hp.starts[t + 1] - hp.starts[t]);
        if (most_rows <= 65536) {
            // on-process columns as 16-bit offsets from the process's first row
            std::vector<uint16_t> c16(hp.col_on.size());
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t t = 0; t < hp.n_p; ++t)
                for (int64_t k = hp.rowptr_on[hp.starts[t]]; k < hp.rowptr_on[hp.starts[t + 1]]; ++k)
                    c16[k] = (uint16_t)(hp.col_on[k] - hp.starts[t]);
            upload(p->d_col16_on, c16, total, kQuadPad);
        } else {
            upload(p->d_col_on, hp.col_on, total, kQuadPad);
        }
        upload(p->d_rp_off, hp.rowptr_off, total);
        auto alloc = [&](auto *&dst, size_t bytes) {
            const size_t cap = std::max(bytes, kMinAlloc);
            HIP_OK(hipMalloc(reinterpret_cast<void **>(&dst), cap));
            total += (int64_t)cap;
            HIP_OK(hipMemset(dst, 0, cap));
        };
        // entry arrays of the off-process blocks: filled in gather order by
        // refresh_schedules
        alloc(p->d_col_off, (hp.col_off.size() + kQuadPad) * 4);
        alloc(p->d_val_off, hp.val_off.size() + kQuadPad * hp.value_size);
        alloc(p->d_slot_off, (hp.col_off.size() + kQuadPad) * 2);
        auto upload_bytes = [&](void *&dst, const std::vector<uint8_t> &src, size_t pad) {
            const size_t cap = std::max(src.size() + pad, kMinAlloc);
            HIP_OK(hipMalloc(&dst, cap));
            total += (int64_t)cap;
            if (!src.empty()) HIP_OK(hipMemcpy(dst, src.data(), src.size(), hipMemcpyHostToDevice));
            if (cap > src.size())
                HIP_OK(hipMemset(static_cast<char *>(dst) + src.size(), 0, cap - src.size()));
        };
        upload_bytes(p->d_val_on, hp.val_on, kQuadPad * (size_t)hp.value_size);
        if (hp.three_way) {
            upload(p->d_rp_nd, hp.rowptr_nd, total);
            alloc(p->d_col_nd, (hp.col_nd.size() + kQuadPad) * 4);
            alloc(p->d_val_nd, hp.val_nd.size() + kQuadPad * hp.value_size);
            alloc(p->d_slot_nd, (hp.col_nd.size() + kQuadPad) * 2);
            alloc(p->d_l2pos, (size_t)p->Gon * 4);
            upload(p->d_l2col, hp.l2_src, total);
            HIP_OK(hipStreamCreateWithFlags(&p->helper, hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
            HIP_OK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
        }
        // band layout arrays: filled by refresh_schedules
        if (hp.mode == NAPSPMV_STANDARD) {
            alloc(p->d_off, (size_t)(p->G + ghost_slack(p->G)) * 2);
        } else {
            alloc(p->d_off, (size_t)p->E * 2);
            alloc(p->d_code, (size_t)(p->G + ghost_slack(p->G)) * 4);
            if (p->E1 > 0) alloc(p->d_s1src, (size_t)p->E1 * 4);
        }
        const int64_t wsb = ws_layout(p).total;
        if (wsb > 0) {
            HIP_OK(hipMalloc(&p->d_ws, (size_t)wsb));
            total += wsb;
        }
        charge(p, total);
        total = 0;
        refresh_schedules(p);
        HIP_OK(hipDeviceSynchronize());
    } catch (...) {
        charge(p, total);
        free_device(p);
        throw;
    }
    p->on_device = true;
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + napspmv::kBlock - 1) / napspmv::kBlock); }

// ---- views -------------------------------------------------------------------

template <typename VT, typename XT>
napspmv::LocalView<VT, XT> local_view(const napspmv_plan_s *p, const Schedules &s, const Ws &ws,
                                      const XT *v, XT *w, int64_t task0, int64_t n_tasks) {
    const bool std_mode = p->hp.mode == NAPSPMV_STANDARD;
    napspmv::LocalView<VT, XT> L;
    L.tasks = s.tasks + task0;
    L.n_tasks = (int32_t)n_tasks;
    L.items = reinterpret_cast<const int4 *>(s.items);
    L.off = p->d_off;
    L.idx = p->d_pgcol;
    L.dpos = p->d_pgpos;
    L.xdst = static_cast<XT *>(std_mode ? ws.ghost : ws.send);
    L.n = (int32_t)p->hp.n;
    L.rowblk = s.onblk;
    L.blkptr = s.onptr;
    L.win = reinterpret_cast<const int2 *>(s.win);
    L.rowptr = p->d_rp_on;
    L.col = p->d_col_on;
    L.col16 = p->d_col16_on;
    L.base = s.onbase;
    L.val = static_cast<const VT *>(p->d_val_on);
    L.v = v;
    L.w = w;
    L.nt = stream_out(p);
    L.nt_band = p->plain_band;
    L.gband = s.gband;
    L.s1band = s.s1band;
    L.s1src = p->d_s1src;
    L.code = p->d_code;
    L.recv = static_cast<const XT *>(ws.recv);
    L.ghost = static_cast<XT *>(ws.ghost);
    return L;
}

// Off-process product view; `on_node` selects a three-way plan's on_node
// block instead of the (off_node) off-process block.
template <typename VT, typename XT>
napspmv::RemoteView<VT, XT> remote_view(const napspmv_plan_s *p, const Schedules &s, const Ws &ws,
                                        const XT *v, XT *w, int64_t blk0, int64_t n_blk,
                                        bool on_node = false) {
    napspmv::RemoteView<VT, XT> R;
    R.n_blocks = (int32_t)n_blk;
    R.rowblk = (on_node ? s.ndblk : s.offblk) + blk0;
    R.blkptr = (on_node ? s.ndptr : s.offptr) + blk0;
    R.rowptr = on_node ? p->d_rp_nd : p->d_rp_off;
    R.col = on_node ? p->d_col_nd : p->d_col_off;
    R.cbase = on_node || !p->d_offbase ? nullptr : p->d_offbase + blk0;
    R.pbase = on_node || !p->d_pbase ? nullptr : p->d_pbase + blk0 * (p->cur_remote_nnz / napspmv::kPackLanes);
    R.col16 = p->d_col16_off;
    R.val = static_cast<const VT *>(on_node ? p->d_val_nd : p->d_val_off);
    R.slot = on_node ? p->d_slot_nd : p->d_slot_off;
    R.ghost = static_cast<const XT *>(p->hp.direct ? ws.recv : ws.ghost);
    R.v = p->hp.direct ? v : nullptr;
    R.w = w;
    R.nt = stream_out(p);
    return R;
}

template <typename XT>
napspmv::ScatterView<XT> scatter_view(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws,
                                      const XT *v, int which) {
    napspmv::ScatterView<XT> S;
    S.items = reinterpret_cast<const int4 *>(sc.sitems);
    S.n_items = (int32_t)sc.n_sitems;
    S.code = p->d_code;
    S.v = v;
    S.recv = static_cast<const XT *>(ws.recv);
    S.ghost = static_cast<XT *>(ws.ghost);
    S.n = (int32_t)p->hp.n;
    S.which = which;
    return S;
}

// ---- single-plan launches ------------------------------------------------------

template <typename VT, typename XT, int CAP, int W>
void launch_local_w(const napspmv::LocalView<VT, XT> &L, hipStream_t s) {
    if (L.n_tasks > 0)
        napspmv::k_local<VT, XT, CAP, W><<<(uint32_t)L.n_tasks, napspmv::kBlock, 0, s>>>(L);
}

template <typename VT, typename XT, int CAP>
void launch_local(int win, const napspmv::LocalView<VT, XT> &L, hipStream_t s) {
    switch (win) {
        case 1024: launch_local_w<VT, XT, CAP, 1024>(L, s); break;
        case 2048: launch_local_w<VT, XT, CAP, 2048>(L, s); break;
        case 4096: launch_local_w<VT, XT, CAP, 4096>(L, s); break;
        default: launch_local_w<VT, XT, CAP, 0>(L, s); break;
    }
}

// The inter-node hop (explicit copy, if any) and the ghost scatter: every
// position (which = 0), only received values (1, with the hop) or only the
// fully local values (2).
template <typename XT, int CAP>
void launch_scatter(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws, const XT *v,
                    hipStream_t s, int which) {
    using namespace napspmv;
    if (which != 2 && p->E > 0 && ws.recv != ws.send)
        k_copy<XT><<<blocks_for(p->E), kBlock, 0, s>>>((int32_t)p->E, static_cast<const XT *>(ws.send),
                                                     static_cast<XT *>(ws.recv));
    if (sc.n_sitems > 0)
        k_scatter<XT, CAP><<<(uint32_t)sc.n_sitems, kBlock, 0, s>>>(scatter_view<XT>(p, sc, ws, v, which));
}

// The off-process product over blocks [blk0, blk0 + n_blk), for the plan's
// remote block size.
template <typename VT, typename XT>
void launch_remote(const napspmv_plan_s *p, const napspmv::RemoteView<VT, XT> &R, hipStream_t s) {
    using namespace napspmv;
    if (R.n_blocks <= 0) return;
    const uint32_t nb = (uint32_t)R.n_blocks;
    switch (p->cur_remote_nnz) {
        case 1024: k_remote<VT, XT, 1024><<<nb, kBlock, 0, s>>>(R); break;
        case 2048: k_remote<VT, XT, 2048><<<nb, kBlock, 0, s>>>(R); break;
        case 4096: k_remote<VT, XT, 4096><<<nb, kBlock, 0, s>>>(R); break;
        default: k_remote<VT, XT, 8192><<<nb, kBlock, 0, s>>>(R); break;
    }
}

// REMOTE stage of a three-way plan (algorithm NAPSpMV): on the caller's
// stream the fully local gathers and the on_node product; meanwhile on the
// helper stream the inter-node hop and the scatter of received values; then,
// joined, the off_node product.
template <typename VT, typename XT, int CAP>
void launch_three_way(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws, const XT *v,
                      XT *w, hipStream_t s) {
    HIP_OK(hipEventRecord(p->ev_fork, s));
    HIP_OK(hipStreamWaitEvent(p->helper, p->ev_fork, 0));
    launch_scatter<XT, CAP>(p, sc, ws, v, p->helper, 1);
    HIP_OK(hipEventRecord(p->ev_join, p->helper));
    if (p->Gon > 0)
        napspmv::k_put<XT><<<blocks_for(p->Gon), napspmv::kBlock, 0, s>>>(
            (int32_t)p->Gon, p->d_l2pos, p->d_l2col, v, static_cast<XT *>(ws.ghost));
    if (sc.n_nd > 0 && p->hp.nnz_nd > 0)
        launch_remote<VT, XT>(p, remote_view<VT, XT>(p, sc, ws, v, w, 0, sc.n_nd, true), s);
    HIP_OK(hipStreamWaitEvent(s, p->ev_join, 0));
    if (p->hp.nnz_off - p->hp.nnz_nd > 0 && sc.n_off > 0)
        launch_remote<VT, XT>(p, remote_view<VT, XT>(p, sc, ws, v, w, 0, sc.n_off), s);
}

template <typename VT, typename XT, int CAP>
void launch_cap(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws, int stage,
                const XT *v, XT *w, hipStream_t s, int64_t task0, int64_t n_tasks, int64_t blk0,
                int64_t n_blk) {
    if (stage == NAPSPMV_STAGE_LOCAL) {
        launch_local<VT, XT, CAP>(p->cur_window, local_view<VT, XT>(p, sc, ws, v, w, task0, n_tasks), s);
        return;
    }
    if (p->hp.three_way) {
        launch_three_way<VT, XT, CAP>(p, sc, ws, v, w, s);
        return;
    }
    if (p->hp.mode == NAPSPMV_NAP) {
        if (p->hp.direct) {
            // direct reads: only the explicit hop, if any; no ghost scatter
            if (p->E > 0 && ws.recv != ws.send)
                napspmv::k_copy<XT><<<blocks_for(p->E), napspmv::kBlock, 0, s>>>(
                    (int32_t)p->E, static_cast<const XT *>(ws.send), static_cast<XT *>(ws.recv));
        } else {
            launch_scatter<XT, CAP>(p, sc, ws, v, s, 0);
        }
    }
    if (p->hp.nnz_off > 0 && n_blk > 0)
        launch_remote<VT, XT>(p, remote_view<VT, XT>(p, sc, ws, v, w, blk0, n_blk), s);
}

template <typename VT, typename XT>
void launch_stage(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws, int stage,
                  const XT *v, XT *w, hipStream_t s, int64_t task0, int64_t n_tasks, int64_t blk0,
                  int64_t n_blk) {
    switch (p->cur_block_nnz) {
        case 1024: launch_cap<VT, XT, 1024>(p, sc, ws, stage, v, w, s, task0, n_tasks, blk0, n_blk); break;
        case 2048: launch_cap<VT, XT, 2048>(p, sc, ws, stage, v, w, s, task0, n_tasks, blk0, n_blk); break;
        case 8192: launch_cap<VT, XT, 8192>(p, sc, ws, stage, v, w, s, task0, n_tasks, blk0, n_blk); break;
        default: launch_cap<VT, XT, 4096>(p, sc, ws, stage, v, w, s, task0, n_tasks, blk0, n_blk); break;
    }
}

// One stage over the task range [task0, task0 + n_tasks) and the
// off-process block range [blk0, blk0 + n_blk) of schedules `sc`.
void run_stage(const napspmv_plan_s *p, const Schedules &sc, const Ws &ws, int stage,
               const void *v, void *w, hipStream_t s, int64_t task0, int64_t n_tasks, int64_t blk0,
               int64_t n_blk) {
    switch (p->hp.dtype) {
        case NAPSPMV_F64:
            launch_stage<double, double>(p, sc, ws, stage, static_cast<const double *>(v),
                                         static_cast<double *>(w), s, task0, n_tasks, blk0, n_blk);
            break;
        case NAPSPMV_F32:
            launch_stage<float, float>(p, sc, ws, stage, static_cast<const float *>(v),
                                       static_cast<float *>(w), s, task0, n_tasks, blk0, n_blk);
            break;
        default:
            launch_stage<uint16_t, float>(p, sc, ws, stage, static_cast<const float *>(v),
                                          static_cast<float *>(w), s, task0, n_tasks, blk0, n_blk);
            break;
    }
    HIP_OK(hipGetLastError());
}

void run_apply(const napspmv_plan_s *p, const Ws &ws, const void *v, void *w, hipStream_t s) {
    const Schedules &sc = p->sched;
    run_stage(p, sc, ws, NAPSPMV_STAGE_LOCAL, v, w, s, 0, sc.n_tasks, 0, sc.n_off);
    run_stage(p, sc, ws, NAPSPMV_STAGE_REMOTE, v, w, s, 0, sc.n_tasks, 0, sc.n_off);
}

int check_vectors(napspmv_plan_t plan, const void *v, void *w) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    if (!v || !w) return fail(NAPSPMV_EINVAL, "v or w is NULL");
    const int64_t bytes = plan->hp.n * vec_bytes(plan->hp.dtype);
    const char *a = static_cast<const char *>(v);
    const char *b = static_cast<const char *>(w);
    if (a < b + bytes && b < a + bytes) return fail(NAPSPMV_EINVAL, "v and w overlap");
    return NAPSPMV_OK;
}

int check_ws(const void *ws) {
    if (ws && (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return fail(NAPSPMV_EINVAL, "workspace must be 256-byte aligned");
    return NAPSPMV_OK;
}

void fill_stats(const napspmv_plan_s *p, napspmv_stats_t *s) {
    const HostPlan &hp = p->hp;
    std::memset(s, 0, sizeof(*s));
    s->n = hp.n;
    s->nnz = hp.nnz;
    s->n_p = hp.n_p;
    s->ppn = hp.ppn;
    s->n_nodes = hp.n_nodes;
    s->mode = hp.mode;
    s->dtype = hp.dtype;
    s->value_bytes = vec_bytes(hp.dtype);
    s->nnz_on = hp.nnz_on;
    s->nnz_off = hp.nnz_off;
    s->ghosts = hp.ghost_ptr.empty() ? 0 : hp.ghost_ptr.back();
    for (int ph = 0; ph < 4; ++ph) {
        const napspmv::PhaseStats &q = hp.stats[ph];
        s->phase[ph] = napspmv_phase_stats_t{q.msgs, q.elems, q.max_msgs_sent, q.max_elems_sent,
                                             q.max_msgs_recv, q.max_elems_recv, q.max_msg_elems};
    }
    s->device_bytes = p->device_bytes;
    s->build_seconds = p->build_s;
    s->upload_seconds = p->upload_s;
    s->flags = p->flags;
}

// ---- batched launches -----------------------------------------------------------

// Descriptor table of a batch: the block prefix arrays of the three
// launches, then one view per product for each launch, each part 256-byte
// aligned.
struct BatchTable {
    size_t pre_local = 0, pre_scatter = 0, pre_remote = 0, local = 0, scatter = 0, remote = 0, total = 0;
};

template <typename VT, typename XT>
BatchTable batch_table(int count) {
    BatchTable t;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (size_t)align_up((int64_t)(off + bytes));
        return at;
    };
    t.pre_local = take(sizeof(int32_t) * (count + 1));
    t.pre_scatter = take(sizeof(int32_t) * (count + 1));
    // the remote views are grouped by block size, one prefix list per group
    t.pre_remote = take(sizeof(int32_t) * (count + kRemoteSizes));
    t.local = take(sizeof(napspmv::LocalView<VT, XT>) * count);
    t.scatter = take(sizeof(napspmv::ScatterView<XT>) * count);
    t.remote = take(sizeof(napspmv::RemoteView<VT, XT>) * count);
    t.total = off;
    return t;
}

size_t batch_bytes(int count) {
    return std::max(batch_table<double, double>(count).total,
                    std::max(batch_table<float, float>(count).total,
                             batch_table<uint16_t, float>(count).total));
}

template <typename VT, typename XT, int CAP, int W>
void batch_launch(napspmv_batch_s *B, int count, const napspmv_plan_t *plans, void *const *ws,
                  const void *const *v, void *const *w, hipStream_t s) {
    using namespace napspmv;
    const BatchTable t = batch_table<VT, XT>(count);
    char *h = static_cast<char *>(B->h_desc[B->next]);
    char *d = static_cast<char *>(B->d_desc[B->next]);
    int32_t *pl = reinterpret_cast<int32_t *>(h + t.pre_local);
    int32_t *ps = reinterpret_cast<int32_t *>(h + t.pre_scatter);
    int32_t *pr = reinterpret_cast<int32_t *>(h + t.pre_remote);
    // remote views grouped by block size: group g holds views [g0[g], g0[g+1])
    // and its prefix list starts at pr[g0[g] + g]
    int g0[kRemoteSizes + 1] = {0};
    for (int i = 0; i < count; ++i) ++g0[remote_size_index(plans[i]->cur_remote_nnz) + 1];
    for (int g = 0; g < kRemoteSizes; ++g) g0[g + 1] += g0[g];
    int fill[kRemoteSizes];
    for (int g = 0; g < kRemoteSizes; ++g) {
        fill[g] = g0[g];
        pr[g0[g] + g] = 0;
    }
    auto *lv = reinterpret_cast<LocalView<VT, XT> *>(h + t.local);
    auto *sv = reinterpret_cast<ScatterView<XT> *>(h + t.scatter);
    auto *rv = reinterpret_cast<RemoteView<VT, XT> *>(h + t.remote);
    pl[0] = ps[0] = 0;
    bool any_nap = false;
    for (int i = 0; i < count; ++i) {
        const napspmv_plan_s *p = plans[i];
        const Ws wp = ws_ptrs(p, ws && ws[i] ? ws[i] : p->d_ws);
        lv[i] = local_view<VT, XT>(p, p->sched, wp, static_cast<const XT *>(v[i]),
                                   static_cast<XT *>(w[i]), 0, p->sched.n_tasks);
        sv[i] = scatter_view<XT>(p, p->sched, wp, static_cast<const XT *>(v[i]), 0);
        const int g = remote_size_index(p->cur_remote_nnz), j = fill[g]++;
        rv[j] = remote_view<VT, XT>(p, p->sched, wp, static_cast<const XT *>(v[i]),
                                    static_cast<XT *>(w[i]), 0,
                                    p->hp.nnz_off > 0 ? p->sched.n_off : 0);
        pr[j + g + 1] = pr[j + g] + rv[j].n_blocks;
        const bool nap = p->hp.mode == NAPSPMV_NAP;
        any_nap = any_nap || nap;
        pl[i + 1] = pl[i] + lv[i].n_tasks;
        ps[i + 1] = ps[i] + (nap && !p->hp.direct ? (int32_t)p->sched.n_sitems : 0);
    }
    HIP_OK(hipMemcpyAsync(d, h, t.total, hipMemcpyHostToDevice, s));
    if (pl[count] > 0)
        k_local_batch<VT, XT, CAP, W><<<(uint32_t)pl[count], kBlock, 0, s>>>(
            reinterpret_cast<const LocalView<VT, XT> *>(d + t.local),
            reinterpret_cast<const int32_t *>(d + t.pre_local), count);
    if (any_nap && ps[count] > 0)
        k_scatter_batch<XT, CAP><<<(uint32_t)ps[count], kBlock, 0, s>>>(
            reinterpret_cast<const ScatterView<XT> *>(d + t.scatter),
            reinterpret_cast<const int32_t *>(d + t.pre_scatter), count);
    for (int g = 0; g < kRemoteSizes; ++g) {
        const int n_g = g0[g + 1] - g0[g];
        if (n_g == 0 || pr[g0[g + 1] + g] == 0) continue;
        const auto *rvd = reinterpret_cast<const RemoteView<VT, XT> *>(d + t.remote) + g0[g];
        const auto *prd = reinterpret_cast<const int32_t *>(d + t.pre_remote) + g0[g] + g;
        const uint32_t nb = (uint32_t)pr[g0[g + 1] + g];
        switch (g) {
            case 0: k_remote_batch<VT, XT, 1024><<<nb, kBlock, 0, s>>>(rvd, prd, n_g); break;
            case 1: k_remote_batch<VT, XT, 2048><<<nb, kBlock, 0, s>>>(rvd, prd, n_g); break;
            case 2: k_remote_batch<VT, XT, 4096><<<nb, kBlock, 0, s>>>(rvd, prd, n_g); break;
            default: k_remote_batch<VT, XT, 8192><<<nb, kBlock, 0, s>>>(rvd, prd, n_g); break;
        }
    }
    HIP_OK(hipGetLastError());
}

template <typename VT, typename XT, int CAP>
void batch_launch_cap(int win, napspmv_batch_s *B, int count, const napspmv_plan_t *plans,
                      void *const *ws, const void *const *v, void *const *w, hipStream_t s) {
    switch (win) {
        case 1024: batch_launch<VT, XT, CAP, 1024>(B, count, plans, ws, v, w, s); break;
        case 2048: batch_launch<VT, XT, CAP, 2048>(B, count, plans, ws, v, w, s); break;
        case 4096: batch_launch<VT, XT, CAP, 4096>(B, count, plans, ws, v, w, s); break;
        default: batch_launch<VT, XT, CAP, 0>(B, count, plans, ws, v, w, s); break;
    }
}

template <typename VT, typename XT>
void batch_launch_t(int cap, int win, napspmv_batch_s *B, int count, const napspmv_plan_t *plans,
                    void *const *ws, const void *const *v, void *const *w, hipStream_t s) {
    switch (cap) {
        case 1024: batch_launch_cap<VT, XT, 1024>(win, B, count, plans, ws, v, w, s); break;
        case 2048: batch_launch_cap<VT, XT, 2048>(win, B, count, plans, ws, v, w, s); break;
        case 8192: batch_launch_cap<VT, XT, 8192>(win, B, count, plans, ws, v, w, s); break;
        default: batch_launch_cap<VT, XT, 4096>(win, B, count, plans, ws, v, w, s); break;
    }
}

// ---- autotuner --------------------------------------------------------------------

std::mutex g_tune_mutex;

// Cache key: the device and the workload's shape (not its values).
std::string tune_key(const napspmv_plan_s *p) {
    hipDeviceProp_t prop;
    std::string dev = "gpu";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = prop.gcnArchName;
    std::ostringstream k;
    k << dev << ";n=" << p->hp.n << ";nnz=" << p->hp.nnz << ";np=" << p->hp.n_p << ";ppn="
      << p->hp.ppn << ";mode=" << p->hp.mode << ";dtype=" << p->hp.dtype << ";G=" << p->G
      << ";on=" << p->hp.nnz_on << ";three_way=" << (p->hp.three_way ? 1 : 0)
      << ";direct=" << (p->hp.direct ? 1 : 0) << ";v=2";
    std::string s = k.str();
    std::replace(s.begin(), s.end(), ' ', '_');
    return s;
}

// Cache lines: key, BLOCK_NNZ, VWINDOW, GATHER_ITEM, REMOTE_NNZ, best ms.
bool cache_lookup(const char *path, const std::string &key, int out[4]) {
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        int a, b, c, d;
        if (in >> k >> a >> b >> c >> d && k == key) {
            out[0] = a;
            out[1] = b;
            out[2] = c;
            out[3] = d;
            found = true;       // the last entry of a key wins
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const int v[4], double ms) {
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    std::ofstream f(path, std::ios::app);
    f << key << ' ' << v[0] << ' ' << v[1] << ' ' << v[2] << ' ' << v[3] << ' ' << ms << '\n';
}

bool valid_cfg(const int c[4]) {
    return valid_block(c[0]) && valid_block(c[3]) &&
           (c[1] == 0 || c[1] == 1024 || c[1] == 2048 || c[1] == 4096) && c[2] >= kMinItem &&
           c[2] <= kMaxItem;
}

// ---- the allocation-free apply ---------------------------------------------------

// Workspace of napspmv_apply_noalloc: one array per GPU, held by the loaded
// code object until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host the name stands for a host-side shadow, not
// a device address): it passes the device address hipGetSymbolAddress gives
// for the current GPU.
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on GPU `dev` (current), looked up on the
// first call for that GPU.
void *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw Error(NAPSPMV_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) % kAlign) != 0)
            throw Error(NAPSPMV_EHIP, "scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int plan_create(const int64_t *rowptr, const int32_t *col, const void *val, int dtype, int64_t n,
                int64_t n_p, int64_t ppn, int mode, int64_t pps, const int64_t *row_starts,
                uint32_t flags, napspmv_plan_t *plan_out, napspmv_stats_t *stats_out) {
    if (!plan_out) return fail(NAPSPMV_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    if (flags & ~(NAPSPMV_HOST_ONLY | NAPSPMV_EXCHANGE_COPY | NAPSPMV_NAP_OWNER_MAP |
                  NAPSPMV_NAP_SPLIT | NAPSPMV_NAP_DEDUP | NAPSPMV_NAP_THREE_WAY |
                  NAPSPMV_NAP_DIRECT | NAPSPMV_PARTITION_STRIDED))
        return fail(NAPSPMV_EINVAL, "unknown flag bits");
    if (pps != 0 && (flags & NAPSPMV_EXCHANGE_COPY))
        return fail(NAPSPMV_EINVAL, "the socket level receives the inter-node messages in place");
    napspmv_plan_s *p = nullptr;
    const int rc = guarded([&]() {
        p = new napspmv_plan_s();
        p->flags = flags;
        const auto t0 = std::chrono::steady_clock::now();
        napspmv::build_plan(p->hp, rowptr, col, val, dtype, n, n_p, ppn, mode, row_starts,
                            flags & (NAPSPMV_NAP_OWNER_MAP | NAPSPMV_NAP_SPLIT | NAPSPMV_NAP_DEDUP |
                                     NAPSPMV_NAP_THREE_WAY | NAPSPMV_NAP_DIRECT),
                            (flags & NAPSPMV_PARTITION_STRIDED) != 0, pps);
        const auto t1 = std::chrono::steady_clock::now();
        p->build_s = std::chrono::duration<double>(t1 - t0).count();
        p->G = p->hp.ghost_ptr.back();
        p->E = (int64_t)p->hp.pack_idx.size();
        p->E1 = (int64_t)p->hp.l1x_col.size();
        p->H = (int64_t)p->hp.scat_src.size();
        p->Gon = (int64_t)p->hp.l2_src.size();
        // automatic off-process block size: the larger block lets a
        // process's blocks share more ghost lines, but a process with fewer
        // off-process entries than it holds would leave half of its LDS idle
        p->auto_remote_nnz = p->hp.nnz_off >= (int64_t)8192 * p->hp.n_p ? 8192 : 4096;
        // automatic on-process block size: 2048 entries for float32 and
        // bfloat16 values (their bands still hold 16 KB of v) -- shorter
        // blocks hold fewer registers and keep more of them in flight per
        // CU; float64 blocks of 4096 entries
        p->auto_block_nnz = p->hp.dtype == NAPSPMV_F64 ? 4096 : 2048;
        if (!(flags & NAPSPMV_HOST_ONLY)) {
            to_device(p);
            napspmv::release_device_arrays(p->hp);
            p->upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
        }
        if (stats_out) fill_stats(p, stats_out);
        *plan_out = p;
        g_last_error.clear();
        return NAPSPMV_OK;
    });
    if (rc != NAPSPMV_OK) delete p;
    return rc;
}

}  // namespace

extern "C" {

int napspmv_plan_create(const int64_t *rowptr, const int32_t *col, const void *val, int dtype,
                        int64_t n, int64_t n_p, int64_t ppn, int mode, const int64_t *row_starts,
                        uint32_t flags, napspmv_plan_t *plan_out, napspmv_stats_t *stats_out) {
    return plan_create(rowptr, col, val, dtype, n, n_p, ppn, mode, 0, row_starts, flags, plan_out,
                       stats_out);
}

int napspmv_plan_create_sockets(const int64_t *rowptr, const int32_t *col, const void *val,
                                int dtype, int64_t n, int64_t n_p, int64_t ppn,
                                int64_t procs_per_socket, const int64_t *row_starts, uint32_t flags,
                                napspmv_plan_t *plan_out, napspmv_stats_t *stats_out) {
    if (procs_per_socket < 1) {
        if (plan_out) *plan_out = nullptr;
        return fail(NAPSPMV_EINVAL, "procs_per_socket must be at least 1");
    }
    return plan_create(rowptr, col, val, dtype, n, n_p, ppn, NAPSPMV_NAP, procs_per_socket,
                       row_starts, flags, plan_out, stats_out);
}

int napspmv_plan_socket_stats(napspmv_plan_t plan, int64_t *procs_per_socket,
                              napspmv_phase_stats_t *out) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (procs_per_socket) *procs_per_socket = plan->hp.pps;
    if (out) {
        if (plan->hp.pps == 0) return fail(NAPSPMV_EINVAL, "the plan has no socket level");
        for (int k = 0; k < 12; ++k) {
            const napspmv::PhaseStats &q = plan->hp.sock_stats[k];
            out[k] = napspmv_phase_stats_t{q.msgs, q.elems, q.max_msgs_sent, q.max_elems_sent,
                                           q.max_msgs_recv, q.max_elems_recv, q.max_msg_elems};
        }
    }
    return NAPSPMV_OK;
}

int napspmv_apply_stage(napspmv_plan_t plan, int stage, const void *v, void *w, void *stream) {
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    if (stage != NAPSPMV_STAGE_LOCAL && stage != NAPSPMV_STAGE_REMOTE)
        return fail(NAPSPMV_EINVAL, "unknown stage");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        const Schedules &sc = plan->sched;
        run_stage(plan, sc, ws_ptrs(plan, plan->d_ws), stage, v, w,
                  static_cast<hipStream_t>(stream), 0, sc.n_tasks, 0, sc.n_off);
        return NAPSPMV_OK;
    });
}

int napspmv_apply_ws(napspmv_plan_t plan, void *ws, const void *v, void *w, void *stream) {
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    if ((rc = check_ws(ws))) return rc;
    return guarded([&]() {
        DeviceGuard g(plan->device);
        run_apply(plan, ws_ptrs(plan, ws ? ws : plan->d_ws), v, w, static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    });
}

int napspmv_apply(napspmv_plan_t plan, const void *v, void *w, void *stream) {
    return napspmv_apply_ws(plan, nullptr, v, w, stream);
}

int64_t napspmv_noalloc_max_workspace_bytes(void) { return kScratchBytes; }

int napspmv_apply_noalloc(napspmv_plan_t plan, const void *v, void *w, void *stream) {
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    const int64_t need = ws_layout(plan).total;
    if (need > kScratchBytes)
        return fail(NAPSPMV_EUNSUPPORTED,
                    "napspmv_apply_noalloc: the plan needs a workspace of " + std::to_string(need) +
                        " bytes, more than the " + std::to_string(kScratchBytes) +
                        " bytes of the static workspace");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        // every apply writes each ghost and send position before it reads it,
        // so nothing left in the array by an earlier call needs clearing
        run_apply(plan, ws_ptrs(plan, scratch_address(plan->device)), v, w,
                  static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    });
}

int64_t napspmv_plan_workspace_bytes(napspmv_plan_t plan) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    return ws_layout(plan).total;
}

int napspmv_plan_prepare_partitions(napspmv_plan_t plan) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    if (plan->hp.mode != NAPSPMV_STANDARD)
        return fail(NAPSPMV_EUNSUPPORTED, "per-partition applies need a standard-mode plan");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        if (!plan->part_ready) build_partitions(plan);
        HIP_OK(hipDeviceSynchronize());
        return NAPSPMV_OK;
    });
}

int napspmv_apply_partition(napspmv_plan_t plan, int64_t part, const void *v, void *w,
                            void *stream) {
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    if (!plan->part_ready) return fail(NAPSPMV_EINVAL, "call napspmv_plan_prepare_partitions first");
    if (part < 0 || part >= plan->hp.n_p) return fail(NAPSPMV_EINVAL, "partition out of range");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        const Schedules &sc = plan->part;
        const Ws wp = ws_ptrs(plan, plan->d_ws);
        const int64_t t0 = sc.task_ptr[part], t1 = sc.task_ptr[part + 1];
        const int64_t b0 = sc.off_ptr[part], b1 = sc.off_ptr[part + 1];
        hipStream_t s = static_cast<hipStream_t>(stream);
        run_stage(plan, sc, wp, NAPSPMV_STAGE_LOCAL, v, w, s, t0, t1 - t0, b0, b1 - b0);
        run_stage(plan, sc, wp, NAPSPMV_STAGE_REMOTE, v, w, s, t0, t1 - t0, b0, b1 - b0);
        return NAPSPMV_OK;
    });
}

int napspmv_batch_create(int max_count, napspmv_batch_t *out) {
    if (!out) return fail(NAPSPMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_count < 1 || max_count > (1 << 20)) return fail(NAPSPMV_EINVAL, "max_count out of range");
    napspmv_batch_s *b = nullptr;
    const int rc = guarded([&]() {
        b = new napspmv_batch_s();
        b->capacity = max_count;
        HIP_OK(hipGetDevice(&b->device));
        b->desc_bytes = batch_bytes(max_count);
        for (int k = 0; k < kBatchRing; ++k) {
            HIP_OK(hipMalloc(&b->d_desc[k], b->desc_bytes));
            HIP_OK(hipHostMalloc(&b->h_desc[k], b->desc_bytes, hipHostMallocDefault));
            HIP_OK(hipEventCreateWithFlags(&b->done[k], hipEventDisableTiming));
        }
        *out = b;
        return NAPSPMV_OK;
    });
    if (rc != NAPSPMV_OK && b) napspmv_batch_destroy(b);
    return rc;
}

int napspmv_batch_apply(napspmv_batch_t batch, int count, const napspmv_plan_t *plans,
                        void *const *ws, const void *const *v, void *const *w, void *stream) {
    if (!batch || !plans || !v || !w) return fail(NAPSPMV_EINVAL, "NULL argument");
    if (count < 1 || count > batch->capacity) return fail(NAPSPMV_EINVAL, "count out of range");
    const napspmv_plan_s *p0 = plans[0];
    for (int i = 0; i < count; ++i) {
        int rc = check_vectors(plans[i], v[i], w[i]);
        if (rc) return rc;
        if ((rc = check_ws(ws ? ws[i] : nullptr))) return rc;
        const napspmv_plan_s *p = plans[i];
        if (p->device != batch->device) return fail(NAPSPMV_EINVAL, "plans on different devices");
        if (p->hp.dtype != p0->hp.dtype || p->cur_block_nnz != p0->cur_block_nnz ||
            p->cur_window != p0->cur_window)
            return fail(NAPSPMV_EINVAL, "a batch needs one value type, BLOCK_NNZ and VWINDOW");
        if (p->hp.mode == NAPSPMV_NAP && (p->flags & NAPSPMV_EXCHANGE_COPY))
            return fail(NAPSPMV_EUNSUPPORTED, "batched applies receive NAP messages in place");
        if (p->hp.three_way)
            return fail(NAPSPMV_EUNSUPPORTED, "batched applies use the two-part product");
    }
    return guarded([&]() {
        DeviceGuard g(batch->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // the ring's next table is reused: the call that last filled it must
        // have been read by the device
        const int k = batch->next;
        if (batch->pending[k]) HIP_OK(hipEventSynchronize(batch->done[k]));
        switch (p0->hp.dtype) {
            case NAPSPMV_F64:
                batch_launch_t<double, double>(p0->cur_block_nnz, p0->cur_window, batch, count,
                                               plans, ws, v, w, s);
                break;
            case NAPSPMV_F32:
                batch_launch_t<float, float>(p0->cur_block_nnz, p0->cur_window, batch, count,
                                             plans, ws, v, w, s);
                break;
            default:
                batch_launch_t<uint16_t, float>(p0->cur_block_nnz, p0->cur_window, batch, count,
                                                plans, ws, v, w, s);
                break;
        }
        HIP_OK(hipEventRecord(batch->done[k], s));
        batch->pending[k] = true;
        batch->next = (k + 1) % kBatchRing;
        return NAPSPMV_OK;
    });
}

int napspmv_batch_destroy(napspmv_batch_t batch) {
    if (!batch) return NAPSPMV_OK;
    try {
        DeviceGuard g(batch->device);
        for (int k = 0; k < kBatchRing; ++k) {
            if (batch->pending[k]) (void)hipEventSynchronize(batch->done[k]);
            if (batch->done[k]) (void)hipEventDestroy(batch->done[k]);
            if (batch->d_desc[k]) (void)hipFree(batch->d_desc[k]);
            if (batch->h_desc[k]) (void)hipHostFree(batch->h_desc[k]);
        }
    } catch (const Error &) {
    }
    delete batch;
    return NAPSPMV_OK;
}

int napspmv_graph_create(napspmv_plan_t plan, const void *v, void *w, void **graph_out) {
    if (!graph_out) return fail(NAPSPMV_EINVAL, "graph_out is NULL");
    *graph_out = nullptr;
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    return guarded([&]() {
        DeviceGuard g(plan->device);
        hipStream_t s = nullptr;
        HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        try {
            HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                run_apply(plan, ws_ptrs(plan, plan->d_ws), v, w, s);
            } catch (...) {
                (void)hipStreamEndCapture(s, &graph);
                throw;
            }
            HIP_OK(hipStreamEndCapture(s, &graph));
            HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        } catch (...) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipStreamDestroy(s);
            throw;
        }
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(s);
        *graph_out = exec;
        return NAPSPMV_OK;
    });
}

int napspmv_graph_launch(void *graph, void *stream) {
    if (!graph) return fail(NAPSPMV_EINVAL, "graph is NULL");
    return guarded([&]() {
        HIP_OK(hipGraphLaunch(static_cast<hipGraphExec_t>(graph), static_cast<hipStream_t>(stream)));
        return NAPSPMV_OK;
    });
}

int napspmv_graph_destroy(void *graph) {
    if (graph) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph));
    return NAPSPMV_OK;
}

int napspmv_plan_autotune(napspmv_plan_t plan, const void *v, void *w, void *stream, int reps,
                          const char *cache_path, double *best_ms) {
    int rc = check_vectors(plan, v, w);
    if (rc) return rc;
    if (reps < 1) reps = 5;
    return guarded([&]() {
        DeviceGuard g(plan->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const std::string key = tune_key(plan);
        int cfg[4];
        if (cache_lookup(cache_path, key, cfg) && valid_cfg(cfg)) {
            plan->block_nnz = cfg[0];
            plan->window = cfg[1];
            plan->item = cfg[2];
            plan->remote_nnz = cfg[3];
            refresh_schedules(plan);
            HIP_OK(hipDeviceSynchronize());
            if (best_ms) *best_ms = -1.0;
            return NAPSPMV_OK;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        double best = 1e30;
        int best_cfg[4] = {cur_cap(plan), cur_win(plan), cur_item(plan), cur_rcap(plan)};
        auto trial = [&](int cap, int win, int item, int rcap) {
            plan->block_nnz = cap;
            plan->window = win;
            plan->item = item;
            plan->remote_nnz = rcap;
            refresh_schedules(plan);
            const Ws wp = ws_ptrs(plan, plan->d_ws);
            run_apply(plan, wp, v, w, s);            // warm-up
            HIP_OK(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run_apply(plan, wp, v, w, s);
            HIP_OK(hipEventRecord(e1, s));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / reps;
            if (per < best) {
                best = per;
                best_cfg[0] = cap;
                best_cfg[1] = win;
                best_cfg[2] = item;
                best_cfg[3] = rcap;
            }
        };
        try {
            // the first launch's parameters with the remote block size held,
            // then the remote block size alone
            const int rcap0 = best_cfg[3];
            for (int cap : {1024, 2048, 4096, 8192})
                for (int win : {0, 1024, 2048, 4096})
                    for (int item : {16384, 65536}) trial(cap, win, item, rcap0);
            const int c0 = best_cfg[0], w0 = best_cfg[1], i0 = best_cfg[2];
            for (int rcap : {1024, 2048, 4096, 8192})
                if (rcap != rcap0) trial(c0, w0, i0, rcap);
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan->block_nnz = best_cfg[0];
        plan->window = best_cfg[1];
        plan->item = best_cfg[2];
        plan->remote_nnz = best_cfg[3];
        refresh_schedules(plan);
        HIP_OK(hipDeviceSynchronize());
        cache_store(cache_path, key, best_cfg, best);
        if (best_ms) *best_ms = best;
        return NAPSPMV_OK;
    });
}

int napspmv_plan_level_stats(napspmv_plan_t plan, int64_t procs_per_socket,
                             napspmv_phase_stats_t *out) {
    if (!plan || !out) return fail(NAPSPMV_EINVAL, "plan or out is NULL");
    if (procs_per_socket < 1 || plan->hp.ppn % procs_per_socket != 0)
        return fail(NAPSPMV_EINVAL, "procs_per_socket must divide ppn");
    return guarded([&]() {
        napspmv::PhaseStats st[8];
        napspmv::level_stats(plan->hp, procs_per_socket, st);
        for (int k = 0; k < 8; ++k)
            out[k] = napspmv_phase_stats_t{st[k].msgs, st[k].elems, st[k].max_msgs_sent,
                                           st[k].max_elems_sent, st[k].max_msgs_recv,
                                           st[k].max_elems_recv, st[k].max_msg_elems};
        return NAPSPMV_OK;
    });
}

int napspmv_plan_rows(napspmv_plan_t plan, int64_t *rows_out) {
    if (!plan || !rows_out) return fail(NAPSPMV_EINVAL, "plan or rows_out is NULL");
    const HostPlan &hp = plan->hp;
    if (hp.strided)
        for (int64_t k = 0; k < hp.n; ++k) rows_out[k] = hp.rows_natural[k];
    else
        for (int64_t k = 0; k < hp.n; ++k) rows_out[k] = k;
    return NAPSPMV_OK;
}

int napspmv_plan_block_kinds(napspmv_plan_t plan, int64_t *kinds_out) {
    if (!plan || !kinds_out) return fail(NAPSPMV_EINVAL, "plan or kinds_out is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "host-only plan");
    for (int i = 0; i < 3; ++i) kinds_out[i] = plan->block_kinds[i];
    return NAPSPMV_OK;
}

int napspmv_plan_stats(napspmv_plan_t plan, napspmv_stats_t *out) {
    if (!plan || !out) return fail(NAPSPMV_EINVAL, "plan or out is NULL");
    fill_stats(plan, out);
    return NAPSPMV_OK;
}

int napspmv_plan_export(napspmv_plan_t plan, int phase, int64_t *n_msgs, int64_t *n_idx,
                        int32_t *src, int32_t *dst, int64_t *ptr, int32_t *idx) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (phase < 0 || phase > 15) return fail(NAPSPMV_EINVAL, "unknown phase");
    if (phase > 3 && plan->hp.pps == 0) return fail(NAPSPMV_EINVAL, "the plan has no socket level");
    const napspmv::Phase &ph = phase < 4 ? plan->hp.phase[phase] : plan->hp.sock_phase[phase - 4];
    if (n_msgs) *n_msgs = (int64_t)ph.src.size();
    if (n_idx) *n_idx = ph.ptr.back();
    if (src) std::copy(ph.src.begin(), ph.src.end(), src);
    if (dst) std::copy(ph.dst.begin(), ph.dst.end(), dst);
    if (ptr) std::copy(ph.ptr.begin(), ph.ptr.end(), ptr);
    if (idx) std::copy(ph.idx.begin(), ph.idx.end(), idx);
    return NAPSPMV_OK;
}

int napspmv_plan_ghosts(napspmv_plan_t plan, int64_t *ghost_ptr, int32_t *ghost_col) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (ghost_ptr) std::copy(plan->hp.ghost_ptr.begin(), plan->hp.ghost_ptr.end(), ghost_ptr);
    if (ghost_col) std::copy(plan->hp.ghost_col.begin(), plan->hp.ghost_col.end(), ghost_col);
    return NAPSPMV_OK;
}

int napspmv_plan_read_ghost_values(napspmv_plan_t plan, const void *ws, void *out, void *stream) {
    if (!plan || !out) return fail(NAPSPMV_EINVAL, "plan or out is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    if (plan->hp.direct)
        return fail(NAPSPMV_EUNSUPPORTED, "a direct-read plan fills no ghost buffer");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
        const Ws wp = ws_ptrs(plan, ws ? const_cast<void *>(ws) : plan->d_ws);
        if (plan->G > 0) {
            // device positions are band-ordered: return the plan's ghost order
            const int64_t vb = vec_bytes(plan->hp.dtype);
            std::vector<uint8_t> dev((size_t)(plan->Gdev * vb));
            HIP_OK(hipMemcpy(dev.data(), wp.ghost, dev.size(), hipMemcpyDeviceToHost));
            uint8_t *o = static_cast<uint8_t *>(out);
            for (int64_t k = 0; k < plan->G; ++k)
                std::memcpy(o + k * vb, dev.data() + (int64_t)plan->gpos[k] * vb, (size_t)vb);
        }
        return NAPSPMV_OK;
    });
}

int napspmv_plan_set_param(napspmv_plan_t plan, int param, int value) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    switch (param) {
        case NAPSPMV_PARAM_BLOCK_NNZ:
            if (value != -1 && !valid_block(value))
                return fail(NAPSPMV_EINVAL, "block entries must be -1, 1024, 2048, 4096 or 8192");
            plan->block_nnz = value;
            break;
        case NAPSPMV_PARAM_REMOTE_NNZ:
            if (value != -1 && !valid_block(value))
                return fail(NAPSPMV_EINVAL, "remote block entries must be -1, 1024, 2048, 4096 or 8192");
            plan->remote_nnz = value;
            break;
        case NAPSPMV_PARAM_GATHER_ITEM:
            if (value != -1 && (value < kMinItem || value > kMaxItem))
                return fail(NAPSPMV_EINVAL, "gather item must be -1 or in [256, 2^24]");
            plan->item = value;
            break;
        case NAPSPMV_PARAM_VWINDOW:
            if (value != -1 && value != 0 && value != 1024 && value != 2048 && value != 4096)
                return fail(NAPSPMV_EINVAL, "window must be -1, 0, 1024, 2048 or 4096");
            plan->window = value;
            break;
        default:
            return fail(NAPSPMV_EINVAL, "unknown parameter");
    }
    if (!plan->on_device) return NAPSPMV_OK;
    return guarded([&]() {
        DeviceGuard g(plan->device);
        HIP_OK(hipDeviceSynchronize());
        refresh_schedules(plan);
        HIP_OK(hipDeviceSynchronize());
        return NAPSPMV_OK;
    });
}

int napspmv_plan_get_param(napspmv_plan_t plan, int param) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    switch (param) {
        case NAPSPMV_PARAM_BLOCK_NNZ: return cur_cap(plan);
        case NAPSPMV_PARAM_REMOTE_NNZ: return cur_rcap(plan);
        case NAPSPMV_PARAM_GATHER_ITEM: return cur_item(plan);
        case NAPSPMV_PARAM_VWINDOW: return cur_win(plan);
        default: return fail(NAPSPMV_EINVAL, "unknown parameter");
    }
}

int napspmv_plan_destroy(napspmv_plan_t plan) {
    if (!plan) return NAPSPMV_OK;
    if (plan->on_device) {
        try {
            DeviceGuard g(plan->device);
            free_device(plan);
        } catch (const Error &) {
            free_device(plan);
        }
    }
    delete plan;
    return NAPSPMV_OK;
}

int napspmv_set_device_budget(int64_t bytes) {
    if (bytes < 0) return fail(NAPSPMV_EINVAL, "budget must be >= 0");
    g_budget = bytes;
    return NAPSPMV_OK;
}

int64_t napspmv_device_bytes_in_use(void) { return g_in_use.load(); }

const char *napspmv_last_error(void) { return g_last_error.c_str(); }

int napspmv_version(void) { return 100; }

}  // extern "C"
