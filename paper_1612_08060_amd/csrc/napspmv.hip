// The C ABI of include/napspmv.h: plan creation (host builder + device
// upload), the apply path (exchange kernels + split product), tuning and
// diagnostics.  Nothing here throws across the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <new>
#include <string>

#include "kernels.hpp"
#include "napspmv.h"
#include "plan_build.hpp"
#include "schedule.hpp"

using napspmv::Error;
using napspmv::HostPlan;

namespace {
constexpr int kMaxItem = 4096;          // gather work item length
constexpr int kMaxRowsPerBlock = napspmv::kMaxRows;  // rows of a product block
}  // namespace

struct napspmv_plan_s {
    HostPlan hp;
    uint32_t flags = 0;
    bool on_device = false;
    int device = 0;
    // tuning (-1 = automatic)
    int block_nnz = -1, bands = -1, window = -1;
    int auto_block_nnz = 4096, auto_bands = 1, auto_window = 1024;
    int cur_block_nnz = 0, cur_bands = 0, cur_window = -1;   // schedules on the device
    int64_t G = 0, E = 0, H = 0, Gon = 0;
    int64_t n_on_blocks = 0, n_off_blocks = 0, n_items = 0, n_tasks = 0;
    int32_t *d_rp_on = nullptr, *d_col_on = nullptr, *d_rp_off = nullptr, *d_col_off = nullptr;
    void *d_val_on = nullptr, *d_val_off = nullptr;
    void *d_ghost = nullptr;
    int32_t *d_gather = nullptr, *d_pack = nullptr;
    void *d_send = nullptr, *d_recv = nullptr;
    int32_t *d_ssrc = nullptr, *d_sdst = nullptr, *d_lsrc = nullptr, *d_ldst = nullptr;
    // schedules: on-process row blocks + windows, off-process row blocks,
    // exchange items, the merged task list of the first launch
    int32_t *d_onblk = nullptr, *d_onptr = nullptr, *d_win = nullptr;
    int32_t *d_offblk = nullptr, *d_offptr = nullptr, *d_items = nullptr, *d_tasks = nullptr;
    int64_t bytes_sched = 0;
    int64_t device_bytes = 0;
    double build_s = 0, upload_s = 0;
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

int64_t vec_bytes(int dtype) { return dtype == NAPSPMV_F64 ? 8 : 4; }

// Column bands of the standard gather: about 2 MiB of v per band.
int pick_bands(int64_t n, int64_t vb) {
    const int64_t b = (n * vb + (2 << 20) - 1) / (2 << 20);
    return (int)std::max<int64_t>(1, std::min<int64_t>(64, b));
}

template <typename T>
void upload(T *&dst, const std::vector<T> &src, int64_t &total) {
    if (src.empty()) return;
    const size_t bytes = src.size() * sizeof(T);
    HIP_OK(hipMalloc(reinterpret_cast<void **>(&dst), bytes));
    total += (int64_t)bytes;
    HIP_OK(hipMemcpy(dst, src.data(), bytes, hipMemcpyHostToDevice));
}

void alloc(void *&dst, int64_t bytes, int64_t &total) {
    if (bytes <= 0) return;
    HIP_OK(hipMalloc(&dst, (size_t)bytes));
    total += bytes;
}

void free_ptr(void *p) {
    if (p) (void)hipFree(p);
}

void charge(napspmv_plan_s *p, int64_t bytes) {
    p->device_bytes += bytes;
    g_in_use += bytes;
}

void free_schedules(napspmv_plan_s *p) {
    void *ptrs[] = {p->d_onblk, p->d_onptr, p->d_win, p->d_offblk, p->d_offptr, p->d_items,
                    p->d_tasks};
    for (void *q : ptrs) free_ptr(q);
    p->d_onblk = p->d_onptr = p->d_win = p->d_offblk = p->d_offptr = nullptr;
    p->d_items = p->d_tasks = nullptr;
    charge(p, -p->bytes_sched);
    p->bytes_sched = 0;
}

void free_device(napspmv_plan_s *p) {
    free_schedules(p);
    void *ptrs[] = {p->d_rp_on, p->d_col_on, p->d_rp_off, p->d_col_off, p->d_val_on,
                    p->d_val_off, p->d_ghost, p->d_gather, p->d_pack, p->d_send,
                    p->d_recv == p->d_send ? nullptr : p->d_recv,
                    p->d_ssrc, p->d_sdst, p->d_lsrc, p->d_ldst};
    for (void *q : ptrs) free_ptr(q);
    p->d_rp_on = p->d_col_on = p->d_rp_off = p->d_col_off = nullptr;
    p->d_val_on = p->d_val_off = p->d_ghost = p->d_send = p->d_recv = nullptr;
    p->d_gather = p->d_pack = p->d_ssrc = p->d_sdst = p->d_lsrc = p->d_ldst = nullptr;
    g_in_use -= p->device_bytes;
    p->device_bytes = 0;
    p->on_device = false;
}

int64_t planned_device_bytes(const HostPlan &hp, uint32_t flags) {
    const int64_t vb = vec_bytes(hp.dtype);
    int64_t b = (int64_t)(hp.rowptr_on.size() + hp.col_on.size() + hp.rowptr_off.size() +
                          hp.col_off.size()) * 4 + (int64_t)(hp.val_on.size() + hp.val_off.size());
    b += (int64_t)hp.ghost_col.size() * vb;
    b += (int64_t)(hp.gather_idx.size() + hp.pack_idx.size() + hp.scat_src.size() +
                   hp.scat_dst.size() + hp.l2_src.size() + hp.l2_dst.size()) * 4;
    if (hp.mode == NAPSPMV_NAP)
        b += (int64_t)hp.pack_idx.size() * vb * ((flags & NAPSPMV_EXCHANGE_COPY) ? 2 : 1);
    return b;
}

// (Re)build every launch schedule for the current tuning: on-process row
// blocks with their v windows, off-process row blocks, the exchange items
// (standard: ghost gather by column band; NAP: pack in order) and the task
// list of the first launch.
void refresh_schedules(napspmv_plan_s *p) {
    const int cap = p->block_nnz >= 0 ? p->block_nnz : p->auto_block_nnz;
    const int win = p->window >= 0 ? p->window : p->auto_window;
    const int bands = p->bands >= 0 ? p->bands : p->auto_bands;
    if (p->d_onblk && cap == p->cur_block_nnz && win == p->cur_window && bands == p->cur_bands)
        return;
    const HostPlan &hp = p->hp;
    std::vector<int32_t> onblk, onptr, wins, offblk, offptr, items, tasks;
    napspmv::row_blocks(hp.rowptr_on.data(), hp.n, cap, kMaxRowsPerBlock, onblk, onptr);
    if (win > 0) napspmv::row_block_windows(onblk, hp.on_lo, hp.on_hi, hp.n, win, wins);
    napspmv::row_blocks(hp.rowptr_off.data(), hp.n, cap, kMaxRowsPerBlock, offblk, offptr);
    if (hp.mode == NAPSPMV_STANDARD)
        napspmv::gather_items(hp.ghost_ptr, hp.ghost_col, hp.n, bands, kMaxItem, items);
    else
        napspmv::flat_items(p->E, kMaxItem, items);
    napspmv::merge_tasks((int64_t)items.size() / 2, (int64_t)onblk.size() - 1, tasks);
    free_schedules(p);
    int64_t total = 0;
    try {
        upload(p->d_onblk, onblk, total);
        upload(p->d_onptr, onptr, total);
        upload(p->d_win, wins, total);
        upload(p->d_offblk, offblk, total);
        upload(p->d_offptr, offptr, total);
        upload(p->d_items, items, total);
        upload(p->d_tasks, tasks, total);
    } catch (...) {
        p->bytes_sched = total;
        charge(p, total);
        throw;
    }
    p->bytes_sched = total;
    charge(p, total);
    p->n_on_blocks = (int64_t)onblk.size() - 1;
    p->n_off_blocks = (int64_t)offblk.size() - 1;
    p->n_items = (int64_t)items.size() / 2;
    p->n_tasks = (int64_t)tasks.size();
    p->cur_block_nnz = cap;
    p->cur_window = win;
    p->cur_bands = bands;
}

void to_device(napspmv_plan_s *p) {
    HostPlan &hp = p->hp;
    HIP_OK(hipGetDevice(&p->device));

    const int64_t need = planned_device_bytes(hp, p->flags);
    const int64_t budget = g_budget.load();
    if (budget > 0 && g_in_use.load() + need > budget)
        throw Error(NAPSPMV_ENOMEM, "device budget exceeded: plan needs " + std::to_string(need) +
                                        " bytes, " + std::to_string(g_in_use.load()) +
                                        " in use of " + std::to_string(budget));
    int64_t total = 0;
    try {
        const int64_t vb = vec_bytes(hp.dtype);
        upload(p->d_rp_on, hp.rowptr_on, total);
        upload(p->d_col_on, hp.col_on, total);
        upload(p->d_rp_off, hp.rowptr_off, total);
        upload(p->d_col_off, hp.col_off, total);
        auto upload_bytes = [&](void *&dst, const std::vector<uint8_t> &src) {
            if (src.empty()) return;
            HIP_OK(hipMalloc(&dst, src.size()));
            total += (int64_t)src.size();
            HIP_OK(hipMemcpy(dst, src.data(), src.size(), hipMemcpyHostToDevice));
        };
        upload_bytes(p->d_val_on, hp.val_on);
        upload_bytes(p->d_val_off, hp.val_off);
        alloc(p->d_ghost, p->G * vb, total);
        upload(p->d_gather, hp.gather_idx, total);
        upload(p->d_pack, hp.pack_idx, total);
        upload(p->d_ssrc, hp.scat_src, total);
        upload(p->d_sdst, hp.scat_dst, total);
        upload(p->d_lsrc, hp.l2_src, total);
        upload(p->d_ldst, hp.l2_dst, total);
        if (hp.mode == NAPSPMV_NAP) {
            alloc(p->d_send, p->E * vb, total);
            if (p->flags & NAPSPMV_EXCHANGE_COPY)
                alloc(p->d_recv, p->E * vb, total);
            else
                p->d_recv = p->d_send;          // receive in place: the exchange is an alias
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

template <typename VT, typename XT, int CAP, int W>
void launch_local_w(napspmv_plan_s *p, const XT *v, XT *w, hipStream_t s) {
    const bool std_mode = p->hp.mode == NAPSPMV_STANDARD;
    XT *xdst = static_cast<XT *>(std_mode ? p->d_ghost : p->d_send);
    const int32_t *idx = std_mode ? p->d_gather : p->d_pack;
    napspmv::k_local<VT, XT, CAP, W><<<(uint32_t)p->n_tasks, napspmv::kBlock, 0, s>>>(
        p->d_tasks, reinterpret_cast<const int2 *>(p->d_items), idx, xdst, p->d_onblk,
        p->d_onptr, reinterpret_cast<const int2 *>(p->d_win), p->d_rp_on, p->d_col_on,
        static_cast<const VT *>(p->d_val_on), v, w);
}

template <typename VT, typename XT, int CAP>
void launch_local(napspmv_plan_s *p, const XT *v, XT *w, hipStream_t s) {
    switch (p->cur_window) {
        case 1024: launch_local_w<VT, XT, CAP, 1024>(p, v, w, s); break;
        case 2048: launch_local_w<VT, XT, CAP, 2048>(p, v, w, s); break;
        case 4096: launch_local_w<VT, XT, CAP, 4096>(p, v, w, s); break;
        default: launch_local_w<VT, XT, CAP, 0>(p, v, w, s); break;
    }
}

template <typename VT, typename XT, int CAP>
void launch_remote(napspmv_plan_s *p, const XT *v, XT *w, hipStream_t s) {
    using namespace napspmv;
    if (p->hp.mode == NAPSPMV_NAP) {
        // the inter-node hop (alias unless copied), then the scatter of the
        // received values to every user on the node, with the fully local
        // on-node values
        if (p->E > 0 && p->d_recv != p->d_send)
            k_copy<XT><<<blocks_for(p->E), kBlock, 0, s>>>((int32_t)p->E,
                                                         static_cast<const XT *>(p->d_send),
                                                         static_cast<XT *>(p->d_recv));
        const uint32_t nb1 = blocks_for(p->H), nb2 = blocks_for(p->Gon);
        if (nb1 + nb2 > 0)
            k_scatter2<XT><<<nb1 + nb2, kBlock, 0, s>>>(
                (int32_t)p->H, p->d_ssrc, p->d_sdst, static_cast<const XT *>(p->d_recv),
                (int32_t)p->Gon, p->d_lsrc, p->d_ldst, v, static_cast<XT *>(p->d_ghost), nb1);
    }
    if (p->hp.nnz_off > 0)
        k_remote<VT, XT, CAP><<<(uint32_t)p->n_off_blocks, kBlock, 0, s>>>(
            p->d_offblk, p->d_offptr, p->d_rp_off, p->d_col_off,
            static_cast<const VT *>(p->d_val_off), static_cast<const XT *>(p->d_ghost), w);
}

template <typename VT, typename XT>
void launch_stage(napspmv_plan_s *p, int stage, const XT *v, XT *w, hipStream_t s) {
    switch (p->cur_block_nnz) {
        case 1024:
            stage == NAPSPMV_STAGE_LOCAL ? launch_local<VT, XT, 1024>(p, v, w, s)
                                         : launch_remote<VT, XT, 1024>(p, v, w, s);
            break;
        case 4096:
            stage == NAPSPMV_STAGE_LOCAL ? launch_local<VT, XT, 4096>(p, v, w, s)
                                         : launch_remote<VT, XT, 4096>(p, v, w, s);
            break;
        default:
            stage == NAPSPMV_STAGE_LOCAL ? launch_local<VT, XT, 2048>(p, v, w, s)
                                         : launch_remote<VT, XT, 2048>(p, v, w, s);
            break;
    }
}

void run_stage(napspmv_plan_s *p, int stage, const void *v, void *w, hipStream_t s) {
    switch (p->hp.dtype) {
        case NAPSPMV_F64:
            launch_stage<double, double>(p, stage, static_cast<const double *>(v),
                                         static_cast<double *>(w), s);
            break;
        case NAPSPMV_F32:
            launch_stage<float, float>(p, stage, static_cast<const float *>(v),
                                       static_cast<float *>(w), s);
            break;
        default:
            launch_stage<uint16_t, float>(p, stage, static_cast<const float *>(v),
                                          static_cast<float *>(w), s);
            break;
    }
    HIP_OK(hipGetLastError());
}

int check_apply(napspmv_plan_t plan, const void *v, void *w) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    if (!v || !w) return fail(NAPSPMV_EINVAL, "v or w is NULL");
    const int64_t bytes = plan->hp.n * vec_bytes(plan->hp.dtype);
    const char *a = static_cast<const char *>(v);
    const char *b = static_cast<const char *>(w);
    if (a < b + bytes && b < a + bytes) return fail(NAPSPMV_EINVAL, "v and w overlap");
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
}

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

}  // namespace

extern "C" {

int napspmv_plan_create(const int64_t *rowptr, const int32_t *col, const void *val, int dtype,
                        int64_t n, int64_t n_p, int64_t ppn, int mode, const int64_t *row_starts,
                        uint32_t flags, napspmv_plan_t *plan_out, napspmv_stats_t *stats_out) {
    if (!plan_out) return fail(NAPSPMV_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    if (flags & ~(NAPSPMV_HOST_ONLY | NAPSPMV_EXCHANGE_COPY))
        return fail(NAPSPMV_EINVAL, "unknown flag bits");
    napspmv_plan_s *p = nullptr;
    const int rc = guarded([&]() {
        p = new napspmv_plan_s();
        p->flags = flags;
        const auto t0 = std::chrono::steady_clock::now();
        napspmv::build_plan(p->hp, rowptr, col, val, dtype, n, n_p, ppn, mode, row_starts);
        const auto t1 = std::chrono::steady_clock::now();
        p->build_s = std::chrono::duration<double>(t1 - t0).count();
        p->G = p->hp.ghost_ptr.back();
        p->E = (int64_t)p->hp.pack_idx.size();
        p->H = (int64_t)p->hp.scat_src.size();
        p->Gon = (int64_t)p->hp.l2_src.size();
        p->auto_bands = pick_bands(n, vec_bytes(dtype));
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

int napspmv_apply_stage(napspmv_plan_t plan, int stage, const void *v, void *w, void *stream) {
    int rc = check_apply(plan, v, w);
    if (rc) return rc;
    if (stage != NAPSPMV_STAGE_LOCAL && stage != NAPSPMV_STAGE_REMOTE)
        return fail(NAPSPMV_EINVAL, "unknown stage");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        run_stage(plan, stage, v, w, static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    });
}

int napspmv_apply(napspmv_plan_t plan, const void *v, void *w, void *stream) {
    int rc = check_apply(plan, v, w);
    if (rc) return rc;
    return guarded([&]() {
        DeviceGuard g(plan->device);
        run_stage(plan, NAPSPMV_STAGE_LOCAL, v, w, static_cast<hipStream_t>(stream));
        run_stage(plan, NAPSPMV_STAGE_REMOTE, v, w, static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    });
}

int napspmv_plan_stats(napspmv_plan_t plan, napspmv_stats_t *out) {
    if (!plan || !out) return fail(NAPSPMV_EINVAL, "plan or out is NULL");
    fill_stats(plan, out);
    return NAPSPMV_OK;
}

int napspmv_plan_export(napspmv_plan_t plan, int phase, int64_t *n_msgs, int64_t *n_idx,
                        int32_t *src, int32_t *dst, int64_t *ptr, int32_t *idx) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (phase < 0 || phase > 3) return fail(NAPSPMV_EINVAL, "unknown phase");
    const napspmv::Phase &ph = plan->hp.phase[phase];
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

int napspmv_plan_read_ghost_values(napspmv_plan_t plan, void *out, void *stream) {
    if (!plan || !out) return fail(NAPSPMV_EINVAL, "plan or out is NULL");
    if (!plan->on_device) return fail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    return guarded([&]() {
        DeviceGuard g(plan->device);
        HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
        if (plan->G > 0)
            HIP_OK(hipMemcpy(out, plan->d_ghost, (size_t)(plan->G * vec_bytes(plan->hp.dtype)),
                             hipMemcpyDeviceToHost));
        return NAPSPMV_OK;
    });
}

int napspmv_plan_set_param(napspmv_plan_t plan, int param, int value) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    switch (param) {
        case NAPSPMV_PARAM_BLOCK_NNZ:
            if (value != -1 && value != 1024 && value != 2048 && value != 4096)
                return fail(NAPSPMV_EINVAL, "block entries must be -1, 1024, 2048 or 4096");
            plan->block_nnz = value;
            break;
        case NAPSPMV_PARAM_GATHER_BANDS:
            if (value != -1 && (value < 1 || value > 4096))
                return fail(NAPSPMV_EINVAL, "bands must be -1 or in [1, 4096]");
            plan->bands = value;
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
        case NAPSPMV_PARAM_BLOCK_NNZ: return plan->block_nnz >= 0 ? plan->block_nnz : plan->auto_block_nnz;
        case NAPSPMV_PARAM_GATHER_BANDS: return plan->bands >= 0 ? plan->bands : plan->auto_bands;
        case NAPSPMV_PARAM_VWINDOW: return plan->window >= 0 ? plan->window : plan->auto_window;
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
