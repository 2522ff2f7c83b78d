// The C ABI of include/napspmv.h: plan creation (host builder + device
// upload), the apply path (exchange kernels + split product) and the
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

using napspmv::Error;
using napspmv::HostPlan;

struct napspmv_plan_s {
    HostPlan hp;
    uint32_t flags = 0;
    bool on_device = false;
    int device = 0;
    int lanes = 0;           // lanes per row of the product (0 = auto)
    int auto_lanes = 8;
    int64_t G = 0, E = 0, H = 0, Gon = 0;
    int32_t *d_rowptr = nullptr, *d_col = nullptr;
    void *d_val = nullptr;
    void *d_ghost = nullptr;
    int32_t *d_gather = nullptr, *d_pack = nullptr;
    void *d_send = nullptr, *d_recv = nullptr;
    int32_t *d_ssrc = nullptr, *d_sdst = nullptr, *d_lsrc = nullptr, *d_ldst = nullptr;
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

int pick_lanes(double mean_row) {
    int l = 1;
    while (l < 64 && 2 * l < mean_row) l *= 2;   // about two entries per lane
    return l;
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

void free_device(napspmv_plan_s *p) {
    void *ptrs[] = {p->d_rowptr, p->d_col, p->d_val, p->d_ghost, p->d_gather, p->d_pack,
                    p->d_send, p->d_recv == p->d_send ? nullptr : p->d_recv,
                    p->d_ssrc, p->d_sdst, p->d_lsrc, p->d_ldst};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    g_in_use -= p->device_bytes;
    p->device_bytes = 0;
    p->on_device = false;
}

int64_t planned_device_bytes(const HostPlan &hp, uint32_t flags) {
    const int64_t vb = vec_bytes(hp.dtype);
    int64_t b = (int64_t)(hp.rowptr.size() + hp.col.size()) * 4 + (int64_t)hp.val.size();
    b += (int64_t)hp.ghost_col.size() * vb;
    b += (int64_t)(hp.gather_idx.size() + hp.pack_idx.size() + hp.scat_src.size() +
                   hp.scat_dst.size() + hp.l2_src.size() + hp.l2_dst.size()) * 4;
    if (hp.mode == NAPSPMV_NAP)
        b += (int64_t)hp.pack_idx.size() * vb * ((flags & NAPSPMV_EXCHANGE_COPY) ? 2 : 1);
    return b;
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
        upload(p->d_rowptr, hp.rowptr, total);
        upload(p->d_col, hp.col, total);
        if (!hp.val.empty()) {
            HIP_OK(hipMalloc(&p->d_val, hp.val.size()));
            total += (int64_t)hp.val.size();
            HIP_OK(hipMemcpy(p->d_val, hp.val.data(), hp.val.size(), hipMemcpyHostToDevice));
        }
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
        HIP_OK(hipDeviceSynchronize());
    } catch (...) {
        p->device_bytes = total;
        g_in_use += total;
        free_device(p);
        throw;
    }
    p->device_bytes = total;
    g_in_use += total;
    p->on_device = true;
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + napspmv::kBlock - 1) / napspmv::kBlock); }

template <typename XT>
void launch_exchange(napspmv_plan_s *p, const XT *v, hipStream_t s) {
    using namespace napspmv;
    if (p->hp.mode == NAPSPMV_STANDARD) {
        if (p->G > 0)
            k_gather<XT><<<blocks_for(p->G), kBlock, 0, s>>>((int32_t)p->G, p->d_gather, v,
                                                           static_cast<XT *>(p->d_ghost));
        return;
    }
    // NAP: pack the inter-node messages straight from the owners' values
    // (the on_node -> off_node step and the pack of the inter-node send
    // buffer in one gather), hop to the receive buffer, then scatter the
    // received values to every user on the destination node together with
    // the fully local on-node values.
    if (p->E > 0)
        k_gather<XT><<<blocks_for(p->E), kBlock, 0, s>>>((int32_t)p->E, p->d_pack, v,
                                                       static_cast<XT *>(p->d_send));
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

template <typename VT, typename XT, int S>
void launch_spmv_s(napspmv_plan_s *p, const XT *v, XT *w, hipStream_t s) {
    constexpr int rows = napspmv::kBlock / S;
    const int64_t n = p->hp.n;
    const uint32_t nb = (uint32_t)((n + rows - 1) / rows);
    napspmv::k_spmv<VT, XT, S><<<nb, napspmv::kBlock, 0, s>>>(
        (int32_t)n, p->d_rowptr, p->d_col, static_cast<const VT *>(p->d_val), v,
        static_cast<const XT *>(p->d_ghost), w);
}

template <typename VT, typename XT>
void launch_spmv(napspmv_plan_s *p, const XT *v, XT *w, hipStream_t s) {
    switch (p->lanes ? p->lanes : p->auto_lanes) {
        case 1: launch_spmv_s<VT, XT, 1>(p, v, w, s); break;
        case 2: launch_spmv_s<VT, XT, 2>(p, v, w, s); break;
        case 4: launch_spmv_s<VT, XT, 4>(p, v, w, s); break;
        case 8: launch_spmv_s<VT, XT, 8>(p, v, w, s); break;
        case 16: launch_spmv_s<VT, XT, 16>(p, v, w, s); break;
        case 32: launch_spmv_s<VT, XT, 32>(p, v, w, s); break;
        default: launch_spmv_s<VT, XT, 64>(p, v, w, s); break;
    }
}

void run_stage(napspmv_plan_s *p, int stage, const void *v, void *w, hipStream_t s) {
    if (stage == NAPSPMV_STAGE_EXCHANGE) {
        if (p->hp.dtype == NAPSPMV_F64)
            launch_exchange<double>(p, static_cast<const double *>(v), s);
        else
            launch_exchange<float>(p, static_cast<const float *>(v), s);
    } else {
        switch (p->hp.dtype) {
            case NAPSPMV_F64:
                launch_spmv<double, double>(p, static_cast<const double *>(v), static_cast<double *>(w), s);
                break;
            case NAPSPMV_F32:
                launch_spmv<float, float>(p, static_cast<const float *>(v), static_cast<float *>(w), s);
                break;
            default:
                launch_spmv<uint16_t, float>(p, static_cast<const float *>(v), static_cast<float *>(w), s);
                break;
        }
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
    try {
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
        p->auto_lanes = pick_lanes(n > 0 ? (double)p->hp.nnz / (double)n : 0.0);
        if (!(flags & NAPSPMV_HOST_ONLY)) {
            to_device(p);
            napspmv::release_device_arrays(p->hp);
            p->upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
        }
        if (stats_out) fill_stats(p, stats_out);
        *plan_out = p;
        g_last_error.clear();
        return NAPSPMV_OK;
    } catch (const Error &e) {
        delete p;
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(NAPSPMV_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        delete p;
        return fail(NAPSPMV_EINVAL, e.what());
    }
}

int napspmv_apply_stage(napspmv_plan_t plan, int stage, const void *v, void *w, void *stream) {
    int rc = check_apply(plan, v, w);
    if (rc) return rc;
    if (stage != NAPSPMV_STAGE_EXCHANGE && stage != NAPSPMV_STAGE_SPMV)
        return fail(NAPSPMV_EINVAL, "unknown stage");
    try {
        DeviceGuard g(plan->device);
        run_stage(plan, stage, v, w, static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    } catch (const Error &e) {
        return fail(e.code, e.what());
    }
}

int napspmv_apply(napspmv_plan_t plan, const void *v, void *w, void *stream) {
    int rc = check_apply(plan, v, w);
    if (rc) return rc;
    try {
        DeviceGuard g(plan->device);
        run_stage(plan, NAPSPMV_STAGE_EXCHANGE, v, w, static_cast<hipStream_t>(stream));
        run_stage(plan, NAPSPMV_STAGE_SPMV, v, w, static_cast<hipStream_t>(stream));
        return NAPSPMV_OK;
    } catch (const Error &e) {
        return fail(e.code, e.what());
    }
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
    try {
        DeviceGuard g(plan->device);
        HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
        if (plan->G > 0)
            HIP_OK(hipMemcpy(out, plan->d_ghost, (size_t)(plan->G * vec_bytes(plan->hp.dtype)),
                             hipMemcpyDeviceToHost));
        return NAPSPMV_OK;
    } catch (const Error &e) {
        return fail(e.code, e.what());
    }
}

int napspmv_plan_set_lanes(napspmv_plan_t plan, int lanes) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    if (lanes != 0 && (lanes < 1 || lanes > 64 || (lanes & (lanes - 1))))
        return fail(NAPSPMV_EINVAL, "lanes per row must be 0 or a power of two up to 64");
    plan->lanes = lanes;
    return NAPSPMV_OK;
}

int napspmv_plan_get_lanes(napspmv_plan_t plan) {
    if (!plan) return fail(NAPSPMV_EINVAL, "plan is NULL");
    return plan->lanes ? plan->lanes : plan->auto_lanes;
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
