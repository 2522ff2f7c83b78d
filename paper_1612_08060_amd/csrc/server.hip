// Serving engine: many resident plans, requests w = A_id v admitted into a
// fixed number of slots (one HIP stream each) as slots and workspace memory
// free up, each slot running one batched launch sequence over the requests
// it holds (napspmv_batch_apply).  Requests that arrive while others run
// join the next free slot, so their work overlaps the work already on the
// device (continuous batching).  Workspaces (ghost and NAP send buffers) come
// from per-plan free lists, allocated on first need within a byte budget;
// a request whose workspace does not fit waits in the queue.
//
// Single-threaded by design: the caller drives it with submit/poll (or
// replays a whole arrival trace natively with napspmv_server_replay).
// Requests follow the caller's stream: submit and replay record a fence
// event on it, and a slot waits for the latest fence before it runs a batch,
// so the caller's writes of v (and w) before the call are seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <string>
#include <vector>

#include "napspmv.h"
#include "plan_build.hpp"

using napspmv::Error;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

struct ServerRequest {
    int plan = 0;
    const void *v = nullptr;
    void *w = nullptr;
    void *ws = nullptr;
    int64_t t_submit = 0, t_done = 0;
    int batch = 0;           // size of the batch the request ran in
    int state = 0;           // 0 queued, 1 running, 2 done
};

struct ServerSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    napspmv_batch_t batch = nullptr;
    std::vector<int64_t> reqs;
    bool busy = false;
    int64_t fence_seen = 0;  // the fence generation this slot's stream already waits for
};

struct ServerPlan {
    napspmv_plan_t plan = nullptr;
    int64_t ws_bytes = 0;
    int key_dtype = 0, key_cap = 0, key_win = 0;
    bool solo = false;      // never batched (explicit exchange copy, three-way product)
    std::vector<void *> free_ws, all_ws;
};

struct napspmv_server_s {
    int device = 0;
    int max_batch = 1;
    int n_slots = 0;
    int64_t budget = 0, ws_in_use = 0;
    std::vector<ServerPlan> plans;
    std::vector<ServerSlot> slots;   // created with the first device plan
    std::deque<int64_t> queue;
    std::vector<ServerRequest> reqs;
    int64_t completed = 0;
    hipEvent_t fence = nullptr;      // recorded on the caller's stream by submit and replay
    int64_t fence_gen = 0;           // how many times it was recorded
};

namespace {

thread_local std::string g_server_error;

int sfail(int code, const std::string &msg) {
    g_server_error = msg;
    return code;
}

#define HIP_SOK(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw Error(NAPSPMV_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename F>
int sguard(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return sfail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return sfail(NAPSPMV_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return sfail(NAPSPMV_EINVAL, e.what());
    }
}

int64_t ws_size(const ServerPlan &P) { return std::max<int64_t>(P.ws_bytes, 256); }

// Streams, events and batch tables of the slots, on the current device: made
// when the first device plan is added, so that creating a server and
// refusing plans needs no GPU.
void release_slot(ServerSlot &sl) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.batch) napspmv_batch_destroy(sl.batch);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    sl = ServerSlot();
}

void ensure_slots(napspmv_server_s *s) {
    if (!s->slots.empty()) return;
    std::vector<ServerSlot> made(s->n_slots);
    try {
        HIP_SOK(hipGetDevice(&s->device));
        if (!s->fence) HIP_SOK(hipEventCreateWithFlags(&s->fence, hipEventDisableTiming));
        for (ServerSlot &sl : made) {
            HIP_SOK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            HIP_SOK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
            const int brc = napspmv_batch_create(s->max_batch, &sl.batch);
            if (brc != NAPSPMV_OK) throw Error(brc, napspmv_last_error());
        }
    } catch (...) {
        for (ServerSlot &sl : made) release_slot(sl);
        throw;
    }
    s->slots = std::move(made);
}

// Order the requests submitted so far after the caller's work on `stream`.
void record_fence(napspmv_server_s *s, void *stream) {
    HIP_SOK(hipEventRecord(s->fence, static_cast<hipStream_t>(stream)));
    ++s->fence_gen;
}

// A workspace for plan `pi`: from its free list, or newly allocated if the
// budget allows (idle workspaces of other plans are released to make room);
// nullptr if neither.
void *take_ws(napspmv_server_s *s, int pi) {
    ServerPlan &P = s->plans[pi];
    if (!P.free_ws.empty()) {
        void *w = P.free_ws.back();
        P.free_ws.pop_back();
        return w;
    }
    const int64_t need = ws_size(P);
    if (s->budget > 0 && need > s->budget) return nullptr;
    for (size_t q = 0; s->budget > 0 && s->ws_in_use + need > s->budget && q < s->plans.size(); ++q) {
        ServerPlan &O = s->plans[q];
        while (!O.free_ws.empty() && s->ws_in_use + need > s->budget) {
            void *x = O.free_ws.back();
            O.free_ws.pop_back();
            O.all_ws.erase(std::find(O.all_ws.begin(), O.all_ws.end(), x));
            (void)hipFree(x);
            s->ws_in_use -= ws_size(O);
        }
    }
    if (s->budget > 0 && s->ws_in_use + need > s->budget) return nullptr;
    void *w = nullptr;
    if (hipMalloc(&w, (size_t)need) != hipSuccess) return nullptr;
    s->ws_in_use += need;
    P.all_ws.push_back(w);
    return w;
}

// Retire finished slots; returns the number of requests completed.
int64_t retire(napspmv_server_s *s) {
    int64_t n = 0;
    for (ServerSlot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) throw Error(NAPSPMV_EHIP, std::string("slot failed: ") + hipGetErrorString(q));
        const int64_t t = now_ns();
        for (int64_t r : sl.reqs) {
            ServerRequest &R = s->reqs[r];
            R.t_done = t;
            R.state = 2;
            s->plans[R.plan].free_ws.push_back(R.ws);
            R.ws = nullptr;
            ++n;
        }
        sl.reqs.clear();
        sl.busy = false;
    }
    s->completed += n;
    return n;
}

// Fill free slots from the queue, oldest request first; a batch takes the
// oldest request's kernel group (value type, block sizes, window) and every
// later queued request of that group that gets a workspace.  A plan that
// batches cannot take (solo) runs alone.
void admit(napspmv_server_s *s) {
    for (ServerSlot &sl : s->slots) {
        if (sl.busy) continue;
        if (s->queue.empty()) return;
        std::vector<int64_t> take;
        int key[3] = {-1, -1, -1};
        for (auto it = s->queue.begin(); it != s->queue.end() && (int)take.size() < s->max_batch;) {
            ServerRequest &R = s->reqs[*it];
            const ServerPlan &P = s->plans[R.plan];
            if (key[0] >= 0 && (P.solo || P.key_dtype != key[0] || P.key_cap != key[1] ||
                                P.key_win != key[2])) {
                ++it;
                continue;
            }
            void *ws = take_ws(s, R.plan);
            if (!ws) {          // no memory for this request yet: it waits
                ++it;
                continue;
            }
            R.ws = ws;
            key[0] = P.key_dtype;
            key[1] = P.key_cap;
            key[2] = P.key_win;
            take.push_back(*it);
            it = s->queue.erase(it);
            if (P.solo) break;
        }
        if (take.empty()) {
            // nothing running will ever release a workspace: the queued
            // requests could wait forever
            bool running = false;
            for (const ServerSlot &o : s->slots) running = running || o.busy;
            if (!running)
                throw Error(NAPSPMV_ENOMEM, "no workspace can be allocated for the queued requests "
                                            "and none is in use");
            return;
        }
        if (sl.fence_seen < s->fence_gen) {
            HIP_SOK(hipStreamWaitEvent(sl.stream, s->fence, 0));
            sl.fence_seen = s->fence_gen;
        }
        const int n = (int)take.size();
        std::vector<napspmv_plan_t> plans(n);
        std::vector<void *> wss(n), ws_out(n);
        std::vector<const void *> vs(n);
        for (int i = 0; i < n; ++i) {
            ServerRequest &R = s->reqs[take[i]];
            plans[i] = s->plans[R.plan].plan;
            wss[i] = R.ws;
            vs[i] = R.v;
            ws_out[i] = R.w;
            R.state = 1;
            R.batch = n;
        }
        // a lone request takes the plain apply path (no descriptor table)
        const int rc = n == 1 ? napspmv_apply_ws(plans[0], wss[0], vs[0], ws_out[0], sl.stream)
                              : napspmv_batch_apply(sl.batch, n, plans.data(), wss.data(),
                                                    vs.data(), ws_out.data(), sl.stream);
        if (rc != NAPSPMV_OK) throw Error(rc, std::string("batch apply: ") + napspmv_last_error());
        HIP_SOK(hipEventRecord(sl.done, sl.stream));
        sl.reqs = take;
        sl.busy = true;
    }
}

}  // namespace

extern "C" {

int napspmv_server_create(int slots, int max_batch, int64_t workspace_budget,
                          napspmv_server_t *out) {
    if (!out) return sfail(NAPSPMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64 || max_batch < 1 || max_batch > 4096 || workspace_budget < 0)
        return sfail(NAPSPMV_EINVAL, "need 1 <= slots <= 64, 1 <= max_batch <= 4096, budget >= 0");
    napspmv_server_s *s = new (std::nothrow) napspmv_server_s();
    if (!s) return sfail(NAPSPMV_ENOMEM, "host allocation failed");
    s->max_batch = max_batch;
    s->n_slots = slots;
    s->budget = workspace_budget;
    *out = s;
    return NAPSPMV_OK;
}

int napspmv_server_add_plan(napspmv_server_t s, napspmv_plan_t plan, int *id_out) {
    if (!s || !plan || !id_out) return sfail(NAPSPMV_EINVAL, "NULL argument");
    const int64_t wsb = napspmv_plan_workspace_bytes(plan);
    if (wsb < 0) return sfail((int)wsb, napspmv_last_error());
    ServerPlan P;
    P.plan = plan;
    P.ws_bytes = wsb;
    // a request whose workspace can never fit would wait forever
    if (s->budget > 0 && ws_size(P) > s->budget)
        return sfail(NAPSPMV_ENOMEM, "the plan's workspace (" + std::to_string(ws_size(P)) +
                                         " bytes) exceeds the server's workspace budget (" +
                                         std::to_string(s->budget) + ")");
    napspmv_stats_t st;
    napspmv_plan_stats(plan, &st);
    if (st.flags & NAPSPMV_HOST_ONLY)
        return sfail(NAPSPMV_EINVAL, "plan was built with NAPSPMV_HOST_ONLY");
    const int rc = sguard([&]() {
        ensure_slots(s);
        return NAPSPMV_OK;
    });
    if (rc != NAPSPMV_OK) return rc;
    P.key_dtype = st.dtype;
    P.key_cap = napspmv_plan_get_param(plan, NAPSPMV_PARAM_BLOCK_NNZ);
    P.key_win = napspmv_plan_get_param(plan, NAPSPMV_PARAM_VWINDOW);
    P.solo = st.mode == NAPSPMV_NAP &&
             (st.flags & (NAPSPMV_EXCHANGE_COPY | NAPSPMV_NAP_THREE_WAY)) != 0;
    s->plans.push_back(P);
    *id_out = (int)s->plans.size() - 1;
    return NAPSPMV_OK;
}

int napspmv_server_submit(napspmv_server_t s, int id, const void *v, void *w, void *stream,
                          int64_t *ticket) {
    if (!s || !v || !w || !ticket) return sfail(NAPSPMV_EINVAL, "NULL argument");
    if (id < 0 || id >= (int)s->plans.size()) return sfail(NAPSPMV_EINVAL, "unknown plan id");
    const int rc = sguard([&]() {
        record_fence(s, stream);
        return NAPSPMV_OK;
    });
    if (rc != NAPSPMV_OK) return rc;
    ServerRequest R;
    R.plan = id;
    R.v = v;
    R.w = w;
    R.t_submit = now_ns();
    s->reqs.push_back(R);
    *ticket = (int64_t)s->reqs.size() - 1;
    s->queue.push_back(*ticket);
    return NAPSPMV_OK;
}

int64_t napspmv_server_poll(napspmv_server_t s) {
    if (!s) return sfail(NAPSPMV_EINVAL, "server is NULL");
    int64_t n = 0;
    const int rc = sguard([&]() {
        n = retire(s);
        admit(s);
        return NAPSPMV_OK;
    });
    return rc == NAPSPMV_OK ? n : rc;
}

int napspmv_server_wait(napspmv_server_t s, int64_t ticket) {
    if (!s || ticket < 0 || ticket >= (int64_t)s->reqs.size())
        return sfail(NAPSPMV_EINVAL, "bad server or ticket");
    while (s->reqs[ticket].state != 2) {
        const int64_t rc = napspmv_server_poll(s);
        if (rc < 0) return (int)rc;
    }
    return NAPSPMV_OK;
}

int napspmv_server_request_info(napspmv_server_t s, int64_t ticket, int64_t *submit_ns,
                                int64_t *done_ns, int *batch_size) {
    if (!s || ticket < 0 || ticket >= (int64_t)s->reqs.size())
        return sfail(NAPSPMV_EINVAL, "bad server or ticket");
    const ServerRequest &R = s->reqs[ticket];
    if (submit_ns) *submit_ns = R.t_submit;
    if (done_ns) *done_ns = R.state == 2 ? R.t_done : -1;
    if (batch_size) *batch_size = R.batch;
    return NAPSPMV_OK;
}

int napspmv_server_replay(napspmv_server_t s, int64_t n, const int *ids, const int64_t *arrival_ns,
                          const void *const *v, void *const *w, void *stream, int64_t *latency_ns,
                          int *batch_sizes) {
    if (!s || n < 0 || (n > 0 && (!ids || !arrival_ns || !v || !w || !latency_ns)))
        return sfail(NAPSPMV_EINVAL, "NULL argument");
    for (int64_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= (int)s->plans.size()) return sfail(NAPSPMV_EINVAL, "unknown plan id");
    return sguard([&]() {
        if (n > 0) record_fence(s, stream);   // every vector was written before the call
        const int64_t first = (int64_t)s->reqs.size();
        const int64_t t0 = now_ns();
        for (int64_t i = 0; i < n; ++i) {
            while (now_ns() - t0 < arrival_ns[i]) {
                retire(s);
                admit(s);
            }
            ServerRequest R;
            R.plan = ids[i];
            R.v = v[i];
            R.w = w[i];
            R.t_submit = t0 + arrival_ns[i];     // latency counts from the scheduled arrival
            s->reqs.push_back(R);
            s->queue.push_back((int64_t)s->reqs.size() - 1);
            retire(s);
            admit(s);
        }
        while (s->completed < (int64_t)s->reqs.size()) {
            retire(s);
            admit(s);
        }
        for (int64_t i = 0; i < n; ++i) {
            const ServerRequest &R = s->reqs[first + i];
            latency_ns[i] = R.t_done - R.t_submit;
            if (batch_sizes) batch_sizes[i] = R.batch;
        }
        return NAPSPMV_OK;
    });
}

int napspmv_server_reserve(napspmv_server_t s, int per_plan) {
    if (!s || per_plan < 0) return sfail(NAPSPMV_EINVAL, "bad server or count");
    return sguard([&]() {
        for (ServerPlan &P : s->plans) {
            const int64_t need = ws_size(P);
            while ((int)P.all_ws.size() < per_plan &&
                   (s->budget == 0 || s->ws_in_use + need <= s->budget)) {
                void *w = nullptr;
                HIP_SOK(hipMalloc(&w, (size_t)need));
                s->ws_in_use += need;
                P.all_ws.push_back(w);
                P.free_ws.push_back(w);
            }
        }
        return NAPSPMV_OK;
    });
}

int64_t napspmv_server_workspace_bytes(napspmv_server_t s) {
    if (!s) return sfail(NAPSPMV_EINVAL, "server is NULL");
    return s->ws_in_use;
}

const char *napspmv_server_last_error(void) { return g_server_error.c_str(); }

int napspmv_server_destroy(napspmv_server_t s) {
    if (!s) return NAPSPMV_OK;
    for (ServerSlot &sl : s->slots) release_slot(sl);
    if (s->fence) (void)hipEventDestroy(s->fence);
    for (ServerPlan &P : s->plans)
        for (void *w : P.all_ws) (void)hipFree(w);
    delete s;
    return NAPSPMV_OK;
}

}  // extern "C"
