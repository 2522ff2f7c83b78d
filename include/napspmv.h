/*
 * napspmv.h -- node-aware parallel sparse matrix-vector multiplication on one
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes w = A v (section 1 of Bienz, Gropp, Olson, "Node aware
 * sparse matrix-vector multiplication") with the rows of the N x N matrix A
 * split into n_p contiguous blocks, one per simulated process, and the
 * processes grouped ppn per node in SMP order: rank r is the pair
 * (r mod ppn, r div ppn) (section 2).  Every block's rows are split into an
 * on-process part (columns the process owns) and an off-process part
 * (columns owned elsewhere, the process's "ghosts") (section 2, the
 * on_process / off_process definitions).  All processes live on one GPU, so
 * every message of the paper's algorithms becomes a device gather or scatter
 * over index lists that a communication plan holds:
 *
 *   standard mode  -- the reference scheme of section 2.1 (algorithm
 *                     standard_spmv): one message per (owner, user) pair.
 *   NAP mode       -- the node-aware scheme of section 4 (algorithm
 *                     NAPSpMV): ghosts deduplicated per destination node,
 *                     gathered on the source node, sent in one inter-node
 *                     message per node pair, scattered on the destination
 *                     node; on-node ghosts go directly.
 *
 * Both modes fill the same ghost values (each process's ghosts, which the
 * plan lists in ascending column order; on the device the buffer is laid
 * out by column band) and run the same split product
 *     w_i = sum_on a_ij v_j + sum_off a_ij ghost_t(j),
 * so their results are bitwise identical.  Each row is summed as algorithm
 * standard_spmv does: sequentially from 0, its on-process entries in stored
 * order, then its off-process entries in stored order, one rounded product
 * and one rounded add per entry.
 *
 * Conventions for every call:
 *   - Return 0 (NAPSPMV_OK) on success or a negative NAPSPMV_E* code; nothing
 *     throws across this interface.  napspmv_last_error() gives a message
 *     for the last failure on the calling thread.
 *   - Host arrays passed in are borrowed for the duration of the call only.
 *   - "device" pointers are HIP device allocations of the GPU that was
 *     current when the plan was created; "stream" is a hipStream_t passed as
 *     void* (NULL is the default stream).
 */
#ifndef NAPSPMV_H
#define NAPSPMV_H

#include <stdint.h>

#if defined(__GNUC__)
#define NAPSPMV_API __attribute__((visibility("default")))
#else
#define NAPSPMV_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define NAPSPMV_OK            0
#define NAPSPMV_EINVAL       (-1)  /* bad argument: invalid CSR, partition, mode, dtype, pointer */
#define NAPSPMV_ENOMEM       (-2)  /* host or device allocation failed, or device budget exceeded */
#define NAPSPMV_EHIP         (-3)  /* a HIP runtime call failed */
#define NAPSPMV_EUNSUPPORTED (-4)  /* valid but outside this build's limits (e.g. nnz >= 2^31) */

/* Modes. */
#define NAPSPMV_STANDARD 0
#define NAPSPMV_NAP      1

/* Value types of A.  The input vector v and the result w are float64 for
 * F64 plans and float32 for F32 and BF16 plans; F32 and BF16 plans
 * accumulate in float32. */
#define NAPSPMV_F64  0
#define NAPSPMV_F32  1
#define NAPSPMV_BF16 2   /* values passed as raw bfloat16 bit patterns (uint16) */

/* Message phases (section 4.2).  A standard plan reports its inter-node
 * messages as INTER and its intra-node messages as L2, so "standard
 * intra-node == NAP fully local" is a field-by-field comparison. */
#define NAPSPMV_PHASE_INTER 0   /* inter-node: standard off-node messages, or NAP node-to-node */
#define NAPSPMV_PHASE_L0    1   /* NAP on_node -> off_node: owner to inter-node sender */
#define NAPSPMV_PHASE_L1    2   /* NAP off_node -> on_node: inter-node receiver to user */
#define NAPSPMV_PHASE_L2    3   /* on_node -> on_node: direct on-node messages */
/* Socket-level phases of a plan built by napspmv_plan_create_sockets: how
 * each intra-node step (L0, L1, L2) travels between sockets.  Phase
 * NAPSPMV_PHASE_SOCKET(step, part) for step = NAPSPMV_PHASE_L0..L2 and part:
 *   ON      the step's messages whose two ranks share a socket (direct)
 *   GATHER  holder -> socket sender, the indices the sender passes on
 *   CROSS   socket sender -> socket receiver, one message per socket pair
 *           (F(a, b): the union of the step's indices from socket a to b)
 *   SCATTER socket receiver -> the other ranks of its socket that need them */
#define NAPSPMV_PART_ON      0
#define NAPSPMV_PART_GATHER  1
#define NAPSPMV_PART_CROSS   2
#define NAPSPMV_PART_SCATTER 3
#define NAPSPMV_PHASE_SOCKET(step, part) (4 * (step) + (part))   /* 4 .. 15 */

/* Plan flags. */
#define NAPSPMV_HOST_ONLY     0x1u  /* build the plan on the host only (no GPU needed):
                                       stats and exports work, apply is refused */
#define NAPSPMV_EXCHANGE_COPY 0x2u  /* NAP: copy the send buffer to a separate receive
                                       buffer (models the inter-node hop) instead of
                                       receiving in place */
/* NAP plan variants (section 4.1; none is the default).  They change which
 * process sends, receives or forwards what, hence the plan's messages and
 * statistics; the ghost values and w are the same bit for bit.  EINVAL with
 * NAPSPMV_STANDARD. */
#define NAPSPMV_NAP_OWNER_MAP 0x4u  /* the inter-node sender of E(n, m) is the local
                                       process of n owning most of its indices
                                       (lowest local number on ties), instead of the
                                       process the volume ranking assigns */
#define NAPSPMV_NAP_SPLIT     0x8u  /* a node with k < ppn partners sends its i-th
                                       partner's E(n, m) through locals i, i+k, ...,
                                       cut into near-equal contiguous pieces; a node
                                       with k' < ppn senders receives the i'-th through
                                       locals ppn-1-i', ppn-1-i'-k', ... (piece c to the
                                       (c mod count)-th) */
#define NAPSPMV_NAP_DEDUP     0x10u /* the fully local (L2) step leaves out the indices
                                       the on_node -> off_node (L0) step already carries
                                       between the same two processes */
/* NAP three-way product (algorithm NAPSpMV, section 4.3): the same messages,
 * but the off-process block is split into its on_node and off_node parts and
 * each row sums its on_process, then on_node, then off_node entries (each in
 * stored order).  The on_node product runs on the caller's stream while the
 * inter-node hop and the scatter run on a helper stream of the plan, joined
 * by events before the off_node product.  Float64 w then equals that
 * three-part order bit for bit (not the two-part order of the default).
 * The helper stream and events belong to the plan: issue the applies of one
 * such plan from one host thread at a time (their order on the GPU is then
 * the call order).  Batches refuse such plans (EUNSUPPORTED); servers run
 * them alone. */
#define NAPSPMV_NAP_THREE_WAY 0x20u
/* NAP, direct reads: the off-process product reads every off-node ghost
 * value in place from the received inter-node buffer and every on-node one
 * from v, the way processes sharing a node's memory can read each other's
 * buffers; the off_node -> on_node and fully local steps move no data and
 * no ghost buffer is filled (napspmv_plan_read_ghost_values is then
 * EUNSUPPORTED).  Same messages, statistics and w.  EINVAL with
 * NAPSPMV_NAP_THREE_WAY. */
#define NAPSPMV_NAP_DIRECT    0x80u
/* Strided partition (section 5): row r, and v_r, on process r mod n_p
 * (row_starts must be NULL; EINVAL with NAPSPMV_NAP_SPLIT, whose pieces
 * follow index order).  The plan, its exports and napspmv_apply work in the
 * process-major numbering that a distributed code stores: position
 * starts[p] + q holds row p + q n_p, with starts[p] = the rows of processes
 * before p.  napspmv_plan_rows gives the original row of every position;
 * v and w of an apply are in process-major order. */
#define NAPSPMV_PARTITION_STRIDED 0x40u

/* Stages of an apply; napspmv_apply runs LOCAL then REMOTE.  LOCAL is one
 * launch: the exchange gather (standard: every ghost from its owner; NAP:
 * the inter-node send buffer) overlapped with the on-process product
 * w = A_on v.  For NAP, the scatter of received and fully local values into
 * the ghost buffer runs band by band inside LOCAL when the exchange is
 * received in place (each band's pack, then its scatter), else in REMOTE
 * after the inter-node hop.  REMOTE: that hop and scatter when not done in
 * LOCAL, then (both modes) the off-process product w += A_off ghost. */
#define NAPSPMV_STAGE_LOCAL  0
#define NAPSPMV_STAGE_REMOTE 1

typedef struct napspmv_plan_s *napspmv_plan_t;
typedef struct napspmv_batch_s *napspmv_batch_t;

/* Per-phase message statistics (section 5 reports the per-process maxima).
 * Element counts are vector values; bytes moved = elems * value_bytes. */
typedef struct {
    int64_t msgs;            /* messages in the phase */
    int64_t elems;           /* vector values carried, summed over messages */
    int64_t max_msgs_sent;   /* most messages sent by one process */
    int64_t max_elems_sent;  /* most values sent by one process */
    int64_t max_msgs_recv;   /* most messages received by one process */
    int64_t max_elems_recv;  /* most values received by one process */
    int64_t max_msg_elems;   /* largest single message */
} napspmv_phase_stats_t;

typedef struct {
    int64_t n, nnz, n_p, ppn, n_nodes;
    int32_t mode, dtype;
    int64_t value_bytes;     /* size of one vector element: 8 (F64) or 4 (F32, BF16) */
    int64_t nnz_on;          /* stored entries whose column the row's process owns */
    int64_t nnz_off;         /* stored entries whose column is a ghost */
    int64_t ghosts;          /* G: sum over processes of their unique ghost columns */
    napspmv_phase_stats_t phase[4];   /* indexed by NAPSPMV_PHASE_* */
    int64_t device_bytes;    /* device memory held by the plan (0 for host-only) */
    double build_seconds;    /* host wall time of the plan build */
    double upload_seconds;   /* host wall time of the device upload */
    uint32_t flags;          /* the NAPSPMV_* plan flags the plan was built with */
} napspmv_stats_t;

/*
 * Build a plan for w = A v.
 *
 * rowptr[n+1], col[nnz], val[nnz]: A in CSR form on the host; nnz = rowptr[n].
 *   rowptr[0] must be 0 and rowptr nondecreasing; 0 <= col[k] < n.  Entries
 *   of a row may come in any order and may repeat a column (repeats are
 *   summed by the product and counted once by the plan).  A stored entry is
 *   a nonzero even if its value is 0: the plan depends on the pattern only.
 *   val holds `dtype` elements (double, float, or uint16 bfloat16 bits); the
 *   library never rounds values.
 * n_p, ppn: processes and processes per node; need n_p >= 1, ppn >= 1,
 *   ppn dividing n_p and n >= n_p.
 * row_starts: NULL for the even contiguous partition of section 2, rank r
 *   owning rows [r*floor(n/n_p), (r+1)*floor(n/n_p)) and the last rank also
 *   the n mod n_p remainder; or n_p+1 strictly increasing boundaries from 0
 *   to n.
 * mode: NAPSPMV_STANDARD or NAPSPMV_NAP.  flags: NAPSPMV_* plan flags.
 * plan_out: receives the plan (set to NULL on failure; nothing leaks).
 * stats_out: optional (may be NULL).
 *
 * Limits: n, nnz and the ghost count must be below 2^31 - 2^16 (EUNSUPPORTED).
 * Without NAPSPMV_HOST_ONLY the plan copies the split matrix and its index
 * lists to the current GPU and allocates its ghost, send and receive buffers
 * there; this call synchronizes with the device.
 */
NAPSPMV_API int napspmv_plan_create(const int64_t *rowptr, const int32_t *col, const void *val,
                        int dtype, int64_t n, int64_t n_p, int64_t ppn, int mode,
                        const int64_t *row_starts, uint32_t flags,
                        napspmv_plan_t *plan_out, napspmv_stats_t *stats_out);

/*
 * A NAP plan with a third hierarchy level (section 6 leaves splitting
 * intra-node messages into on-socket and off-socket ones to future work; the
 * introduction notes that socket information could be used the way node
 * information is).  Sockets hold procs_per_socket consecutive ranks (it must
 * divide ppn).  The inter-node messages and the three intra-node steps are
 * those of the NAP plan (phases INTER, L0, L1, L2, and napspmv_stats_t's
 * phase statistics); each intra-node step then travels as section 4 routes
 * inter-node messages, one level down: its messages inside a socket go
 * directly; for every ordered socket pair (a, b) of a node the union F(a, b)
 * of its other indices from a to b goes in one message from a socket sender
 * of a to a socket receiver of b (the partners of a ranked by |F(a, b)|
 * descending, ties by ascending socket, the k-th sent by rank k mod
 * procs_per_socket of a; the senders to b ranked by |F(b, a)| descending,
 * ties by ascending socket, the k-th received by rank procs_per_socket - 1 -
 * (k mod procs_per_socket) of b); each index's holder (its owner, or for
 * L1 the inter-node receiver) hands it to the socket sender first, and the
 * socket receiver forwards it to the other ranks of b that need it.
 * procs_per_socket = ppn or 1 gives the NAP plan's messages.  Arguments as
 * napspmv_plan_create (mode NAP); flags may hold NAPSPMV_HOST_ONLY and
 * NAPSPMV_PARTITION_STRIDED only (EINVAL otherwise).  On the device the
 * cross-socket messages of L2 are gathered from v with the inter-node send
 * buffer, those of L1 are copied from the received buffer into a
 * cross-socket buffer, and the ghosts they serve read those buffers;
 * napspmv_apply gives the NAP plan's w bit for bit.
 */
NAPSPMV_API int napspmv_plan_create_sockets(const int64_t *rowptr, const int32_t *col,
                                            const void *val, int dtype, int64_t n, int64_t n_p,
                                            int64_t ppn, int64_t procs_per_socket,
                                            const int64_t *row_starts, uint32_t flags,
                                            napspmv_plan_t *plan_out, napspmv_stats_t *stats_out);

/* Statistics of the 12 socket-level phases (out[NAPSPMV_PHASE_SOCKET(step,
 * part) - 4], caller-owned, may be NULL) and the plan's procs_per_socket (0
 * if it has no socket level; may be NULL).  EINVAL for out on a plan
 * without a socket level. */
NAPSPMV_API int napspmv_plan_socket_stats(napspmv_plan_t plan, int64_t *procs_per_socket,
                                          napspmv_phase_stats_t *out);

/* The same socket split as a filter of any plan's own messages (section 6:
 * intra-node messages split into on-socket and off-socket).  Sockets hold
 * procs_per_socket consecutive ranks (it must divide ppn).  out[2 phase]
 * receives the
 * statistics of the phase's messages whose source and destination share a
 * socket, out[2 phase + 1] those of the others (8 entries, caller-owned).
 * Inter-node messages are always off-socket.  Works for host-only plans. */
NAPSPMV_API int napspmv_plan_level_stats(napspmv_plan_t plan, int64_t procs_per_socket,
                                         napspmv_phase_stats_t *out);

/* rows_out[k] (n entries, caller-owned host array) = the original row index
 * held at position k of the plan's numbering: k itself unless the plan was
 * built with NAPSPMV_PARTITION_STRIDED.  Works for host-only plans. */
NAPSPMV_API int napspmv_plan_rows(napspmv_plan_t plan, int64_t *rows_out);

/*
 * w = A v on the GPU, asynchronously on `stream` (standard_spmv or NAPSpMV,
 * sections 2.1 and 4.3): fill the ghost buffer from v along the plan's
 * messages, then the split product.
 *
 * v, w: device arrays of n elements (double for F64 plans, float otherwise),
 *   caller-owned, not overlapping.  No allocation, no host synchronization,
 *   no host-device copy.  The plan's ghost/send/receive buffers are reused,
 *   so at most one apply per plan may be in flight at a time (applies on one
 *   stream are ordered, which suffices).
 */
NAPSPMV_API int napspmv_apply(napspmv_plan_t plan, const void *v, void *w, void *stream);

/* One stage of napspmv_apply (NAPSPMV_STAGE_*), for per-stage timing.
 * STAGE_REMOTE reads the ghost buffer and partial w the last STAGE_LOCAL
 * wrote. */
NAPSPMV_API int napspmv_apply_stage(napspmv_plan_t plan, int stage, const void *v, void *w,
                        void *stream);

/* Bytes of a caller-owned workspace for this plan: the ghost buffer and, for
 * NAP plans, the inter-node send (and receive) buffers. */
NAPSPMV_API int64_t napspmv_plan_workspace_bytes(napspmv_plan_t plan);

/* napspmv_apply with a caller-owned workspace `ws` (device memory of
 * napspmv_plan_workspace_bytes bytes, 256-byte aligned; NULL = the plan's
 * own).  Applies of one plan with different workspaces may be in flight at
 * the same time (on different streams); the workspace must not be shared by
 * two applies in flight.  Allocates nothing. */
NAPSPMV_API int napspmv_apply_ws(napspmv_plan_t plan, void *ws, const void *v, void *w,
                                 void *stream);

/*
 * napspmv_apply for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels and result bits as napspmv_apply_ws, but the
 * workspace is a static array of the library (64 MiB, see
 * napspmv_noalloc_max_workspace_bytes; held on each GPU the library runs on
 * until the process ends) instead of the plan's own or the caller's.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library call);
 * the first call on a GPU looks up the array's device address once.  A plan
 * whose workspace (napspmv_plan_workspace_bytes) is larger is refused with
 * NAPSPMV_EUNSUPPORTED.  Every call on one GPU shares the one array: calls
 * whose applies overlap on the device (on different streams, or from
 * different threads) race and give wrong results; applies issued on one
 * stream are ordered and safe.  No part of the array needs to start at
 * zero: an apply writes every position it later reads.
 */
NAPSPMV_API int napspmv_apply_noalloc(napspmv_plan_t plan, const void *v, void *w, void *stream);
NAPSPMV_API int64_t napspmv_noalloc_max_workspace_bytes(void);

/*
 * Batched applies: `count` independent products w[i] = A_i v[i] (plans
 * plans[i], different matrices or the same one with different workspaces)
 * in one launch sequence -- one first launch over every product's exchange
 * and on-process work, one NAP scatter launch if any plan is NAP, one second
 * launch over every off-process product (one per REMOTE_NNZ among the
 * plans).  All plans must share the value type, BLOCK_NNZ and VWINDOW (else
 * EINVAL), be on the batch's device, receive
 * NAP messages in place and use the two-part product (no NAPSPMV_NAP_THREE_WAY).  ws may be NULL (every plan's own workspace) or hold
 * per-product workspaces (NULL entries = the plan's own).  The batch object
 * owns a ring of 4 device descriptor tables (each with a pinned host copy)
 * for up to max_count products: call k uploads table k mod 4 with an
 * asynchronous copy, and waits for the device only if the call 4 before it
 * has not yet been read.  Use one batch object per stream.  A graph that
 * captures a call replays the upload of that call's table, which later
 * calls of the same object overwrite: give captured calls a batch object of
 * their own.  napspmv_batch_apply allocates nothing.
 */
NAPSPMV_API int napspmv_batch_create(int max_count, napspmv_batch_t *out);
NAPSPMV_API int napspmv_batch_apply(napspmv_batch_t batch, int count, const napspmv_plan_t *plans,
                                    void *const *ws, const void *const *v, void *const *w,
                                    void *stream);
NAPSPMV_API int napspmv_batch_destroy(napspmv_batch_t batch);

/* Per-partition applies (standard plans): the rows of one process only --
 * its own ghost gather and its split product -- as one pair of launches,
 * the way each process of standard_spmv (section 2.1) computes its rows.
 * prepare builds the per-partition launch schedules (allocates, synchronizes);
 * apply_partition allocates nothing. */
NAPSPMV_API int napspmv_plan_prepare_partitions(napspmv_plan_t plan);
NAPSPMV_API int napspmv_apply_partition(napspmv_plan_t plan, int64_t part, const void *v, void *w,
                                        void *stream);

/* A HIP graph (hipGraphExec_t, returned as void*) that replays
 * napspmv_apply(plan, v, w) on the stream it is launched on.  The graph
 * holds the plan's pointers: destroy it before the plan, and re-create it
 * after changing a tuning parameter. */
NAPSPMV_API int napspmv_graph_create(napspmv_plan_t plan, const void *v, void *w, void **graph_out);
NAPSPMV_API int napspmv_graph_launch(void *graph, void *stream);
NAPSPMV_API int napspmv_graph_destroy(void *graph);

/* Autotuner: times every (BLOCK_NNZ, VWINDOW, GATHER_ITEM) candidate, then
 * every REMOTE_NNZ with the best of those, on
 * this plan with `reps` applies each (HIP events on `stream`; w is
 * overwritten) and keeps the fastest.  With cache_path (may be NULL), a
 * result already cached for the same device and workload shape is used
 * without timing, and a new result is appended.  *best_ms (may be NULL)
 * receives the best time per apply, or -1 when the cache answered.  No
 * candidate changes any result bit.  Synchronizes; may allocate. */
NAPSPMV_API int napspmv_plan_autotune(napspmv_plan_t plan, const void *v, void *w, void *stream,
                                      int reps, const char *cache_path, double *best_ms);

/*
 * Serving engine (plan reuse over many products, the amortisation argument
 * of section 5).  Resident plans take requests w = A_id v; requests wait in
 * a queue until one of `slots` slots (each its own HIP stream) is free and
 * their workspace fits in `workspace_budget` bytes (0 = no cap; idle
 * workspaces of other plans are released to make room), and each free slot
 * then runs up to `max_batch` queued requests of one kernel group (value
 * type, BLOCK_NNZ, VWINDOW; oldest request first) as one batched launch
 * sequence (a NAP plan with NAPSPMV_EXCHANGE_COPY or NAPSPMV_NAP_THREE_WAY
 * always runs alone, by napspmv_apply_ws).  Requests that arrive while slots
 * are busy are admitted as slots free up, so their work overlaps the work
 * already on the device.  Single-threaded: one caller drives a server.
 * Every result is bitwise the result of napspmv_apply on the same plan and
 * vector.
 *
 * server_create makes no HIP call; the slots' streams, events and batch
 * tables are made on the current GPU when the first plan is added.
 * server_add_plan refuses a host-only plan (EINVAL) and a plan whose
 * workspace exceeds a non-zero budget (ENOMEM: its requests could never
 * run).  server_submit and server_replay take the caller's stream (void*
 * hipStream_t, NULL = the default stream): the server records an event on it
 * and runs the requests after the caller's work issued there before the call
 * (writes of v, w).  Results are ready once server_wait (or poll, or replay)
 * has reported the request done.
 * server_poll retires finished slots and admits queued requests; it returns
 * the number of requests completed by this call, or a negative error code
 * (ENOMEM if requests are queued, none is running and no workspace can be
 * allocated for them).
 * server_replay replays an arrival trace natively: request i (plan ids[i],
 * vectors v[i], w[i]) arrives arrival_ns[i] after the call starts; it
 * returns when every request is done, with latency_ns[i] = completion -
 * arrival and (if not NULL) batch_sizes[i] = the size of its batch.
 * server_reserve allocates, for every resident plan, workspaces until it
 * holds per_plan of them (within the budget; none is released), so that a
 * later replay or submit need not allocate.
 * Messages of failed server calls: napspmv_server_last_error().
 */
typedef struct napspmv_server_s *napspmv_server_t;
NAPSPMV_API int napspmv_server_create(int slots, int max_batch, int64_t workspace_budget,
                                      napspmv_server_t *out);
NAPSPMV_API int napspmv_server_add_plan(napspmv_server_t server, napspmv_plan_t plan, int *id_out);
NAPSPMV_API int napspmv_server_reserve(napspmv_server_t server, int per_plan);
NAPSPMV_API int napspmv_server_submit(napspmv_server_t server, int id, const void *v, void *w,
                                      void *stream, int64_t *ticket_out);
NAPSPMV_API int64_t napspmv_server_poll(napspmv_server_t server);
NAPSPMV_API int napspmv_server_wait(napspmv_server_t server, int64_t ticket);
NAPSPMV_API int napspmv_server_request_info(napspmv_server_t server, int64_t ticket,
                                            int64_t *submit_ns, int64_t *done_ns, int *batch_size);
NAPSPMV_API int napspmv_server_replay(napspmv_server_t server, int64_t n, const int *ids,
                                      const int64_t *arrival_ns, const void *const *v,
                                      void *const *w, void *stream, int64_t *latency_ns,
                                      int *batch_sizes);
NAPSPMV_API int64_t napspmv_server_workspace_bytes(napspmv_server_t server);
NAPSPMV_API const char *napspmv_server_last_error(void);
NAPSPMV_API int napspmv_server_destroy(napspmv_server_t server);

/* Copy the plan's statistics into *out. */
NAPSPMV_API int napspmv_plan_stats(napspmv_plan_t plan, napspmv_stats_t *out);

/*
 * Canonical export of one phase's messages (section 5's statistics are
 * computed from them), for bit-exact comparison: messages sorted by (src,
 * dst), indices ascending by global column inside a message, one message
 * per (src, dst) pair.  phase: NAPSPMV_PHASE_INTER .. L2, or a socket-level
 * phase NAPSPMV_PHASE_SOCKET(step, part) of a plan built with a socket level
 * (EINVAL otherwise).  Two-call pattern: pass NULL arrays to get *n_msgs and
 * *n_idx, then arrays of n_msgs (src, dst), n_msgs+1 (ptr) and n_idx (idx)
 * elements.
 */
NAPSPMV_API int napspmv_plan_export(napspmv_plan_t plan, int phase, int64_t *n_msgs, int64_t *n_idx,
                        int32_t *src, int32_t *dst, int64_t *ptr, int32_t *idx);

/* The ghost lists gh(t): ghost_ptr[n_p+1] offsets into ghost_col[G], each
 * list ascending.  Either array may be NULL. */
NAPSPMV_API int napspmv_plan_ghosts(napspmv_plan_t plan, int64_t *ghost_ptr, int32_t *ghost_col);

/* Diagnostic: copy the ghost buffer of workspace `ws` (NULL = the plan's own;
 * G elements of the vector type) into host memory `out`; synchronizes
 * `stream` first. */
NAPSPMV_API int napspmv_plan_read_ghost_values(napspmv_plan_t plan, const void *ws, void *out,
                                               void *stream);

/* Layout of the off-process row blocks of a device plan (the
 * local_spmv(A_off, ghosts) step of the split product, Algorithm 1), as
 * counts written to the caller's host int64 array kinds_out[3]:
 *   [0] plain   gather order, int32 ghost positions and 16-bit slots
 *   [1] packed  gather order, position and slot in one 32-bit word whose
 *               position is an offset from a base shared by 16 lanes
 *   [2] narrow  stored order, 16-bit positions from a per-block base
 * (blocks without entries are not counted; plans with direct reads count
 * every block as plain).  The layout never changes a result bit; it follows
 * BLOCK_NNZ and REMOTE_NNZ.  EINVAL for a NULL argument or a host-only
 * plan. */
NAPSPMV_API int napspmv_plan_block_kinds(napspmv_plan_t plan, int64_t *kinds_out);

/* Tuning parameters of the apply kernels (NAPSPMV_PARAM_*); -1 restores the
 * automatic value.  No parameter changes any result bit.  Setting one on a
 * device plan rebuilds and re-uploads the launch schedules (it allocates and
 * synchronizes the device): do not call it while an apply of the plan is in
 * flight.
 *   BLOCK_NNZ     entries per row block of the on-process product (a block
 *                 of several rows holds at most BLOCK_NNZ - 7, so that its
 *                 aligned vector loads stay within BLOCK_NNZ); the bands of
 *                 the exchange buffers hold BLOCK_NNZ * 8 bytes of v
 *                 (BLOCK_NNZ columns of a float64 vector, twice as many of
 *                 a float32 one): 1024, 2048, 4096, 8192 (automatic: 4096
 *                 for float64 values, 2048 for float32 and bfloat16)
 *   REMOTE_NNZ    entries per row block of the off-process product (at
 *                 most REMOTE_NNZ - 7 for a block of several rows): 1024,
 *                 2048, 4096, 8192 (automatic: 8192 when the plan has at
 *                 least 8192 off-process entries per process, else 4096)
 *   GATHER_ITEM   most entries of one exchange work item (a slice of one
 *                 band of the ghost or send buffer), 256 .. 2^24
 *                 (automatic: 65536).  A NAP plan that receives in place
 *                 packs and scatters whole bands in one item each when this
 *                 is automatic or at least the widest band of its send
 *                 buffer, else it keeps the separate scatter launch.
 *   VWINDOW       on-process product: most elements of v a row block stages
 *                 in LDS, 0 (none), 1024, 2048, 4096 (automatic: 1024)

 * get_param returns the value in effect, or a negative error code. */
#define NAPSPMV_PARAM_BLOCK_NNZ    0
#define NAPSPMV_PARAM_GATHER_ITEM  1
#define NAPSPMV_PARAM_VWINDOW      2
#define NAPSPMV_PARAM_REMOTE_NNZ   3

NAPSPMV_API int napspmv_plan_set_param(napspmv_plan_t plan, int param, int value);
NAPSPMV_API int napspmv_plan_get_param(napspmv_plan_t plan, int param);

/* Release the plan and its device memory.  NULL is accepted.  The caller
 * must not destroy a plan with an apply in flight. */
NAPSPMV_API int napspmv_plan_destroy(napspmv_plan_t plan);

/* Process-wide cap on device memory held by all live plans; 0 (the
 * default) means no cap.  A create that would exceed it fails with
 * NAPSPMV_ENOMEM before allocating anything. */
NAPSPMV_API int napspmv_set_device_budget(int64_t bytes);
NAPSPMV_API int64_t napspmv_device_bytes_in_use(void);

/* Message for the last failed call on this thread ("" if none). */
NAPSPMV_API const char *napspmv_last_error(void);

/* Interface version (major * 100 + minor). */
NAPSPMV_API int napspmv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NAPSPMV_H */
