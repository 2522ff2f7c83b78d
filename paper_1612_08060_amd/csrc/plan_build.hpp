// Host-side construction of standard and node-aware communication plans.
//
// Section 2 (row blocks, ranks as (local, node) pairs), section 2.1 (the
// standard messages P(r), D(r, t)) and section 4 (node sets N, E; the T/U
// mapping; inter-node messages G, I; the three local steps) of Bienz, Gropp,
// Olson, "Node aware sparse matrix-vector multiplication".
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace napspmv {

// Error raised by the builder; `code` is a NAPSPMV_E* value.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

// One phase in canonical order: messages sorted by (src, dst), indices of a
// message ascending, message k's indices are idx[ptr[k] .. ptr[k+1]).
struct Phase {
    std::vector<int32_t> src, dst;
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> idx;
};

struct PhaseStats {
    int64_t msgs = 0, elems = 0, max_msgs_sent = 0, max_elems_sent = 0;
    int64_t max_msgs_recv = 0, max_elems_recv = 0, max_msg_elems = 0;
};

struct HostPlan {
    int64_t n = 0, nnz = 0, n_p = 0, ppn = 0, n_nodes = 0;
    int mode = 0, dtype = 0;
    int64_t value_size = 8;            // bytes of one stored value of A
    std::vector<int64_t> starts;       // row block boundaries, n_p + 1
    // Strided partition (row r on process r mod n_p): the plan works on the
    // process-major renumbering (position starts[r mod n_p] + r div n_p);
    // rows_natural[k] is the original row at position k.  Empty otherwise.
    bool strided = false;
    std::vector<int32_t> rows_natural;
    std::vector<int64_t> ghost_ptr;    // n_p + 1
    std::vector<int32_t> ghost_col;    // G, each process's list ascending
    int64_t nnz_on = 0, nnz_off = 0;

    // Split CSR as the device reads it (section 2, the on_process and
    // off_process blocks): two CSR matrices over the same rows, each keeping
    // the stored order of its entries.  col_on holds columns of v; col_off
    // holds positions in the concatenated ghost buffer.
    std::vector<int32_t> rowptr_on, col_on;      // n + 1, nnz_on
    std::vector<uint8_t> val_on;                 // nnz_on * value_size
    std::vector<int32_t> rowptr_off, col_off;    // n + 1, nnz_off
    std::vector<uint8_t> val_off;                // nnz_off * value_size
    // Three-way plans only: the on_node part of the off-process block (ghosts
    // owned by another process of the row's node), taken out of
    // rowptr_off/col_off/val_off, which then hold the off_node part.
    // nnz_off still counts both parts.
    bool three_way = false;
    bool direct = false;       // NAP direct reads (no ghost buffer on the device)
    std::vector<int32_t> rowptr_nd, col_nd;      // n + 1, nnz_nd
    std::vector<uint8_t> val_nd;                 // nnz_nd * value_size
    int64_t nnz_nd = 0;
    // Smallest and largest on-process column of each row (lo > hi if none):
    // the window of v a row block reads directly.
    std::vector<int32_t> on_lo, on_hi;

    Phase phase[4];                    // INTER, L0, L1, L2
    PhaseStats stats[4];

    // Third hierarchy level (sockets of `pps` consecutive ranks; 0 = none):
    // the socket routes of the three intra-node steps, sock_phase[4 (s - 1)
    // + part] for step s = L0, L1, L2 and part = on, gather, cross,
    // scatter (NAPSPMV_PHASE_L0_ON ... minus 4).
    int64_t pps = 0;
    Phase sock_phase[12];
    PhaseStats sock_stats[12];

    // Device index lists.
    std::vector<int32_t> gather_idx;              // standard: ghost[k] = v[gather_idx[k]]
    // NAP: send[k] = v[pack_idx[k]]: the inter-node messages in canonical
    // order, then (socket plans) the cross-socket messages of the fully
    // local step; pack_group[k] groups the entries of one destination (node
    // or socket) inside a column band of the send buffer
    std::vector<int32_t> pack_idx, pack_group;
    // socket plans: cross-socket messages of the off_node -> on_node step,
    // l1x[k] = recv[l1x_src[k]] (entries of the send buffer), column
    // l1x_col[k], grouped by destination socket
    std::vector<int32_t> l1x_col, l1x_src, l1x_group;
    // NAP: ghost[scat_dst[k]] = received value scat_src[k] (an entry of the
    // send buffer, or pack_idx.size() + an entry of l1x);
    // ghost[l2_dst[k]] = v[l2_src[k]]
    std::vector<int32_t> scat_src, scat_dst;
    std::vector<int32_t> l2_src, l2_dst;
};

// Validates the inputs and builds the plan.  `variant` holds NAPSPMV_NAP_*
// flags (NAP mode only); `strided` selects the strided partition (then
// row_starts must be NULL).  Throws Error or std::bad_alloc.
// `pps` > 0 (NAP mode, no variant) adds the socket level: sockets of pps
// consecutive ranks (pps dividing ppn).
void build_plan(HostPlan &hp, const int64_t *rowptr, const int32_t *col, const void *val,
                int dtype, int64_t n, int64_t n_p, int64_t ppn, int mode,
                const int64_t *row_starts, uint32_t variant, bool strided = false,
                int64_t pps = 0);

// Message statistics split by a third hierarchy level (section 6 names
// on-socket and off-socket intra-node messages): sockets of `pps`
// consecutive ranks; out[2 ph] = messages of phase ph whose source and
// destination share a socket, out[2 ph + 1] = the others.
void level_stats(const HostPlan &hp, int64_t pps, PhaseStats out[8]);

// Frees the host copy of the on-process block after upload.  Row pointers,
// row windows, the off-process (and on_node) entries and the exchange index
// lists stay: launch schedules, the band layout of the exchange buffers and
// the gather order of the off-process blocks are rebuilt from them when the
// block size changes.
void release_device_arrays(HostPlan &hp);

}  // namespace napspmv
