// Host construction of the communication plans.  See plan_build.hpp.
//
// Everything is built by sorting and cutting runs, never by sets of sets:
//  * gh(t), the off-process columns of process t, sorted and unique, is the
//    union over its rows of the off_process block (section 2).
//  * Standard messages (section 2.1): since gh(t) is sorted and every owner
//    holds a contiguous column range, the runs of gh(t) with equal owner r
//    are exactly D(r, t), and the ghost buffer of t is t's receive buffer in
//    arrival order.
//  * E(n, m) (section 4.1): for destination node m, the off-node columns of
//    gh(t) over the processes t of m, sorted and unique; its runs by source
//    node are E(n, m) for every n.
//  * T/U mapping (rule stated after the definitions of T and U): the partners
//    of node n sorted by (|E(n, m)| descending, m ascending), the k-th sent
//    by local process k mod ppn; the senders to node n sorted by the same key
//    (what n sends to each of them, 0 if nothing), the k-th received by local
//    process ppn - 1 - (k mod ppn).  No partner is split over processes.
//  * I((p, n), (q, m)) = E(n, m) between the T-process and the U-process.
//  * Variants (flags): the owner mapping (the T-process of a pair is the
//    local process owning most of E(n, m)), the split of a partner over
//    several processes when a node has fewer partners or senders than ppn
//    (section 4.1), and the fully local step deduplicated against the
//    on_node -> off_node step; and the three-way product, which keeps the
//    sets and splits the off-process block into its on_node and off_node
//    parts (algorithm NAPSpMV's three local products).
//  * on_node -> off_node (L0): the indices of the inter-node messages sent by
//    s that s does not own, unique per (owner, s).
//  * off_node -> on_node (L1): every off-node ghost j of t arrives at the
//    U-process q of its node pair; if q != t, q forwards it to t.
//  * on_node -> on_node (L2): the runs of gh(t) owned by another process of
//    t's node (the standard intra-node messages).
//  * Socket level (a third level of the hierarchy, which section 6 leaves
//    to future work): sockets of pps consecutive ranks route each of the
//    three intra-node steps as section 4 routes inter-node messages, one
//    level down.  The step's messages whose ranks share a socket stay; for
//    an ordered socket pair (a, b) of a node, F(a, b) = the sorted union of
//    the indices its other messages carry from a to b; the partners of a are
//    ranked by (|F(a, b)| descending, b ascending), the k-th sent by rank
//    k mod pps of a, the senders to b by (|F(b, a)| descending, a
//    ascending), the k-th received by rank pps - 1 - (k mod pps) of b; the
//    holder of each index (unique in a node) hands it to the socket sender,
//    and the socket receiver forwards it to the other ranks of b whose
//    message carried it.
#include "plan_build.hpp"

#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>

#include <omp.h>

#include "napspmv.h"

namespace napspmv {
namespace {

// Sizes stay below 2^31 - 2^16 so that every 32-bit index a kernel forms
// (an index plus at most one block's worth of work) is representable.
constexpr int64_t kInt32Max = 0x7fffffff - 0x10000;

constexpr uint32_t kVariantFlags =
    NAPSPMV_NAP_OWNER_MAP | NAPSPMV_NAP_SPLIT | NAPSPMV_NAP_DEDUP | NAPSPMV_NAP_THREE_WAY |
    NAPSPMV_NAP_DIRECT;

struct Owner {
    const std::vector<int64_t> &starts;
    int64_t block;     // > 0 for the even partition (fast path)
    int64_t n_p;
    int64_t operator()(int64_t j) const {
        if (block > 0) {
            int64_t r = j / block;
            return r < n_p ? r : n_p - 1;
        }
        return (std::upper_bound(starts.begin(), starts.end(), j) - starts.begin()) - 1;
    }
};

// A message before canonical ordering: `len` indices at `data`.
struct MsgRef {
    int32_t src, dst;
    const int32_t *data;
    int64_t len;
};

void finalize_phase(std::vector<MsgRef> &refs, Phase &ph) {
    std::sort(refs.begin(), refs.end(), [](const MsgRef &a, const MsgRef &b) {
        return a.src != b.src ? a.src < b.src : a.dst < b.dst;
    });
    const size_t m = refs.size();
    ph.src.resize(m);
    ph.dst.resize(m);
    ph.ptr.assign(m + 1, 0);
    for (size_t k = 0; k < m; ++k) {
        ph.src[k] = refs[k].src;
        ph.dst[k] = refs[k].dst;
        ph.ptr[k + 1] = ph.ptr[k] + refs[k].len;
    }
    ph.idx.resize(ph.ptr[m]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < (int64_t)m; ++k)
        std::memcpy(ph.idx.data() + ph.ptr[k], refs[k].data, sizeof(int32_t) * refs[k].len);
}

// A (src, dst, index) triple of a message.
struct Trip {
    int32_t s, d, j;
    bool operator<(const Trip &o) const {
        return s != o.s ? s < o.s : d != o.d ? d < o.d : j < o.j;
    }
    bool operator==(const Trip &o) const { return s == o.s && d == o.d && j == o.j; }
};

// A phase from triples already sorted by (src, dst, index) and unique.
void phase_from_sorted_triples(const std::vector<Trip> &t, Phase &ph) {
    ph = Phase();
    ph.idx.resize(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
        if (k == 0 || t[k].s != t[k - 1].s || t[k].d != t[k - 1].d) {
            if (k) ph.ptr.push_back((int64_t)k);
            ph.src.push_back(t[k].s);
            ph.dst.push_back(t[k].d);
        }
        ph.idx[k] = t[k].j;
    }
    if (!t.empty()) ph.ptr.push_back((int64_t)t.size());
}

// The socket route of one intra-node step `in` (see the file comment):
// out[0..3] = its on-socket, gather, cross and scatter messages.  For the
// cross messages, also the sorted keys (destination socket) * n + index
// (`cross_key`) with the position of each in out[2].idx (`cross_pos`).
// Nodes are independent: each node's messages (a contiguous run of `in`,
// sorted by source) are routed in parallel and the results concatenated,
// which keeps every phase sorted by (source, destination).
void socket_route(const Phase &in, int64_t n, int64_t ppn, int64_t pps, Phase out[4],
                  std::vector<int64_t> *cross_key = nullptr,
                  std::vector<int64_t> *cross_pos = nullptr) {
    const int64_t m = (int64_t)in.src.size();
    const int64_t n_nodes = m ? in.src[m - 1] / ppn + 1 : 0;
    std::vector<int64_t> first(n_nodes + 1, m);
    for (int64_t k = m - 1; k >= 0; --k) first[in.src[k] / ppn] = k;
    for (int64_t x = n_nodes - 1; x >= 0; --x) first[x] = std::min(first[x], first[x + 1]);
    struct NodeOut {
        std::vector<MsgRef> on;
        std::vector<Trip> gather, cross, scatter;
    };
    std::vector<NodeOut> per(n_nodes);
    bool two_holders = false;
#pragma omp parallel for schedule(dynamic, 1) reduction(|| : two_holders)
    for (int64_t node = 0; node < n_nodes; ++node) {
        NodeOut &o = per[node];
        struct Off {
            int32_t a, b;      // source and destination socket
            int32_t j, x, y;   // index, holder, user
        };
        std::vector<Off> off;
        for (int64_t k = first[node]; k < first[node + 1]; ++k) {
            const int32_t a = (int32_t)(in.src[k] / pps), b = (int32_t)(in.dst[k] / pps);
            const int64_t len = in.ptr[k + 1] - in.ptr[k];
            if (a == b) {
                o.on.push_back(MsgRef{in.src[k], in.dst[k], in.idx.data() + in.ptr[k], len});
                continue;
            }
            for (int64_t e = in.ptr[k]; e < in.ptr[k + 1]; ++e)
                off.push_back(Off{a, b, in.idx[e], in.src[k], in.dst[k]});
        }
        std::sort(off.begin(), off.end(), [](const Off &u, const Off &v) {
            return u.a != v.a ? u.a < v.a : u.b != v.b ? u.b < v.b : u.j != v.j ? u.j < v.j : u.y < v.y;
        });
        // F(a, b): unique (a, b, j) with its holder; a holder is unique per
        // (a, j) inside the node
        struct FE {
            int32_t a, b, j, h;
        };
        std::vector<FE> F;
        for (size_t k = 0; k < off.size(); ++k)
            if (k == 0 || off[k].a != off[k - 1].a || off[k].b != off[k - 1].b || off[k].j != off[k - 1].j)
                F.push_back(FE{off[k].a, off[k].b, off[k].j, off[k].x});
        {
            std::vector<std::pair<int64_t, int32_t>> hold(F.size());
            for (size_t k = 0; k < F.size(); ++k) hold[k] = {(int64_t)F[k].a * n + F[k].j, F[k].h};
            std::sort(hold.begin(), hold.end());
            for (size_t k = 1; k < hold.size(); ++k)
                if (hold[k].first == hold[k - 1].first && hold[k].second != hold[k - 1].second)
                    two_holders = true;
        }
        struct SP {
            int32_t a, b;
            int64_t begin, end, vol = 0, back = 0;
            int32_t sender = 0, receiver = 0;
        };
        std::vector<SP> sp;
        for (size_t k = 0; k < F.size(); ++k) {
            if (k == 0 || F[k].a != F[k - 1].a || F[k].b != F[k - 1].b)
                sp.push_back(SP{F[k].a, F[k].b, (int64_t)k, (int64_t)k});
            sp.back().end = (int64_t)k + 1;
        }
        for (SP &q : sp) q.vol = q.end - q.begin;
        for (SP &q : sp)
            for (const SP &r : sp)
                if (r.a == q.b && r.b == q.a) q.back = r.vol;
        std::vector<size_t> ord(sp.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
            const SP &u = sp[x], &v = sp[y];
            if (u.a != v.a) return u.a < v.a;
            if (u.vol != v.vol) return u.vol > v.vol;
            return u.b < v.b;
        });
        for (size_t k = 0, run = 0; k < ord.size(); ++k) {
            run = (k > 0 && sp[ord[k]].a == sp[ord[k - 1]].a) ? run + 1 : 0;
            sp[ord[k]].sender = (int32_t)(sp[ord[k]].a * pps + (int64_t)run % pps);
        }
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
            const SP &u = sp[x], &v = sp[y];
            if (u.b != v.b) return u.b < v.b;
            if (u.back != v.back) return u.back > v.back;
            return u.a < v.a;
        });
        for (size_t k = 0, run = 0; k < ord.size(); ++k) {
            run = (k > 0 && sp[ord[k]].b == sp[ord[k - 1]].b) ? run + 1 : 0;
            sp[ord[k]].receiver = (int32_t)(sp[ord[k]].b * pps + pps - 1 - (int64_t)run % pps);
        }
        for (const SP &q : sp)
            for (int64_t k = q.begin; k < q.end; ++k) {
                o.cross.push_back(Trip{q.sender, q.receiver, F[k].j});
                if (F[k].h != q.sender) o.gather.push_back(Trip{F[k].h, q.sender, F[k].j});
            }
        size_t q = 0;
        for (const Off &f : off) {
            while (sp[q].a != f.a || sp[q].b != f.b) ++q;     // off and sp share the (a, b) order
            if (f.y != sp[q].receiver) o.scatter.push_back(Trip{sp[q].receiver, f.y, f.j});
        }
        for (auto *t : {&o.cross, &o.gather, &o.scatter}) {
            std::sort(t->begin(), t->end());
            t->erase(std::unique(t->begin(), t->end()), t->end());
        }
    }
    if (two_holders) throw Error(NAPSPMV_EINVAL, "socket level: an index with two holders on one socket");
    std::vector<MsgRef> on;
    for (const NodeOut &o : per) on.insert(on.end(), o.on.begin(), o.on.end());
    finalize_phase(on, out[0]);
    auto concat = [&](std::vector<Trip> NodeOut::*part, Phase &ph) {
        std::vector<Trip> all;
        size_t total = 0;
        for (const NodeOut &o : per) total += (o.*part).size();
        all.reserve(total);
        for (NodeOut &o : per) {
            all.insert(all.end(), (o.*part).begin(), (o.*part).end());
            std::vector<Trip>().swap(o.*part);
        }
        phase_from_sorted_triples(all, ph);
    };
    concat(&NodeOut::gather, out[1]);
    concat(&NodeOut::cross, out[2]);
    concat(&NodeOut::scatter, out[3]);
    if (cross_key) {
        const Phase &c = out[2];
        const int64_t nm = (int64_t)c.src.size();
        std::vector<int64_t> cfirst(n_nodes + 1, nm);
        for (int64_t k = nm - 1; k >= 0; --k) cfirst[c.src[k] / ppn] = k;
        for (int64_t x = n_nodes - 1; x >= 0; --x) cfirst[x] = std::min(cfirst[x], cfirst[x + 1]);
        cross_key->assign(c.idx.size(), 0);
        cross_pos->assign(c.idx.size(), 0);
        // per node, sorted by (destination socket, index); the destination
        // sockets of successive nodes ascend, so the concatenation is sorted
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t node = 0; node < n_nodes; ++node) {
            const int64_t e0 = cfirst[node] < nm ? c.ptr[cfirst[node]] : (int64_t)c.idx.size();
            const int64_t e1 = cfirst[node + 1] < nm ? c.ptr[cfirst[node + 1]] : (int64_t)c.idx.size();
            std::vector<std::pair<int64_t, int64_t>> kp;
            kp.reserve((size_t)(e1 - e0));
            for (int64_t k = cfirst[node]; k < cfirst[node + 1]; ++k)
                for (int64_t e = c.ptr[k]; e < c.ptr[k + 1]; ++e)
                    kp.emplace_back((int64_t)(c.dst[k] / pps) * n + c.idx[e], e);
            std::sort(kp.begin(), kp.end());
            for (size_t x = 0; x < kp.size(); ++x) {
                (*cross_key)[e0 + x] = kp[x].first;
                (*cross_pos)[e0 + x] = kp[x].second;
            }
        }
    }
}

int64_t lookup(const std::vector<int64_t> &keys, const std::vector<int64_t> &vals, int64_t key) {
    auto it = std::lower_bound(keys.begin(), keys.end(), key);
    if (it == keys.end() || *it != key) throw Error(NAPSPMV_EINVAL, "socket level: missing route");
    return vals[it - keys.begin()];
}

// Statistics of the messages of `ph` for which keep(k) holds (all if null).
PhaseStats phase_stats(const Phase &ph, int64_t n_p, const std::function<bool(size_t)> &keep = nullptr) {
    PhaseStats s;
    const size_t m = ph.src.size();
    std::vector<int64_t> ms(n_p, 0), es(n_p, 0), mr(n_p, 0), er(n_p, 0);
    for (size_t k = 0; k < m; ++k) {
        if (keep && !keep(k)) continue;
        int64_t len = ph.ptr[k + 1] - ph.ptr[k];
        s.msgs += 1;
        s.elems += len;
        ms[ph.src[k]] += 1;
        es[ph.src[k]] += len;
        mr[ph.dst[k]] += 1;
        er[ph.dst[k]] += len;
        s.max_msg_elems = std::max(s.max_msg_elems, len);
    }
    for (int64_t r = 0; r < n_p; ++r) {
        s.max_msgs_sent = std::max(s.max_msgs_sent, ms[r]);
        s.max_elems_sent = std::max(s.max_elems_sent, es[r]);
        s.max_msgs_recv = std::max(s.max_msgs_recv, mr[r]);
        s.max_elems_recv = std::max(s.max_elems_recv, er[r]);
    }
    return s;
}

void validate(const int64_t *rowptr, const int32_t *col, const void *val, int dtype, int64_t n,
              int64_t n_p, int64_t ppn, int mode, const int64_t *row_starts) {
    if (!rowptr) throw Error(NAPSPMV_EINVAL, "rowptr is NULL");
    if (dtype != NAPSPMV_F64 && dtype != NAPSPMV_F32 && dtype != NAPSPMV_BF16)
        throw Error(NAPSPMV_EINVAL, "dtype must be F64, F32 or BF16");
    if (mode != NAPSPMV_STANDARD && mode != NAPSPMV_NAP)
        throw Error(NAPSPMV_EINVAL, "mode must be STANDARD or NAP");
    if (n_p < 1 || ppn < 1) throw Error(NAPSPMV_EINVAL, "need n_p >= 1 and ppn >= 1");
    if (n_p % ppn != 0) throw Error(NAPSPMV_EINVAL, "ppn must divide n_p");
    if (n < n_p) throw Error(NAPSPMV_EINVAL, "need n >= n_p (one row per process at least)");
    if (n > kInt32Max) throw Error(NAPSPMV_EUNSUPPORTED, "n must be below 2^31 - 2^16");
    if (rowptr[0] != 0) throw Error(NAPSPMV_EINVAL, "rowptr[0] must be 0");
    bool mono = true;
#pragma omp parallel for reduction(&& : mono)
    for (int64_t i = 0; i < n; ++i) mono = mono && rowptr[i + 1] >= rowptr[i];
    if (!mono) throw Error(NAPSPMV_EINVAL, "rowptr must be nondecreasing");
    const int64_t nnz = rowptr[n];
    if (nnz > kInt32Max) throw Error(NAPSPMV_EUNSUPPORTED, "nnz must be below 2^31 - 2^16");
    if (nnz > 0 && (!col || !val)) throw Error(NAPSPMV_EINVAL, "col or val is NULL");
    bool inrange = true;
#pragma omp parallel for reduction(&& : inrange)
    for (int64_t k = 0; k < nnz; ++k) inrange = inrange && col[k] >= 0 && col[k] < n;
    if (!inrange) throw Error(NAPSPMV_EINVAL, "column index out of range [0, n)");
    if (row_starts) {
        if (row_starts[0] != 0 || row_starts[n_p] != n)
            throw Error(NAPSPMV_EINVAL, "row_starts must run from 0 to n");
        for (int64_t r = 0; r < n_p; ++r)
            if (row_starts[r + 1] <= row_starts[r])
                throw Error(NAPSPMV_EINVAL, "row_starts must be strictly increasing");
    }
}

}  // namespace

void level_stats(const HostPlan &hp, int64_t pps, PhaseStats out[8]) {
    for (int ph = 0; ph < 4; ++ph) {
        const Phase &P = hp.phase[ph];
        out[2 * ph] = phase_stats(P, hp.n_p, [&](size_t k) { return P.src[k] / pps == P.dst[k] / pps; });
        out[2 * ph + 1] = phase_stats(P, hp.n_p, [&](size_t k) { return P.src[k] / pps != P.dst[k] / pps; });
    }
}

void release_device_arrays(HostPlan &hp) {
    std::vector<int32_t>().swap(hp.col_on);
    std::vector<uint8_t>().swap(hp.val_on);
    std::vector<int32_t>().swap(hp.gather_idx);
}

namespace {

// Strided partition (section 5: row r on process r mod n_p) as the
// contiguous partition of the symmetrically permuted matrix P A P^T, with
// row r at position starts[r mod n_p] + r div n_p: every set of the paper
// depends only on which process owns which index, so the plan of the
// permuted matrix is the strided plan with indices renumbered.
void build_strided(HostPlan &hp, const int64_t *rowptr, const int32_t *col, const void *val,
                   int dtype, int64_t n, int64_t n_p, int64_t ppn, int mode, uint32_t variant,
                   int64_t pps) {
    std::vector<int64_t> st(n_p + 1, 0);
    for (int64_t p = 0; p < n_p; ++p) st[p + 1] = st[p] + (n - p + n_p - 1) / n_p;
    auto pos = [&](int64_t r) { return st[r % n_p] + r / n_p; };
    std::vector<int32_t> natural(n);
    for (int64_t r = 0; r < n; ++r) natural[pos(r)] = (int32_t)r;
    const int64_t vs = dtype == NAPSPMV_F64 ? 8 : dtype == NAPSPMV_F32 ? 4 : 2;
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t k = 0; k < n; ++k) rp[k + 1] = rp[k] + (rowptr[natural[k] + 1] - rowptr[natural[k]]);
    std::vector<int32_t> c2(rp[n]);
    std::vector<uint8_t> v2((size_t)(rp[n] * vs));
    const uint8_t *vb = static_cast<const uint8_t *>(val);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t r = natural[k], len = rowptr[r + 1] - rowptr[r];
        for (int64_t e = 0; e < len; ++e) c2[rp[k] + e] = (int32_t)pos(col[rowptr[r] + e]);
        if (len) std::memcpy(&v2[(size_t)(rp[k] * vs)], vb + rowptr[r] * vs, (size_t)(len * vs));
    }
    build_plan(hp, rp.data(), c2.data(), v2.data(), dtype, n, n_p, ppn, mode, st.data(), variant,
               false, pps);
    hp.strided = true;
    hp.rows_natural.swap(natural);
}

// The socket level of a NAP plan (see the file comment) and its device
// lists: the cross-socket messages of the fully local step join the send
// buffer (gathered from v like the inter-node messages), those of the
// off_node -> on_node step form the l1x buffer (copied from the received
// buffer), and every ghost whose step crosses a socket reads the cross
// buffer of its destination socket instead of v or the received buffer.
void build_sockets(HostPlan &hp, int64_t pps) {
    hp.pps = pps;
    const int64_t n = hp.n, ppn = hp.ppn, n_p = hp.n_p;
    std::vector<int64_t> l1_key, l1_pos, l2_key, l2_pos;
    socket_route(hp.phase[NAPSPMV_PHASE_L0], n, ppn, pps, hp.sock_phase + 0);
    socket_route(hp.phase[NAPSPMV_PHASE_L1], n, ppn, pps, hp.sock_phase + 4, &l1_key, &l1_pos);
    socket_route(hp.phase[NAPSPMV_PHASE_L2], n, ppn, pps, hp.sock_phase + 8, &l2_key, &l2_pos);
    const int64_t n_sock = n_p / pps;
    const int64_t E = (int64_t)hp.pack_idx.size();
    // fully local cross messages: gathered from v into the send buffer
    const Phase &x2 = hp.sock_phase[8 + 2];
    for (size_t k = 0; k < x2.src.size(); ++k)
        for (int64_t e = x2.ptr[k]; e < x2.ptr[k + 1]; ++e) {
            hp.pack_idx.push_back(x2.idx[e]);
            hp.pack_group.push_back((int32_t)(hp.n_nodes + x2.dst[k] / pps));
        }
    const int64_t E_send = (int64_t)hp.pack_idx.size();
    // the send-buffer entry holding each received index, per destination node
    std::vector<int64_t> rkey, rpos;
    {
        // bucketed by destination node, each bucket sorted in parallel
        const Phase &I = hp.phase[NAPSPMV_PHASE_INTER];
        const int64_t nn = hp.n_nodes;
        std::vector<int64_t> cnt(nn + 1, 0);
        for (size_t k = 0; k < I.src.size(); ++k) cnt[I.dst[k] / ppn + 1] += I.ptr[k + 1] - I.ptr[k];
        for (int64_t x = 0; x < nn; ++x) cnt[x + 1] += cnt[x];
        std::vector<std::pair<int64_t, int64_t>> kp(I.idx.size());
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (size_t k = 0; k < I.src.size(); ++k) {
            const int64_t node = I.dst[k] / ppn;
            for (int64_t e = I.ptr[k]; e < I.ptr[k + 1]; ++e)
                kp[fill[node]++] = {node * n + I.idx[e], e};
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t x = 0; x < nn; ++x) std::sort(kp.begin() + cnt[x], kp.begin() + cnt[x + 1]);
        rkey.resize(kp.size());
        rpos.resize(kp.size());
        for (size_t x = 0; x < kp.size(); ++x) {
            rkey[x] = kp[x].first;
            rpos[x] = kp[x].second;
        }
    }
    // off_node -> on_node cross messages: copied from the received buffer
    const Phase &x1 = hp.sock_phase[4 + 2];
    const int64_t E1 = (int64_t)x1.idx.size();
    hp.l1x_col.assign(x1.idx.begin(), x1.idx.end());
    hp.l1x_src.resize(E1);
    hp.l1x_group.resize(E1);
    bool unrouted = false;
#pragma omp parallel for schedule(dynamic, 16) reduction(|| : unrouted)
    for (int64_t k = 0; k < (int64_t)x1.src.size(); ++k)
        for (int64_t e = x1.ptr[k]; e < x1.ptr[k + 1]; ++e) {
            const int64_t key = (int64_t)(x1.src[k] / ppn) * n + x1.idx[e];
            auto it = std::lower_bound(rkey.begin(), rkey.end(), key);
            if (it == rkey.end() || *it != key) {
                unrouted = true;
                continue;
            }
            hp.l1x_src[e] = (int32_t)rpos[it - rkey.begin()];
            hp.l1x_group[e] = (int32_t)(hp.n_nodes + n_sock + x1.dst[k] / pps);
        }
    if (unrouted) throw Error(NAPSPMV_EINVAL, "socket level: missing route");
    // re-route the ghosts whose step crosses a socket
    auto rank_of_slot = [&](int64_t slot) {
        return (int64_t)(std::upper_bound(hp.ghost_ptr.begin(), hp.ghost_ptr.end(), slot) -
                         hp.ghost_ptr.begin()) - 1;
    };
    const Phase &I = hp.phase[NAPSPMV_PHASE_INTER];
    std::vector<int32_t> recv_rank(E);
    for (size_t k = 0; k < I.src.size(); ++k)
        for (int64_t e = I.ptr[k]; e < I.ptr[k + 1]; ++e) recv_rank[e] = I.dst[k];
    bool missing = false;
#pragma omp parallel for schedule(static) reduction(|| : missing)
    for (int64_t k = 0; k < (int64_t)hp.scat_src.size(); ++k) {
        const int64_t t = rank_of_slot(hp.scat_dst[k]);
        const int64_t e = hp.scat_src[k], q = recv_rank[e];
        if (q != t && q / pps != t / pps) {
            const int64_t key = (t / pps) * n + I.idx[e];
            auto it = std::lower_bound(l1_key.begin(), l1_key.end(), key);
            if (it == l1_key.end() || *it != key)
                missing = true;
            else
                hp.scat_src[k] = (int32_t)(E_send + l1_pos[it - l1_key.begin()]);
        }
    }
    if (missing) throw Error(NAPSPMV_EINVAL, "socket level: missing route");
    std::vector<int32_t> ls, ld;
    for (size_t k = 0; k < hp.l2_src.size(); ++k) {
        const int64_t t = rank_of_slot(hp.l2_dst[k]);
        const int32_t j = hp.l2_src[k];
        const int64_t own = std::upper_bound(hp.starts.begin(), hp.starts.end(), (int64_t)j) -
                            hp.starts.begin() - 1;
        if (own / pps == t / pps) {
            ls.push_back(j);
            ld.push_back(hp.l2_dst[k]);
        } else {
            hp.scat_src.push_back((int32_t)(E + lookup(l2_key, l2_pos, (t / pps) * n + j)));
            hp.scat_dst.push_back(hp.l2_dst[k]);
        }
    }
    hp.l2_src.swap(ls);
    hp.l2_dst.swap(ld);
    if (E_send + (int64_t)hp.l1x_col.size() > kInt32Max)
        throw Error(NAPSPMV_EUNSUPPORTED, "send and cross-socket buffers must stay below 2^31 - 2^16");
}

}  // namespace

void build_plan(HostPlan &hp, const int64_t *rowptr, const int32_t *col, const void *val,
                int dtype, int64_t n, int64_t n_p, int64_t ppn, int mode,
                const int64_t *row_starts, uint32_t variant, bool strided, int64_t pps) {
    validate(rowptr, col, val, dtype, n, n_p, ppn, mode, row_starts);
    if (pps != 0) {
        if (mode != NAPSPMV_NAP) throw Error(NAPSPMV_EINVAL, "the socket level needs a NAP plan");
        if (pps < 1 || ppn % pps != 0) throw Error(NAPSPMV_EINVAL, "procs_per_socket must divide ppn");
        if (variant) throw Error(NAPSPMV_EINVAL, "the socket level takes no NAP plan variant");
    }
    if (variant & ~kVariantFlags) throw Error(NAPSPMV_EINVAL, "unknown plan variant flag");
    if (variant && mode != NAPSPMV_NAP)
        throw Error(NAPSPMV_EINVAL, "plan variant flags apply to NAP plans only");
    if ((variant & NAPSPMV_NAP_DIRECT) && (variant & NAPSPMV_NAP_THREE_WAY))
        throw Error(NAPSPMV_EINVAL, "direct reads and the three-way product do not combine");
    hp.direct = (variant & NAPSPMV_NAP_DIRECT) != 0;
    if (strided) {
        if (row_starts) throw Error(NAPSPMV_EINVAL, "a strided partition takes no row_starts");
        if (variant & NAPSPMV_NAP_SPLIT)
            throw Error(NAPSPMV_EINVAL,
                        "the split variant cuts E(n, m) in index order, which a strided "
                        "partition does not keep");
        build_strided(hp, rowptr, col, val, dtype, n, n_p, ppn, mode, variant, pps);
        return;
    }
    hp.n = n;
    hp.nnz = rowptr[n];
    hp.n_p = n_p;
    hp.ppn = ppn;
    hp.n_nodes = n_p / ppn;
    hp.mode = mode;
    hp.dtype = dtype;
    hp.value_size = dtype == NAPSPMV_F64 ? 8 : dtype == NAPSPMV_F32 ? 4 : 2;

    // Row blocks R(r) (section 2): even partition, remainder on the last rank.
    hp.starts.resize(n_p + 1);
    int64_t block = 0;
    if (row_starts) {
        std::copy(row_starts, row_starts + n_p + 1, hp.starts.begin());
    } else {
        block = n / n_p;
        for (int64_t r = 0; r < n_p; ++r) hp.starts[r] = block * r;
        hp.starts[n_p] = n;
    }
    const Owner owner{hp.starts, block, n_p};
    auto node_of = [&](int64_t r) { return r / ppn; };

    // gh(t): sorted unique off-process columns of each process.
    std::vector<std::vector<int32_t>> gh(n_p);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_p; ++t) {
        const int64_t lo = hp.starts[t], hi = hp.starts[t + 1];
        std::vector<int32_t> g;
        g.reserve((size_t)(rowptr[hi] - rowptr[lo]) / 2);
        for (int64_t k = rowptr[lo]; k < rowptr[hi]; ++k)
            if (col[k] < lo || col[k] >= hi) g.push_back(col[k]);
        std::sort(g.begin(), g.end());
        g.erase(std::unique(g.begin(), g.end()), g.end());
        gh[t].swap(g);
    }
    hp.ghost_ptr.assign(n_p + 1, 0);
    for (int64_t t = 0; t < n_p; ++t) hp.ghost_ptr[t + 1] = hp.ghost_ptr[t] + (int64_t)gh[t].size();
    const int64_t G = hp.ghost_ptr[n_p];
    if (G > kInt32Max) throw Error(NAPSPMV_EUNSUPPORTED, "ghost count must be below 2^31 - 2^16");
    hp.ghost_col.resize(G);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_p; ++t)
        std::copy(gh[t].begin(), gh[t].end(), hp.ghost_col.begin() + hp.ghost_ptr[t]);

    // Split CSR: the on-process and off-process entries of every row, each in
    // stored order; off-process columns become ghost positions.
    const int64_t vs = hp.value_size;
    const uint8_t *vbytes = static_cast<const uint8_t *>(val);
    hp.rowptr_on.assign(n + 1, 0);
    hp.rowptr_off.assign(n + 1, 0);
    hp.on_lo.assign(n, 0x7fffffff);
    hp.on_hi.assign(n, -1);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_p; ++t) {
        const int64_t lo = hp.starts[t], hi = hp.starts[t + 1];
        for (int64_t i = lo; i < hi; ++i) {
            int32_t on = 0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                if (col[k] >= lo && col[k] < hi) {
                    ++on;
                    hp.on_lo[i] = std::min(hp.on_lo[i], col[k]);
                    hp.on_hi[i] = std::max(hp.on_hi[i], col[k]);
                }
            }
            hp.rowptr_on[i + 1] = on;
            hp.rowptr_off[i + 1] = (int32_t)(rowptr[i + 1] - rowptr[i]) - on;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        hp.rowptr_on[i + 1] += hp.rowptr_on[i];
        hp.rowptr_off[i + 1] += hp.rowptr_off[i];
    }
    hp.nnz_on = hp.rowptr_on[n];
    hp.nnz_off = hp.rowptr_off[n];
    hp.col_on.resize(hp.nnz_on);
    hp.col_off.resize(hp.nnz_off);
    hp.val_on.resize((size_t)(hp.nnz_on * vs));
    hp.val_off.resize((size_t)(hp.nnz_off * vs));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_p; ++t) {
        const int64_t lo = hp.starts[t], hi = hp.starts[t + 1];
        const std::vector<int32_t> &g = gh[t];
        const int64_t gbase = hp.ghost_ptr[t];
        for (int64_t i = lo; i < hi; ++i) {
            int64_t a = hp.rowptr_on[i], b = hp.rowptr_off[i];
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int32_t j = col[k];
                if (j >= lo && j < hi) {
                    hp.col_on[a] = j;
                    std::memcpy(&hp.val_on[(size_t)(a * vs)], vbytes + k * vs, (size_t)vs);
                    ++a;
                } else {
                    const int64_t pos = std::lower_bound(g.begin(), g.end(), j) - g.begin();
                    hp.col_off[b] = (int32_t)(gbase + pos);
                    std::memcpy(&hp.val_off[(size_t)(b * vs)], vbytes + k * vs, (size_t)vs);
                    ++b;
                }
            }
        }
    }

    // Three-way plans: move the on_node entries of every row (stored order
    // kept) out of the off-process block.
    if (variant & NAPSPMV_NAP_THREE_WAY) {
        hp.three_way = true;
        std::vector<uint8_t> on_node(hp.nnz_off);
        hp.rowptr_nd.assign(n + 1, 0);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t t = 0; t < n_p; ++t) {
            const int64_t nlo = hp.starts[node_of(t) * ppn], nhi = hp.starts[(node_of(t) + 1) * ppn];
            for (int64_t i = hp.starts[t]; i < hp.starts[t + 1]; ++i) {
                int32_t c = 0;
                for (int64_t b = hp.rowptr_off[i]; b < hp.rowptr_off[i + 1]; ++b) {
                    const int32_t j = hp.ghost_col[hp.col_off[b]];
                    on_node[b] = j >= nlo && j < nhi;
                    c += on_node[b];
                }
                hp.rowptr_nd[i + 1] = c;
            }
        }
        for (int64_t i = 0; i < n; ++i) hp.rowptr_nd[i + 1] += hp.rowptr_nd[i];
        hp.nnz_nd = hp.rowptr_nd[n];
        std::vector<int32_t> rp_fn(n + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            rp_fn[i + 1] = rp_fn[i] + (hp.rowptr_off[i + 1] - hp.rowptr_off[i]) -
                           (hp.rowptr_nd[i + 1] - hp.rowptr_nd[i]);
        std::vector<int32_t> col_fn(rp_fn[n]);
        std::vector<uint8_t> val_fn((size_t)(rp_fn[n] * vs));
        hp.col_nd.resize(hp.nnz_nd);
        hp.val_nd.resize((size_t)(hp.nnz_nd * vs));
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = hp.rowptr_nd[i], f = rp_fn[i];
            for (int64_t b = hp.rowptr_off[i]; b < hp.rowptr_off[i + 1]; ++b) {
                const uint8_t *src = &hp.val_off[(size_t)(b * vs)];
                if (on_node[b]) {
                    hp.col_nd[a] = hp.col_off[b];
                    std::memcpy(&hp.val_nd[(size_t)(a * vs)], src, (size_t)vs);
                    ++a;
                } else {
                    col_fn[f] = hp.col_off[b];
                    std::memcpy(&val_fn[(size_t)(f * vs)], src, (size_t)vs);
                    ++f;
                }
            }
        }
        hp.rowptr_off.swap(rp_fn);
        hp.col_off.swap(col_fn);
        hp.val_off.swap(val_fn);
    }

    // Runs of gh(t) by owner: the standard messages D(r, t).
    std::vector<std::vector<MsgRef>> runs(n_p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_p; ++t) {
        const std::vector<int32_t> &g = gh[t];
        const int32_t *base = hp.ghost_col.data() + hp.ghost_ptr[t];
        size_t a = 0;
        while (a < g.size()) {
            const int64_t r = owner(g[a]);
            size_t b = a + 1;
            while (b < g.size() && g[b] < hp.starts[r + 1]) ++b;
            runs[t].push_back(MsgRef{(int32_t)r, (int32_t)t, base + a, (int64_t)(b - a)});
            a = b;
        }
    }
    {
        std::vector<MsgRef> inter, intra;
        for (int64_t t = 0; t < n_p; ++t)
            for (const MsgRef &m : runs[t]) {
                if (node_of(m.src) == node_of(m.dst))
                    intra.push_back(m);
                else if (mode == NAPSPMV_STANDARD)
                    inter.push_back(m);
            }
        if (mode == NAPSPMV_STANDARD) finalize_phase(inter, hp.phase[NAPSPMV_PHASE_INTER]);
        finalize_phase(intra, hp.phase[NAPSPMV_PHASE_L2]);
    }
    std::vector<std::vector<MsgRef>>().swap(runs);

    if (mode == NAPSPMV_STANDARD) {
        hp.gather_idx = hp.ghost_col;   // the ghost buffer is every receive buffer in order
    } else {
        const int64_t nn = hp.n_nodes;
        // E(., m) for every destination node m: sorted unique off-node ghosts.
        std::vector<std::vector<int32_t>> Em(nn);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t m = 0; m < nn; ++m) {
            std::vector<int32_t> e;
            for (int64_t t = m * ppn; t < (m + 1) * ppn; ++t)
                for (int32_t j : gh[t])
                    if (node_of(owner(j)) != m) e.push_back(j);
            std::sort(e.begin(), e.end());
            e.erase(std::unique(e.begin(), e.end()), e.end());
            Em[m].swap(e);
        }
        // Node pairs (n -> m) with |E(n, m)|, grouped by destination m, n ascending.
        struct Pair {
            int32_t n, m;
            int64_t start, len;        // range in Em[m]
            int64_t kT = 0, kU = 0;    // rank among n's partners / among m's senders
            int32_t send_local = 0, recv_local = 0;
            int64_t piece_begin = 0, piece_end = 0;
        };
        // One inter-node message: a contiguous piece of E(n, m) (the whole set
        // unless the split variant cuts it).
        struct Piece {
            int32_t send_rank, recv_rank;
            int64_t start, len;        // range in Em[m]
            int64_t send_off = 0;      // offset in the send buffer
        };
        std::vector<Pair> pairs;
        std::vector<int64_t> pairs_of_m(nn + 1, 0);
        for (int64_t m = 0; m < nn; ++m) {
            const std::vector<int32_t> &e = Em[m];
            size_t a = 0;
            while (a < e.size()) {
                const int64_t src_node = node_of(owner(e[a]));
                const int64_t end_row = hp.starts[(src_node + 1) * ppn];
                size_t b = a + 1;
                while (b < e.size() && e[b] < end_row) ++b;
                Pair p;
                p.n = (int32_t)src_node;
                p.m = (int32_t)m;
                p.start = (int64_t)a;
                p.len = (int64_t)(b - a);
                pairs.push_back(p);
                a = b;
            }
            pairs_of_m[m + 1] = (int64_t)pairs.size();
        }
        const int64_t np_ = (int64_t)pairs.size();
        std::vector<int64_t> partners(nn, 0);    // |N(n)|
        for (const Pair &p : pairs) ++partners[p.n];
        // |E(a, b)| lookup through pairs sorted by (n, m).
        std::vector<int64_t> by_src(np_);
        std::iota(by_src.begin(), by_src.end(), 0);
        std::sort(by_src.begin(), by_src.end(), [&](int64_t x, int64_t y) {
            return pairs[x].n != pairs[y].n ? pairs[x].n < pairs[y].n : pairs[x].m < pairs[y].m;
        });
        auto vol = [&](int64_t a, int64_t b) -> int64_t {
            auto it = std::lower_bound(by_src.begin(), by_src.end(), 0, [&](int64_t x, int) {
                return pairs[x].n != a ? pairs[x].n < a : pairs[x].m < b;
            });
            if (it != by_src.end() && pairs[*it].n == a && pairs[*it].m == b) return pairs[*it].len;
            return 0;
        };
        // T: partners of n by (|E(n, m)| desc, m asc) -> local k mod ppn.
        std::vector<int64_t> ord(by_src);
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
            const Pair &a = pairs[x], &b = pairs[y];
            if (a.n != b.n) return a.n < b.n;
            if (a.len != b.len) return a.len > b.len;
            return a.m < b.m;
        });
        for (int64_t k = 0, run = 0; k < np_; ++k) {
            run = (k > 0 && pairs[ord[k]].n == pairs[ord[k - 1]].n) ? run + 1 : 0;
            Pair &p = pairs[ord[k]];
            p.kT = run;
            p.send_local = (int32_t)(run % ppn);
        }
        if (variant & NAPSPMV_NAP_OWNER_MAP) {
            // The local process of n owning the most of E(n, m), lowest on ties.
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t x = 0; x < np_; ++x) {
                Pair &p = pairs[x];
                std::vector<int64_t> held(ppn, 0);
                const int32_t *e = Em[p.m].data() + p.start;
                for (int64_t a = 0; a < p.len; ++a) ++held[owner(e[a]) - (int64_t)p.n * ppn];
                p.send_local = (int32_t)(std::max_element(held.begin(), held.end()) - held.begin());
            }
        }
        // U: senders of m by (|E(m, n)| desc, n asc) -> local ppn-1-(k mod ppn).
        std::vector<int64_t> back(np_);
        for (int64_t x = 0; x < np_; ++x) back[x] = vol(pairs[x].m, pairs[x].n);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
            const Pair &a = pairs[x], &b = pairs[y];
            if (a.m != b.m) return a.m < b.m;
            if (back[x] != back[y]) return back[x] > back[y];
            return a.n < b.n;
        });
        for (int64_t k = 0, run = 0; k < np_; ++k) {
            run = (k > 0 && pairs[ord[k]].m == pairs[ord[k - 1]].m) ? run + 1 : 0;
            Pair &p = pairs[ord[k]];
            p.kU = run;
            p.recv_local = (int32_t)(ppn - 1 - run % ppn);
        }
        // Pieces.  Under the split variant a node with k < ppn partners sends
        // the i-th through locals i, i + k, ... < ppn, E cut into that many
        // near-equal contiguous pieces; a node with k' < ppn senders receives
        // the i'-th through locals ppn-1-i', ppn-1-i'-k', ..., piece c going to
        // the (c mod count)-th of them.
        const bool split = (variant & NAPSPMV_NAP_SPLIT) != 0;
        std::vector<Piece> pieces;
        pieces.reserve((size_t)np_);
        for (int64_t x = 0; x < np_; ++x) {
            Pair &p = pairs[x];
            const int64_t k_snd = partners[p.n];
            const int64_t k_rcv = pairs_of_m[p.m + 1] - pairs_of_m[p.m];
            const bool s_split = split && k_snd < ppn, r_split = split && k_rcv < ppn;
            const int64_t cs = s_split ? (ppn - p.kT + k_snd - 1) / k_snd : 1;
            const int64_t cr = r_split ? (ppn - p.kU + k_rcv - 1) / k_rcv : 1;
            p.piece_begin = (int64_t)pieces.size();
            for (int64_t c = 0; c < cs; ++c) {
                const int64_t a = c * p.len / cs, b = (c + 1) * p.len / cs;
                if (b == a) continue;
                const int64_t sl = s_split ? p.kT + c * k_snd : p.send_local;
                const int64_t rl = r_split ? ppn - 1 - p.kU - (c % cr) * k_rcv : p.recv_local;
                Piece q;
                q.send_rank = (int32_t)(p.n * ppn + sl);
                q.recv_rank = (int32_t)(p.m * ppn + rl);
                q.start = p.start + a;
                q.len = b - a;
                pieces.push_back(q);
            }
            p.piece_end = (int64_t)pieces.size();
        }
        const int64_t npc = (int64_t)pieces.size();
        // INTER messages in canonical order define the send buffer layout.
        std::vector<int64_t> pair_of_piece(npc);
        for (int64_t x = 0; x < np_; ++x)
            for (int64_t c = pairs[x].piece_begin; c < pairs[x].piece_end; ++c) pair_of_piece[c] = x;
        std::vector<int64_t> canon(npc);
        std::iota(canon.begin(), canon.end(), 0);
        std::sort(canon.begin(), canon.end(), [&](int64_t x, int64_t y) {
            const Piece &a = pieces[x], &b = pieces[y];
            return a.send_rank != b.send_rank ? a.send_rank < b.send_rank
                                              : a.recv_rank < b.recv_rank;
        });
        {
            std::vector<MsgRef> refs(npc);
            int64_t off = 0;
            for (int64_t k = 0; k < npc; ++k) {
                Piece &q = pieces[canon[k]];
                q.send_off = off;
                off += q.len;
                refs[k] = MsgRef{q.send_rank, q.recv_rank,
                                 Em[pairs[pair_of_piece[canon[k]]].m].data() + q.start, q.len};
            }
            finalize_phase(refs, hp.phase[NAPSPMV_PHASE_INTER]);
            hp.pack_idx = hp.phase[NAPSPMV_PHASE_INTER].idx;
        }
        // L0: per inter-node sender s, the indices it sends but does not own.
        std::vector<std::vector<int32_t>> l0(n_p);
        {
            std::vector<std::vector<int64_t>> pieces_of_s(n_p);
            for (int64_t c = 0; c < npc; ++c) pieces_of_s[pieces[c].send_rank].push_back(c);
            std::vector<std::vector<MsgRef>> l0runs(n_p);
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t s = 0; s < n_p; ++s) {
                std::vector<int32_t> &d = l0[s];
                for (int64_t c : pieces_of_s[s]) {
                    const Piece &q = pieces[c];
                    const int32_t *e = Em[pairs[pair_of_piece[c]].m].data();
                    for (int64_t a = q.start; a < q.start + q.len; ++a) {
                        const int32_t j = e[a];
                        if (j < hp.starts[s] || j >= hp.starts[s + 1]) d.push_back(j);
                    }
                }
                std::sort(d.begin(), d.end());
                d.erase(std::unique(d.begin(), d.end()), d.end());
                size_t a = 0;
                while (a < d.size()) {
                    const int64_t r = owner(d[a]);
                    size_t b = a + 1;
                    while (b < d.size() && d[b] < hp.starts[r + 1]) ++b;
                    l0runs[s].push_back(MsgRef{(int32_t)r, (int32_t)s, d.data() + a, (int64_t)(b - a)});
                    a = b;
                }
            }
            std::vector<MsgRef> refs;
            for (int64_t s = 0; s < n_p; ++s) refs.insert(refs.end(), l0runs[s].begin(), l0runs[s].end());
            finalize_phase(refs, hp.phase[NAPSPMV_PHASE_L0]);
        }
        // Per destination t: scatter entries (off-node ghosts), fully local
        // gathers (on-node ghosts) and the L1 forwards.
        {
            std::vector<std::vector<int32_t>> ssrc(n_p), sdst(n_p), lsrc(n_p), ldst(n_p);
            std::vector<std::vector<int32_t>> l1j(n_p);
            std::vector<std::vector<MsgRef>> l1runs(n_p);
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t t = 0; t < n_p; ++t) {
                const int64_t m = node_of(t);
                const std::vector<int32_t> &g = gh[t];
                std::vector<std::pair<int32_t, int32_t>> fwd;   // (q, j)
                for (size_t pos = 0; pos < g.size(); ++pos) {
                    const int32_t j = g[pos];
                    const int64_t n_src = node_of(owner(j));
                    const int32_t slot = (int32_t)(hp.ghost_ptr[t] + (int64_t)pos);
                    if (n_src == m) {
                        lsrc[t].push_back(j);
                        ldst[t].push_back(slot);
                        continue;
                    }
                    // the pair (n_src -> m) among the pairs of m (n ascending)
                    auto lo = pairs.begin() + pairs_of_m[m], hi = pairs.begin() + pairs_of_m[m + 1];
                    auto it = std::lower_bound(lo, hi, n_src,
                                               [](const Pair &p, int64_t v) { return p.n < v; });
                    const Pair &p = *it;
                    const int32_t *e = Em[m].data();
                    const int64_t at = std::lower_bound(e + p.start, e + p.start + p.len, j) - e;
                    // the piece holding position `at` (pieces of a pair ascend)
                    auto pb = pieces.begin() + p.piece_begin, pe = pieces.begin() + p.piece_end;
                    const Piece &q = *(std::upper_bound(pb, pe, at, [](int64_t v, const Piece &c) {
                                           return v < c.start;
                                       }) - 1);
                    ssrc[t].push_back((int32_t)(q.send_off + (at - q.start)));
                    sdst[t].push_back(slot);
                    if (q.recv_rank != t) fwd.emplace_back(q.recv_rank, j);
                }
                std::stable_sort(fwd.begin(), fwd.end(),
                                 [](const std::pair<int32_t, int32_t> &a,
                                    const std::pair<int32_t, int32_t> &b) { return a.first < b.first; });
                l1j[t].resize(fwd.size());
                for (size_t k = 0; k < fwd.size(); ++k) l1j[t][k] = fwd[k].second;
                size_t a = 0;
                while (a < fwd.size()) {
                    size_t b = a + 1;
                    while (b < fwd.size() && fwd[b].first == fwd[a].first) ++b;
                    l1runs[t].push_back(MsgRef{fwd[a].first, (int32_t)t, l1j[t].data() + a, (int64_t)(b - a)});
                    a = b;
                }
            }
            std::vector<MsgRef> refs;
            for (int64_t t = 0; t < n_p; ++t) refs.insert(refs.end(), l1runs[t].begin(), l1runs[t].end());
            finalize_phase(refs, hp.phase[NAPSPMV_PHASE_L1]);
            auto flatten = [&](std::vector<std::vector<int32_t>> &parts, std::vector<int32_t> &out) {
                std::vector<int64_t> off(n_p + 1, 0);
                for (int64_t t = 0; t < n_p; ++t) off[t + 1] = off[t] + (int64_t)parts[t].size();
                out.resize(off[n_p]);
#pragma omp parallel for schedule(dynamic, 16)
                for (int64_t t = 0; t < n_p; ++t) {
                    std::copy(parts[t].begin(), parts[t].end(), out.begin() + off[t]);
                    std::vector<int32_t>().swap(parts[t]);
                }
            };
            flatten(ssrc, hp.scat_src);
            flatten(sdst, hp.scat_dst);
            flatten(lsrc, hp.l2_src);
            flatten(ldst, hp.l2_dst);
        }
        if (variant & NAPSPMV_NAP_DEDUP) {
            // The fully local step drops what the on_node -> off_node step
            // already carries between the same two processes (l0[t] holds the
            // indices t receives there).  The device still fills those ghost
            // slots from v: on one device both copies are the same read.
            std::vector<std::vector<int32_t>> keep(n_p);
            std::vector<std::vector<MsgRef>> runs2(n_p);
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t t = 0; t < n_p; ++t) {
                const std::vector<int32_t> &d = l0[t];
                for (int32_t j : gh[t])
                    if (node_of(owner(j)) == node_of(t) && !std::binary_search(d.begin(), d.end(), j))
                        keep[t].push_back(j);
                const std::vector<int32_t> &g = keep[t];
                size_t a = 0;
                while (a < g.size()) {
                    const int64_t r = owner(g[a]);
                    size_t b = a + 1;
                    while (b < g.size() && g[b] < hp.starts[r + 1]) ++b;
                    runs2[t].push_back(MsgRef{(int32_t)r, (int32_t)t, g.data() + a, (int64_t)(b - a)});
                    a = b;
                }
            }
            std::vector<MsgRef> refs;
            for (int64_t t = 0; t < n_p; ++t) refs.insert(refs.end(), runs2[t].begin(), runs2[t].end());
            hp.phase[NAPSPMV_PHASE_L2] = Phase();
            finalize_phase(refs, hp.phase[NAPSPMV_PHASE_L2]);
        }
        // send-buffer groups: the destination node of every inter-node entry
        const Phase &I = hp.phase[NAPSPMV_PHASE_INTER];
        hp.pack_group.resize(hp.pack_idx.size());
        for (size_t k = 0; k < I.src.size(); ++k)
            for (int64_t e = I.ptr[k]; e < I.ptr[k + 1]; ++e)
                hp.pack_group[e] = (int32_t)(I.dst[k] / ppn);
        if (pps > 0) build_sockets(hp, pps);
    }
    for (int ph = 0; ph < 4; ++ph) hp.stats[ph] = phase_stats(hp.phase[ph], n_p);
    for (int ph = 0; ph < 12; ++ph) hp.sock_stats[ph] = phase_stats(hp.sock_phase[ph], n_p);
}

}  // namespace napspmv
