// gfx950 kernels of the apply path: the exchanges that carry the plan's
// messages, and the split CSR product.
//
// An apply is two product launches, as algorithm standard_spmv (section 2.1)
// and NAPSpMV (section 4.3) order the work: the first launch runs the
// exchange that fills the ghost buffer (or the NAP send buffer and, when it
// is received in place, band by band the NAP scatter into the ghost buffer)
// together with the on-process product local_spmv(A_on, v), which needs no
// received value; the second adds the off-process product
// local_spmv(A_off, ghost) into w (for NAP with the explicit hop, after the
// hop and the scatter of received values).  The first launch interleaves
// its two kinds of blocks on every CU, the overlap of local work with
// communication that the paper's algorithms make.
//
// Every kernel is HBM-bound (the product does 2 flops per 12-16 bytes), so
// the design is about bytes and latency, not arithmetic: 256-thread blocks of
// four wave64s; matrix streams (values, columns) read once with non-temporal
// loads so they do not evict the vector and the ghost buffer from L2;
// exchange buffers laid out by column band so every exchange writes in order
// from a slice of v staged in LDS; all loads of a block issued at once; and
// an XCD-aware block order, so that each of the eight L2 caches sees one
// contiguous range of the work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schedule.hpp"

namespace napspmv {

constexpr int kBlock = 256;

// Hardware hands workgroup b to XCD b mod 8.  Remap so that XCD x runs the
// logical blocks [x*q + min(x, r), ...) of a grid of nb = 8q + r blocks: a
// bijection on [0, nb) that gives each XCD one contiguous range.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    const uint32_t x = b & 7u, k = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + k;
}

// Widening streaming loads of a stored value of A into the accumulation type.
__device__ __forceinline__ double load_val(const double *p, int32_t k) {
    return __builtin_nontemporal_load(p + k);
}
__device__ __forceinline__ float load_val(const float *p, int32_t k) {
    return __builtin_nontemporal_load(p + k);
}
__device__ __forceinline__ float load_val(const uint16_t *p, int32_t k) {
    const uint16_t b = __builtin_nontemporal_load(p + k);
    return __uint_as_float((uint32_t)b << 16);   // bfloat16 -> float32 is exact
}

// dst[dpos[k]] = src[sidx[k]] for k < n: a short indexed copy (the fully
// local step of a three-way apply).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_put(int32_t n, const int32_t *__restrict__ dpos,
                                                const int32_t *__restrict__ sidx,
                                                const T *__restrict__ src, T *__restrict__ dst) {
    const uint32_t k = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (k < (uint32_t)n) dst[__builtin_nontemporal_load(dpos + k)] = src[__builtin_nontemporal_load(sidx + k)];
}

// dst[k] = src[k]: the explicit inter-node hop (send buffer -> receive buffer).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int32_t n, const T *__restrict__ src,
                                                 T *__restrict__ dst) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k < (uint32_t)n) dst[k] = src[k];
}

// Exchange buffers (the ghost buffer, the NAP send buffer) are laid out band
// by band: band b holds, in order, the entries whose source column of v lies
// in [b*CAP, (b+1)*CAP), grouped by message (each process's ghosts, or each
// inter-node message) in ascending column.  A band item (x = b >= 0, entries
// [y, y+z)) stages that slice of the source vector in LDS with coalesced
// loads and then writes its entries in order: dst[k] = lds[off[k]], a
// streaming write fed by LDS reads, instead of one scattered L2 read per
// entry.  An indexed item (x = -1) is the plain form, dst[dpos[k]] =
// src[idx[k]] over entries [y, y+z), used by the per-process launches.
template <typename T, int CAP>
__device__ __forceinline__ void stage_band(int32_t band, int32_t n, const T *__restrict__ src,
                                           T *lds) {
    const int64_t c0 = (int64_t)band * CAP;
#pragma unroll
    for (int u = 0; u < CAP / kBlock; ++u) {
        const int64_t c = c0 + u * kBlock + threadIdx.x;
        if (c < n) lds[u * kBlock + threadIdx.x] = src[c];
    }
    __syncthreads();
}

// NT: a non-temporal store (past the caches).  A compile-time choice: with a
// run-time one the compiler merges the two stores and keeps neither hint.
template <bool NT, typename T>
__device__ __forceinline__ void store_out(T x, T *p) {
    if constexpr (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

// E consecutive entries of an E-aligned run of an array, as one vector.
template <typename T, int E>
using Vec = T __attribute__((ext_vector_type(E)));

template <int E, typename T>
__device__ __forceinline__ Vec<T, E> load_vec(const T *p, int32_t k) {
    return __builtin_nontemporal_load(reinterpret_cast<const Vec<T, E> *>(p + k));
}

// dst[k] = lds[off[k]] for k in [begin, end), by aligned runs of E = 16 bytes
// of values: each lane loads E offsets at once and stores E values with one
// 16-byte store, so a wave moves several entries' bytes per instruction and
// every store instruction writes whole lines; the few entries before the
// first and after the last aligned run go one per lane.
template <typename T, bool NT>
__device__ __forceinline__ void band_copy(int32_t begin, int32_t end,
                                          const uint16_t *__restrict__ off, T *__restrict__ dst,
                                          const T *lds) {
    constexpr int E = 16 / sizeof(T);
    const int32_t tid = (int32_t)threadIdx.x;
    const int32_t a = min((begin + E - 1) & -E, end), b = max(end & -E, a);
    if (begin + tid < a) store_out<NT>(lds[off[begin + tid]], dst + begin + tid);
    if (b + tid < end) store_out<NT>(lds[off[b + tid]], dst + b + tid);
    int32_t q = a + E * tid;
    for (; q + 3 * E * kBlock < b; q += 4 * E * kBlock) {
        Vec<uint16_t, E> o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = load_vec<E>(off, q + E * u * kBlock);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Vec<T, E> x;
#pragma unroll
            for (int j = 0; j < E; ++j) x[j] = lds[o[u][j]];
            store_out<NT>(x, reinterpret_cast<Vec<T, E> *>(dst + q + E * u * kBlock));
        }
    }
    for (; q < b; q += E * kBlock) {
        const Vec<uint16_t, E> o = load_vec<E>(off, q);
        Vec<T, E> x;
#pragma unroll
        for (int j = 0; j < E; ++j) x[j] = lds[o[j]];
        store_out<NT>(x, reinterpret_cast<Vec<T, E> *>(dst + q));
    }
}

template <typename T, int CAP>
__device__ __forceinline__ void exchange_item(int4 it, int32_t n, const uint16_t *__restrict__ off,
                                              const int32_t *__restrict__ idx,
                                              const int32_t *__restrict__ dpos,
                                              const T *__restrict__ src, T *__restrict__ dst,
                                              T *lds, bool nt) {
    const int32_t end = it.y + it.z;
    if (it.x >= 0) {
        stage_band<T, CAP>(it.x, n, src, lds);
        if (nt)
            band_copy<T, true>(it.y, end, off, dst, lds);
        else
            band_copy<T, false>(it.y, end, off, dst, lds);
        return;
    }
    int32_t k = it.y + (int32_t)threadIdx.x;
    for (; k + 3 * kBlock < end; k += 4 * kBlock) {
        int32_t j[4], d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            j[u] = __builtin_nontemporal_load(idx + k + u * kBlock);
            d[u] = __builtin_nontemporal_load(dpos + k + u * kBlock);
        }
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = src[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[d[u]] = x[u];
    }
    for (; k < end; k += kBlock)
        dst[__builtin_nontemporal_load(dpos + k)] = src[__builtin_nontemporal_load(idx + k)];
}

// NAP scatter of one band of the ghost buffer (band-ordered like the
// exchange buffers): each ghost position's code says where its value comes
// from: bit 31 set, the fully local step, column offset code & 0x7fffffff
// inside the band of v (staged in LDS); clear, the received inter-node
// buffer at position code.  `which` = 0 fills every position, 1 only
// received values, 2 only fully local values.
constexpr uint32_t kFromV = 0x80000000u;

template <typename T, bool NT>
__device__ __forceinline__ void scatter_values(int4 it, int32_t which,
                                               const uint32_t *__restrict__ code,
                                               const T *recv, T *__restrict__ ghost,
                                               const T *lds) {
    const int32_t end = it.y + it.z;
    int32_t k = it.y + (int32_t)threadIdx.x;
    for (; k + 3 * kBlock < end; k += 4 * kBlock) {
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = __builtin_nontemporal_load(code + k + u * kBlock);
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool fv = (c[u] & kFromV) != 0;
            if (fv ? which != 1 : which != 2) x[u] = fv ? lds[c[u] & ~kFromV] : recv[c[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool fv = (c[u] & kFromV) != 0;
            if (fv ? which != 1 : which != 2) store_out<NT>(x[u], ghost + k + u * kBlock);
        }
    }
    for (; k < end; k += kBlock) {
        const uint32_t c = __builtin_nontemporal_load(code + k);
        const bool fv = (c & kFromV) != 0;
        if (fv ? which != 1 : which != 2) store_out<NT>(fv ? lds[c & ~kFromV] : recv[c], ghost + k);
    }
}

template <typename T, int CAP>
__device__ __forceinline__ void scatter_item(int4 it, int32_t n, int32_t which,
                                             const uint32_t *__restrict__ code,
                                             const T *__restrict__ v, const T *__restrict__ recv,
                                             T *__restrict__ ghost, T *lds) {
    if (which != 1) stage_band<T, CAP>(it.x, n, v, lds);
    scatter_values<T, false>(it, which, code, recv, ghost, lds);
}

// NAP pack and scatter of one column band b in one item, when the exchange
// is received in place: every received value a ghost of band b takes was
// packed from band b of v (the ghost's own column), so once this item has
// packed band b's part of the send buffer, the same workgroup can scatter
// band b of the ghost buffer from it (the off_node -> on_node step and the
// receiver's own use), and the fully local positions from the band of v
// still in LDS.  The pack uses plain stores: its values are read back at
// once, from this CU's cache.  item = (b, first send entry, count, 1).
// A plan with a socket level also copies, between the two, the received
// values of band b that cross a socket in the off_node -> on_node step into
// their cross-socket buffer (s1band: its band boundaries, as positions of
// the received region; s1src: the received position of each entry), which
// the scatter then reads like the received buffer.
template <typename T, int CAP>
__device__ __forceinline__ void pack_scatter_item(int4 it, int32_t n, const uint16_t *__restrict__ off,
                                                  const T *__restrict__ v, T *send,
                                                  const int32_t *__restrict__ gband,
                                                  const int32_t *__restrict__ s1band,
                                                  const int32_t *__restrict__ s1src,
                                                  const uint32_t *__restrict__ code,
                                                  const T *recv, T *__restrict__ ghost, T *lds,
                                                  bool nt) {
    stage_band<T, CAP>(it.x, n, v, lds);
    band_copy<T, false>(it.y, it.y + it.z, off, send, lds);
    // the band's packed values are visible to the whole workgroup (recv and
    // send are the same memory: no restrict on either)
    __syncthreads();
    if (s1band) {
        const int32_t b0 = s1band[it.x], b1 = s1band[it.x + 1];
        if (b1 > b0) {
            const int32_t e = s1band[0];     // first position of the cross-socket buffer
            for (int32_t k = b0 + (int32_t)threadIdx.x; k < b1; k += kBlock)
                send[k] = recv[__builtin_nontemporal_load(s1src + (k - e))];
            __syncthreads();
        }
    }
    const int4 sit = make_int4(it.x, gband[it.x], gband[it.x + 1] - gband[it.x], 1);
    if (nt)
        scatter_values<T, true>(sit, 0, code, recv, ghost, lds);
    else
        scatter_values<T, false>(sit, 0, code, recv, ghost, lds);
}

// acc + p[q0] + p[q0 + 1] + ... + p[q1 - 1], added one at a time in that
// order (the rounding of the sequential sum), with the LDS reads issued
// eight (then four) at a time so that their latencies overlap instead of
// adding up.
template <typename XT>
__device__ __forceinline__ XT sum_in_order(XT acc, const XT *p, int32_t q0, int32_t q1) {
    int32_t q = q0;
    for (; q + 8 <= q1; q += 8) {
        XT t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) t[i] = p[q + i];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = acc + t[i];
    }
    if (q + 4 <= q1) {
        XT t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) t[i] = p[q + i];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc = acc + t[i];
        q += 4;
    }
    for (; q < q1; ++q) acc = acc + p[q];
    return acc;
}

// Row blocks of a split CSR product.  A block owns rows [r0, r1) and
// entries [k0, k1) of one of the two CSR parts, at most CAP of them (else a
// single long row).  Every thread first issues all its loads at once, by
// aligned runs of E entries (product_runs, remote_product_runs): its share
// of the entries, of the block's v window, of the row pointers and, for the
// off-process part, of the partial sums.  Then it gathers the vector
// operands, forms the products a * x into LDS, and one thread per row adds
// its products in stored order to the row's running sum: 0 for the
// on-process part (REMOTE = false), the partial w[r] of the first launch for
// the off-process part (REMOTE = true; rows without off-process entries are
// not touched).  Each row is therefore the sequential sum, product by
// product, of its on-process entries then its off-process entries in stored
// order.
//
// x comes from `xsrc` (v for the on-process part, the ghost buffer for the
// off-process part), or, for on-process columns inside the block's window
// win = (first, length) of v, from a copy of that window staged in LDS.
//
// Columns come as CT (int32, or uint16 offsets from `cbase`: the first row
// of the block's process for on-process columns when every process holds at
// most 65536 rows, the block's first ghost position for a narrow
// off-process block).
//
// Rows per block: on-process blocks hold at most kMaxRowsOn rows (two row
// slots per thread: fewer registers, more blocks in flight), off-process
// blocks, which cover a few rows' worth of entries each, kMaxRows.
constexpr int kMaxRows = 1024;
constexpr int kMaxRowsOn = 512;

// A block that is a single row whose entries' aligned span is longer than
// CAP (the schedules cut every block of several rows shorter), in stored
// order: walked in chunks of CAP products, each chunk's products added by
// one thread in order.
template <typename VT, typename XT, typename CT, int CAP, bool REMOTE, bool DIRECT, bool NTW>
__device__ __forceinline__ void row_in_chunks(int32_t r0, int32_t k0, int32_t k1,
                                              const CT *__restrict__ col, int32_t cbase,
                                              const VT *__restrict__ val,
                                              const XT *__restrict__ xsrc, XT *__restrict__ w,
                                              XT *prod, const XT *__restrict__ vsrc) {
    const int tid = threadIdx.x;
    XT s = REMOTE ? w[r0] : (XT)0;
    for (int32_t base = k0; base < k1; base += CAP) {
        const int32_t lim = (k1 - base) < CAP ? (k1 - base) : CAP;
        for (int32_t q = tid; q < lim; q += kBlock) {
            const int32_t k = base + q;
            const int32_t c = cbase + (int32_t)__builtin_nontemporal_load(col + k);
            prod[q] = (XT)load_val(val, k) *
                      (DIRECT ? (c < 0 ? vsrc : xsrc)[c & 0x7fffffff] : xsrc[c]);
        }
        __syncthreads();
        if (tid == 0) s = sum_in_order(s, prod, 0, lim);
        __syncthreads();
    }
    if (tid == 0) store_out<NTW>(s, w + r0);
}

// A block without entries (rows whose part is empty, e.g. the zero block of
// a saddle-point matrix) loads nothing.  The on-process part still writes
// its rows' zero sums; the off-process part leaves them as they are.
template <typename XT, bool REMOTE, bool NTW>
__device__ __forceinline__ void empty_block(int32_t r0, int32_t r1, XT *__restrict__ w) {
    if (!REMOTE)
        for (int32_t r = r0 + (int32_t)threadIdx.x; r < r1; r += kBlock) store_out<NTW>((XT)0, w + r);
}

// A stored value of A widened into the accumulation type.
__device__ __forceinline__ double widen(double a) { return a; }
__device__ __forceinline__ float widen(float a) { return a; }
__device__ __forceinline__ float widen(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Entries per lane of the on-process product: runs of 16 bytes of values
// (more for bfloat16, whose columns and values are both 2 bytes).
template <typename VT, int CAP>
constexpr int product_run() {
    constexpr int e = sizeof(VT) == 8 ? 2 : (sizeof(VT) == 4 ? 4 : 8);
    return e * kBlock <= CAP ? e : CAP / kBlock;
}

// Row block in stored order with E consecutive entries per lane (the
// on-process product; with REMOTE, an off-process block the host keeps in
// stored order, adding into the partial w): each lane loads the columns and
// values of its entries as aligned runs (one vector load each), so a wave
// moves E times the bytes per load instruction of one entry per lane, and
// writes its E products to LDS with one vector store.  The
// runs cover [k0 & -E, k1); LDS position q holds the product of entry
// (k0 & -E) + q.  Entries of the runs outside [k0, k1) (a neighbouring
// block's, or the arrays' zero padding past the last entry) are loaded and
// discarded, and their columns are not used to read x.  Each row adds its
// products in stored order.  A block whose aligned span is longer than CAP
// (a single row) goes to row_in_chunks.
template <typename VT, typename XT, typename CT, int CAP, int W, bool NTW, int E,
          bool REMOTE = false, int ROWS = kMaxRows>
__device__ __forceinline__ void product_runs(int32_t r0, int32_t r1, int32_t k0, int32_t k1,
                                             int2 win, const int32_t *__restrict__ rowptr,
                                             const CT *__restrict__ col, int32_t cbase,
                                             const VT *__restrict__ val,
                                             const XT *__restrict__ xsrc, XT *__restrict__ w,
                                             XT *prod, XT *wbuf) {
    static_assert(!REMOTE || W == 0, "off-process blocks stage no window");
    static_assert(E > 1 && CAP % (E * kBlock) == 0, "runs must tile the block");
    const int32_t k0a = k0 & -E;
    if (k1 == k0) {
        empty_block<XT, REMOTE, NTW>(r0, r1, w);
        return;
    }
    if (k1 - k0a > CAP) {
        row_in_chunks<VT, XT, CT, CAP, REMOTE, false, NTW>(r0, k0, k1, col, cbase, val, xsrc, w,
                                                           prod, nullptr);
        return;
    }
    constexpr int Q = CAP / (E * kBlock);
    constexpr int R = ROWS / kBlock;
    const int32_t tid = (int32_t)threadIdx.x;
    // Every load below is unconditional (a load under a per-lane condition
    // makes the compiler wait for the loads before it), on runs clamped to
    // the block's last one, so all of them can be in flight at once.
    const int32_t klast = (k1 - 1) & -E;
    int32_t c[E * Q];
    XT a[E * Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) {
        const int32_t e = min(k0a + E * (u * kBlock + tid), klast);
        const Vec<CT, E> cq = load_vec<E>(col, e);
        const Vec<VT, E> aq = load_vec<E>(val, e);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            c[E * u + j] = cbase + (int32_t)cq[j];
            a[E * u + j] = widen(aq[j]);
        }
    }
    XT t[W > 0 ? W / kBlock : 1];
    if (W > 0) {
        const int32_t qlast = win.y > 0 ? win.y - 1 : 0;
#pragma unroll
        for (int u = 0; u < W / kBlock; ++u) t[u] = xsrc[win.x + min(u * kBlock + tid, qlast)];
    }
    int32_t rb[R], re[R];
    XT s[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t r = min(r0 + i * kBlock + tid, r1 - 1);
        rb[i] = rowptr[r];
        re[i] = rowptr[r + 1];
        s[i] = REMOTE ? w[r] : (XT)0;
    }
    XT x[E * Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int32_t e = k0a + E * (u * kBlock + tid) + j;
            // a column outside the block may be another process's offset:
            // read the block's own base column instead (a column of v, or a
            // ghost position of this block)
            if (e < k0 || e >= k1) c[E * u + j] = cbase;
            const int32_t cc = c[E * u + j];
            const bool inwin = W > 0 && (uint32_t)(cc - win.x) < (uint32_t)win.y;
            x[E * u + j] = xsrc[inwin ? win.x : cc];
        }
    }
    if (W > 0) {
#pragma unroll
        for (int u = 0; u < W / kBlock; ++u) {
            const int32_t q = u * kBlock + tid;
            if (q < win.y) wbuf[q] = t[u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < Q; ++u) {
        const int32_t e0 = k0a + E * (u * kBlock + tid);
        if (e0 < k1) {
            Vec<XT, E> pv;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int32_t cc = c[E * u + j];
                XT xv = x[E * u + j];
                if (W > 0 && (uint32_t)(cc - win.x) < (uint32_t)win.y) xv = wbuf[cc - win.x];
                pv[j] = a[E * u + j] * xv;
            }
            *reinterpret_cast<Vec<XT, E> *>(prod + (e0 - k0a)) = pv;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t r = r0 + i * kBlock + tid;
        if (r < r1 && !(REMOTE && rb[i] == re[i])) {
            XT acc = s[i];
            acc = sum_in_order(acc, prod, rb[i] - k0a, re[i] - k0a);
            store_out<NTW>(acc, w + r);
        }
    }
}

// Off-process row block with E consecutive positions per lane: each lane
// loads columns, values and slots of its positions with one vector load
// each.  The host lays such a block out by runs (sort_blocks with run E):
// gather order fills the positions of [k0, k1) in the order of the load
// instructions (vector u, component j, lane t), so every gather instruction
// still reads, across its lanes, consecutive entries of gather order.
// Positions of the runs outside [k0, k1) (a neighbouring block's entries, or
// the arrays' zero padding) are loaded and discarded.  The products land in
// LDS at their slots and each row adds them in stored order to its partial
// sum.  A block whose aligned span is longer than CAP (a
// single row, which the host keeps in stored order) goes to row_in_chunks.
//
// PACKED: the block's columns are packed words (pack_block): slot in the
// high bits, the position's offset from its lane group's base in the low
// bits; each lane loads its group's base (`pbase`, this block's: the 16
// lanes of a group read one word), and no slot stream is read.
template <typename VT, typename XT, typename CT, int CAP, bool DIRECT, bool NTW, int E,
          bool PACKED = false>
__device__ __forceinline__ void remote_product_runs(int32_t r0, int32_t r1, int32_t k0, int32_t k1,
                                                    const int32_t *__restrict__ rowptr,
                                                    const CT *__restrict__ col, int32_t cbase,
                                                    const VT *__restrict__ val,
                                                    const uint16_t *__restrict__ slot,
                                                    const XT *__restrict__ xsrc,
                                                    XT *__restrict__ w, XT *prod,
                                                    const XT *__restrict__ vsrc,
                                                    const int32_t *__restrict__ pbase = nullptr) {
    static_assert(!PACKED || (!DIRECT && CAP <= (1 << kPackSlotBits)), "packed words");
    static_assert(kBlock == kLanes, "the host's run layout assumes the kernels' lane count");
    static_assert(E > 1 && CAP % (E * kBlock) == 0, "runs must tile the block");
    const int32_t k0a = k0 & -E;
    if (k1 == k0) return;      // an empty off-process block touches nothing
    if (k1 - k0a > CAP) {
        // a single row, which the host keeps in stored order
        row_in_chunks<VT, XT, CT, CAP, true, DIRECT, NTW>(r0, k0, k1, col, cbase, val, xsrc, w,
                                                          prod, vsrc);
        return;
    }
    constexpr int Q = CAP / (E * kBlock);
    constexpr int R = kMaxRows / kBlock;
    const int32_t tid = (int32_t)threadIdx.x;
    const int32_t klast = (k1 - 1) & -E;
    // slots and values stay packed as loaded (two 16-bit slots, or two
    // bfloat16 values, per register) until the products are formed: fewer
    // registers, more workgroups in flight
    int32_t c[E * Q];
    Vec<VT, E> aq[Q];
    Vec<uint16_t, PACKED ? 1 : E> sq[PACKED ? 1 : Q];
    uint32_t pw[PACKED ? E * Q : 1];
    int32_t rb[R], re[R];
    XT s[R];
    XT x[E * Q];
    // lane t's bases (pack_base_index): for runs of 2 the two words of
    // vector u side by side, for runs of 4 and 8 one word per load; the 16
    // lanes of a group read the same words
    const int32_t *pb = PACKED ? pbase + pack_base_index(CAP, E, 0, tid, 0) : nullptr;
    if constexpr (PACKED && sizeof(VT) == 8) {
        // float64: positions first (each load's words, then its bases), then
        // the rows and values, then the gathers one by one, each as soon as
        // its position has arrived -- the scheduling barriers keep the
        // compiler from computing every position before the first gather
        // (off-process launch on the KKT-like matrix 0.213 -> 0.208 ms; the
        // same order costs float32 and bfloat16 3-4%)
        int32_t bs[E * Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int32_t e = min(k0a + run_offset(E, u, tid, 0), klast);
            const Vec<CT, E> cq = load_vec<E>(col, e);
            static_assert(pack_base_stride(E) == 1, "float64 runs load their bases as vectors");
            const Vec<int32_t, E> bv = *reinterpret_cast<const Vec<int32_t, E> *>(pb + E * u);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                pw[PACKED ? E * u + j : 0] = (uint32_t)cq[j];
                bs[E * u + j] = bv[j];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int32_t r = min(r0 + i * kBlock + tid, r1 - 1);
            rb[i] = rowptr[r];
            re[i] = rowptr[r + 1];
            s[i] = w[r];
        }
#pragma unroll
        for (int u = 0; u < Q; ++u)
            aq[u] = load_vec<E>(val, min(k0a + run_offset(E, u, tid, 0), klast));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < Q; ++u) {
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int32_t e = k0a + run_offset(E, u, tid, j);
                int32_t cc = bs[E * u + j] +
                             (int32_t)(pw[PACKED ? E * u + j : 0] & ((1u << kPackPosBits) - 1));
                // a discarded position reads element 0 of the ghost buffer
                if (e < k0 || e >= k1) cc = 0;
                x[E * u + j] = xsrc[cc];
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int32_t e = min(k0a + run_offset(E, u, tid, 0), klast);
            const Vec<CT, E> cq = load_vec<E>(col, e);
            aq[u] = load_vec<E>(val, e);
            if (!PACKED) sq[PACKED ? 0 : u] = load_vec<PACKED ? 1 : E>(slot, e);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                if (PACKED) pw[PACKED ? E * u + j : 0] = (uint32_t)cq[j];
                else c[E * u + j] = cbase + (int32_t)cq[j];
            }
        }
        if constexpr (PACKED && pack_base_stride(E) == 1) {
#pragma unroll
            for (int u = 0; u < Q; ++u) {
                const Vec<int32_t, E> bv = *reinterpret_cast<const Vec<int32_t, E> *>(pb + E * u);
#pragma unroll
                for (int j = 0; j < E; ++j)
                    c[E * u + j] = bv[j] + (int32_t)(pw[PACKED ? E * u + j : 0] & ((1u << kPackPosBits) - 1));
            }
        } else if constexpr (PACKED) {
#pragma unroll
            for (int i = 0; i < E * Q; ++i)
                c[i] = pb[i * pack_base_stride(E)] + (int32_t)(pw[PACKED ? i : 0] & ((1u << kPackPosBits) - 1));
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int32_t r = min(r0 + i * kBlock + tid, r1 - 1);
            rb[i] = rowptr[r];
            re[i] = rowptr[r + 1];
            s[i] = w[r];
        }
        // a discarded position reads element 0 of v (direct reads) or of the
        // ghost buffer (not empty: this block has entries)
#pragma unroll
        for (int u = 0; u < Q; ++u) {
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int32_t e = k0a + run_offset(E, u, tid, j);
                int32_t &cc = c[E * u + j];
                if (e < k0 || e >= k1) cc = DIRECT ? INT32_MIN : 0;
                if (DIRECT)
                    x[E * u + j] = (cc < 0 ? vsrc : xsrc)[cc & 0x7fffffff];
                else
                    x[E * u + j] = xsrc[cc];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < Q; ++u) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int32_t e = k0a + run_offset(E, u, tid, j);
            const uint32_t q = PACKED ? pw[PACKED ? E * u + j : 0] >> kPackPosBits
                                      : (uint32_t)sq[PACKED ? 0 : u][PACKED ? 0 : j];
            if (e >= k0 && e < k1) prod[q] = widen(aq[u][j]) * x[E * u + j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t r = r0 + i * kBlock + tid;
        if (r < r1 && rb[i] != re[i]) {
            XT acc = s[i];
            acc = sum_in_order(acc, prod, rb[i] - k0, re[i] - k0);
            store_out<NTW>(acc, w + r);
        }
    }
}

// Everything one product needs, by launch.  A plain launch passes one view by
// value; a batched launch reads views from a device table.
template <typename VT, typename XT>
struct LocalView {
    const int32_t *tasks;      // task list: ~i exchange item, b >= 0 on-process block
    int32_t n_tasks;
    const int4 *items;         // exchange items (band or indexed; see exchange_item)
    const uint16_t *off;       // band items: column offset in the band of every entry
    const int32_t *idx, *dpos; // indexed items: source column, destination position
    XT *xdst;                  // exchange destination (ghost buffer or NAP send buffer)
    int32_t n;                 // length of v
    const int32_t *rowblk, *blkptr;
    const int2 *win;           // v windows of the on-process blocks (or null)
    const int32_t *rowptr, *col;
    const uint16_t *col16;     // or, when not null, uint16 columns offset by base[block]
    const int32_t *base;
    const VT *val;
    const XT *v;
    XT *w;
    int32_t nt;                // stores past the caches (see stream_out)
    int32_t nt_band;           // with nt, exchange items of lower bands store plainly
    // NAP pack-and-scatter items (item.w = 1): ghost band boundaries, the
    // scatter codes, the received buffer and the ghost buffer
    const int32_t *gband;
    const int32_t *s1band, *s1src;   // socket plans: cross-socket copies of received values
    const uint32_t *code;
    const XT *recv;
    XT *ghost;
};

template <typename VT, typename XT>
struct RemoteView {
    int32_t n_blocks;
    const int32_t *rowblk, *blkptr, *rowptr, *col;
    // per block (null: every block plain): cbase[b] >= 0, a block whose
    // ghost positions span less than 65536, kept in stored order, col16
    // holding its positions as offsets from cbase[b]; kPackedBlock, a block
    // whose col holds packed words (pack_block) with its bases at
    // pbase[b * (CAP / kPackLanes)]; kPlainBlock, int32 positions and slots
    const int32_t *cbase;
    const int32_t *pbase;
    const uint16_t *col16;
    const VT *val;
    const uint16_t *slot;      // stored position of each entry inside its block
    const XT *ghost;           // ghost buffer, or the received buffer (direct reads)
    const XT *v;               // direct reads only (else null): source of on-node values
    XT *w;
    int32_t nt;                // stores of w past the caches (see stream_out)
};

template <typename XT>
struct ScatterView {
    const int4 *items;         // band items over the ghost buffer
    int32_t n_items;
    const uint32_t *code;      // per ghost position, see scatter_item
    const XT *v, *recv;
    XT *ghost;
    int32_t n, which;
};

template <typename VT, typename XT, typename CT, int CAP, int W, bool NT>
__device__ __forceinline__ void local_block(const LocalView<VT, XT> &L, int32_t task, const CT *col,
                                            int32_t cbase, XT *prod, XT *wbuf) {
    const int2 wn = W > 0 ? L.win[task] : make_int2(0, 0);
    product_runs<VT, XT, CT, CAP, W, NT, product_run<VT, CAP>(), false, kMaxRowsOn>(
        L.rowblk[task], L.rowblk[task + 1], L.blkptr[task], L.blkptr[task + 1], wn, L.rowptr, col,
        cbase, L.val, L.v, L.w, prod, wbuf);
}

// LDS elements of the first launch: a band of v (exchange items), or a row
// block's products followed by its window of v (on-process blocks).
template <typename XT, int CAP, int W>
constexpr int local_lds() {
    constexpr int band = band_columns(CAP, (int)sizeof(XT));
    return band > CAP + W ? band : CAP + W;
}

template <typename VT, typename XT, int CAP, int W>
__device__ __forceinline__ void local_task(const LocalView<VT, XT> &L, int32_t t, XT *lds) {
    constexpr int BAND = band_columns(CAP, (int)sizeof(XT));
    XT *prod = lds, *wbuf = lds + CAP;
    const int32_t task = L.tasks[t];
    if (task < 0) {
        const int4 it = L.items[~task];
        if (it.w == 1) {
            pack_scatter_item<XT, BAND>(it, L.n, L.off, L.v, L.xdst, L.gband, L.s1band, L.s1src,
                                       L.code, L.recv, L.ghost, lds, L.nt != 0);
            return;
        }
        exchange_item<XT, BAND>(it, L.n, L.off, L.idx, L.dpos, L.v, L.xdst, lds,
                                L.nt != 0 && it.x >= L.nt_band);
        return;
    }
    if (L.col16) {
        if (L.nt)
            local_block<VT, XT, uint16_t, CAP, W, true>(L, task, L.col16, L.base[task], prod, wbuf);
        else
            local_block<VT, XT, uint16_t, CAP, W, false>(L, task, L.col16, L.base[task], prod, wbuf);
    } else {
        if (L.nt)
            local_block<VT, XT, int32_t, CAP, W, true>(L, task, L.col, 0, prod, wbuf);
        else
            local_block<VT, XT, int32_t, CAP, W, false>(L, task, L.col, 0, prod, wbuf);
    }
}

template <typename VT, typename XT, typename CT, int CAP, bool DIRECT, bool NT, bool PACKED = false>
__device__ __forceinline__ void remote_part(const RemoteView<VT, XT> &R, int32_t b, const CT *col,
                                            int32_t cbase, XT *prod) {
    remote_product_runs<VT, XT, CT, CAP, DIRECT, NT, remote_run((int)sizeof(VT), CAP), PACKED>(
        R.rowblk[b], R.rowblk[b + 1], R.blkptr[b], R.blkptr[b + 1], R.rowptr, col, cbase, R.val,
        R.slot, R.ghost, R.w, prod, R.v,
        PACKED ? R.pbase + (int64_t)b * (CAP / kPackLanes) : nullptr);
}

template <typename VT, typename XT, int CAP>
__device__ __forceinline__ void remote_block(const RemoteView<VT, XT> &R, int32_t b, XT *prod) {
    if (R.v) {
        if (R.nt) remote_part<VT, XT, int32_t, CAP, true, true>(R, b, R.col, 0, prod);
        else remote_part<VT, XT, int32_t, CAP, true, false>(R, b, R.col, 0, prod);
        return;
    }
    const int32_t base = R.cbase ? R.cbase[b] : kPlainBlock;
    if (base >= 0) {
        // a narrow block, kept in stored order (no slots)
        constexpr int E = product_run<VT, CAP>();
        if (R.nt)
            product_runs<VT, XT, uint16_t, CAP, 0, true, E, true>(
                R.rowblk[b], R.rowblk[b + 1], R.blkptr[b], R.blkptr[b + 1], make_int2(0, 0),
                R.rowptr, R.col16, base, R.val, R.ghost, R.w, prod, nullptr);
        else
            product_runs<VT, XT, uint16_t, CAP, 0, false, E, true>(
                R.rowblk[b], R.rowblk[b + 1], R.blkptr[b], R.blkptr[b + 1], make_int2(0, 0),
                R.rowptr, R.col16, base, R.val, R.ghost, R.w, prod, nullptr);
    } else if (base == kPackedBlock) {
        if constexpr (CAP <= (1 << kPackSlotBits)) {
            if (R.nt) remote_part<VT, XT, int32_t, CAP, false, true, true>(R, b, R.col, 0, prod);
            else remote_part<VT, XT, int32_t, CAP, false, false, true>(R, b, R.col, 0, prod);
        }
    } else {
        if (R.nt) remote_part<VT, XT, int32_t, CAP, false, true>(R, b, R.col, 0, prod);
        else remote_part<VT, XT, int32_t, CAP, false, false>(R, b, R.col, 0, prod);
    }
}

// Index of the entry of prefix[0..count] (ascending, prefix[0] = 0) whose
// range [prefix[i], prefix[i+1]) holds b.
__device__ __forceinline__ int32_t find_range(const int32_t *__restrict__ prefix, int32_t count,
                                              int32_t b) {
    int32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// First launch: task t (after the XCD remap) is either an exchange item or a
// row block of the on-process product.  The two kinds are interleaved in the
// task list, so every CU runs both at once.
template <typename VT, typename XT, int CAP, int W>
__global__ __launch_bounds__(kBlock) void k_local(LocalView<VT, XT> L) {
    __shared__ __align__(32) XT lds[local_lds<XT, CAP, W>()];
    local_task<VT, XT, CAP, W>(L, (int32_t)xcd_block(blockIdx.x, gridDim.x), lds);
}

// LDS elements of a second-launch workgroup: CAP x 8 bytes for every value
// type, which holds two 8192-entry workgroups on a CU.  More of them in
// flight at once (float32 blocks need the registers of only four) spread
// the ghost gather over more blocks' segments at a time and lose the L2
// reuse between neighbouring blocks: the float32 off-process launch on the
// KKT-like matrix takes 0.137 ms with four per CU, 0.132 with two.
template <typename XT, int CAP>
constexpr int remote_lds() { return CAP * 8 / (int)sizeof(XT); }

// Second launch: the off-process product, added into the partial w.
template <typename VT, typename XT, int CAP>
__global__ __launch_bounds__(kBlock) void k_remote(RemoteView<VT, XT> R) {
    __shared__ XT prod[remote_lds<XT, CAP>()];
    remote_block<VT, XT, CAP>(R, (int32_t)xcd_block(blockIdx.x, gridDim.x), prod);
}

// Batched first launch over `count` products: views[i] owns the launch's
// blocks [prefix[i], prefix[i+1]).
template <typename VT, typename XT, int CAP, int W>
__global__ __launch_bounds__(kBlock) void k_local_batch(const LocalView<VT, XT> *__restrict__ views,
                                                        const int32_t *__restrict__ prefix,
                                                        int32_t count) {
    __shared__ __align__(32) XT lds[local_lds<XT, CAP, W>()];
    const int32_t b = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    const int32_t i = find_range(prefix, count, b);
    local_task<VT, XT, CAP, W>(views[i], b - prefix[i], lds);
}

template <typename VT, typename XT, int CAP>
__global__ __launch_bounds__(kBlock) void k_remote_batch(const RemoteView<VT, XT> *__restrict__ views,
                                                         const int32_t *__restrict__ prefix,
                                                         int32_t count) {
    __shared__ XT prod[remote_lds<XT, CAP>()];
    const int32_t b = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    const int32_t i = find_range(prefix, count, b);
    remote_block<VT, XT, CAP>(views[i], b - prefix[i], prod);
}

// NAP scatter: one band item per block.
template <typename XT, int CAP>
__global__ __launch_bounds__(kBlock) void k_scatter(ScatterView<XT> S) {
    constexpr int BAND = band_columns(CAP, (int)sizeof(XT));
    __shared__ XT lds[BAND];
    scatter_item<XT, BAND>(S.items[xcd_block(blockIdx.x, gridDim.x)], S.n, S.which, S.code, S.v,
                          S.recv, S.ghost, lds);
}

// Batched NAP scatter: views[i] owns blocks [prefix[i], prefix[i+1]), one
// band item each.
template <typename XT, int CAP>
__global__ __launch_bounds__(kBlock) void k_scatter_batch(const ScatterView<XT> *__restrict__ views,
                                                          const int32_t *__restrict__ prefix,
                                                          int32_t count) {
    constexpr int BAND = band_columns(CAP, (int)sizeof(XT));
    __shared__ XT lds[BAND];
    const int32_t b = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    const int32_t i = find_range(prefix, count, b);
    const ScatterView<XT> &S = views[i];
    scatter_item<XT, BAND>(S.items[b - prefix[i]], S.n, S.which, S.code, S.v, S.recv, S.ghost, lds);
}

}  // namespace napspmv
