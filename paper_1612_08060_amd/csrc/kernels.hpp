// gfx950 kernels of the apply path: index gathers and scatters that carry
// the plan's messages, and the split CSR product.
//
// An apply is two product launches, as algorithm standard_spmv (section 2.1)
// and NAPSpMV (section 4.3) order the work: the first launch runs the
// exchange that fills the ghost buffer (or the NAP send buffer) together
// with the on-process product local_spmv(A_on, v), which needs no received
// value; the second adds the off-process product local_spmv(A_off, ghost)
// into w.  The first launch interleaves its two kinds of blocks on every CU,
// so the exchange, bound by random L2 requests, overlaps the on-process
// product, bound by HBM streaming: the overlap of local work with
// communication the paper's algorithms make, on one GPU.
//
// Every kernel is HBM-bound (the product does 2 flops per 12-16 bytes), so
// the design is about bytes and latency, not arithmetic: 256-thread blocks of
// four wave64s; matrix streams (values, column tags) read once with
// non-temporal loads so they do not evict the vector and the ghost buffer
// from L2; many independent loads in flight per lane; and an XCD-aware block
// order, so that each of the eight L2 caches sees one contiguous range of the
// work (the vector window and the ghost segments of the processes an XCD is
// working on stay in that XCD's L2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Two indexed copies in one launch, XCD-aware: ghost[d1[k]] = s1v[s1[k]]
// (received inter-node values, to their users on the node) in the first nb1
// logical blocks, ghost[d2[k]] = s2v[s2[k]] (fully local on-node values) in
// the rest.  Each ghost slot appears in exactly one of the two lists, once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter2(
    int32_t n1, const int32_t *__restrict__ s1, const int32_t *__restrict__ d1,
    const T *__restrict__ s1v, int32_t n2, const int32_t *__restrict__ s2,
    const int32_t *__restrict__ d2, const T *__restrict__ s2v, T *__restrict__ ghost,
    uint32_t nb1) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    if (b < nb1) {
        const uint32_t k = b * kBlock + threadIdx.x;
        if (k < (uint32_t)n1)
            ghost[__builtin_nontemporal_load(d1 + k)] = s1v[__builtin_nontemporal_load(s1 + k)];
    } else {
        const uint32_t k = (b - nb1) * kBlock + threadIdx.x;
        if (k < (uint32_t)n2)
            ghost[__builtin_nontemporal_load(d2 + k)] = s2v[__builtin_nontemporal_load(s2 + k)];
    }
}

// dst[k] = src[k]: the explicit inter-node hop (send buffer -> receive buffer).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int32_t n, const T *__restrict__ src,
                                                 T *__restrict__ dst) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k < (uint32_t)n) dst[k] = src[k];
}

// dst[k] = src[idx[k]] for k in [start, start + len): one work item of a
// phase's concatenated messages (the standard ghost gather, or the NAP pack
// of the inter-node send buffer).  Four independent loads per lane in flight.
template <typename T>
__device__ __forceinline__ void gather_item(int2 it, const int32_t *__restrict__ idx,
                                            const T *__restrict__ src, T *__restrict__ dst) {
    const int32_t end = it.x + it.y;
    int32_t k = it.x + (int32_t)threadIdx.x;
    for (; k + 3 * kBlock < end; k += 4 * kBlock) {
        int32_t j[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = __builtin_nontemporal_load(idx + k + u * kBlock);
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = src[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[k + u * kBlock] = x[u];
    }
    for (; k < end; k += kBlock) dst[k] = src[__builtin_nontemporal_load(idx + k)];
}

// One row block of a split CSR product.  The block owns rows [r0, r1) (at
// most kMaxRows) and entries [k0, k1) of one of the two CSR parts, at most
// CAP of them (else a single long row, walked in chunks of CAP).  Every
// thread first issues all its loads at once: its share of the entries
// (coalesced, independent), of the block's v window, of the row pointers and,
// for the off-process part, of the partial sums.  Then it gathers the vector
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
constexpr int kMaxRows = 1024;

template <typename VT, typename XT, int CAP, int W, bool REMOTE>
__device__ __forceinline__ void product_block(int32_t r0, int32_t r1, int32_t k0, int32_t k1,
                                              int2 win, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const VT *__restrict__ val,
                                              const XT *__restrict__ xsrc, XT *__restrict__ w,
                                              XT *prod, XT *wbuf) {
    constexpr int U = CAP / kBlock;
    constexpr int R = kMaxRows / kBlock;
    const int tid = threadIdx.x;
    if (k1 - k0 > CAP) {
        XT s = REMOTE ? w[r0] : (XT)0;
        for (int32_t base = k0; base < k1; base += CAP) {
            const int32_t lim = (k1 - base) < CAP ? (k1 - base) : CAP;
            for (int32_t q = tid; q < lim; q += kBlock) {
                const int32_t k = base + q;
                prod[q] = (XT)load_val(val, k) * xsrc[__builtin_nontemporal_load(col + k)];
            }
            __syncthreads();
            if (tid == 0)
                for (int32_t q = 0; q < lim; ++q) s = s + prod[q];
            __syncthreads();
        }
        if (tid == 0) w[r0] = s;
        return;
    }
    int32_t c[U];
    XT a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * kBlock + tid;
        if (k < k1) {
            c[u] = __builtin_nontemporal_load(col + k);
            a[u] = (XT)load_val(val, k);
        }
    }
    XT t[W > 0 ? W / kBlock : 1];
    if (W > 0) {
#pragma unroll
        for (int u = 0; u < W / kBlock; ++u) {
            const int32_t q = u * kBlock + tid;
            if (q < win.y) t[u] = xsrc[win.x + q];
        }
    }
    int32_t rb[R], re[R];
    XT s[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t r = r0 + i * kBlock + tid;
        if (r < r1) {
            rb[i] = rowptr[r];
            re[i] = rowptr[r + 1];
            s[i] = REMOTE ? w[r] : (XT)0;
        }
    }
    XT x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * kBlock + tid;
        if (k < k1 && !(W > 0 && (uint32_t)(c[u] - win.x) < (uint32_t)win.y)) x[u] = xsrc[c[u]];
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
    for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * kBlock + tid;
        if (k < k1) {
            if (W > 0 && (uint32_t)(c[u] - win.x) < (uint32_t)win.y) x[u] = wbuf[c[u] - win.x];
            prod[k - k0] = a[u] * x[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t r = r0 + i * kBlock + tid;
        if (r < r1 && !(REMOTE && rb[i] == re[i])) {
            XT acc = s[i];
            for (int32_t q = rb[i] - k0; q < re[i] - k0; ++q) acc = acc + prod[q];
            w[r] = acc;
        }
    }
}

// First launch: tasks[b] (after the XCD remap) is either an exchange item
// (~i: xdst[k] = v[idx[k]] over items[i]) or a row block of the on-process
// product (b >= 0: rows rowblk[b].., entries blkptr[b].., window win[b]).
// The two kinds are interleaved in the task list, so every CU runs both at
// once.
template <typename VT, typename XT, int CAP, int W>
__global__ __launch_bounds__(kBlock) void k_local(
    const int32_t *__restrict__ tasks, const int2 *__restrict__ items,
    const int32_t *__restrict__ idx, XT *__restrict__ xdst,
    const int32_t *__restrict__ rowblk, const int32_t *__restrict__ blkptr,
    const int2 *__restrict__ win, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const VT *__restrict__ val, const XT *__restrict__ v,
    XT *__restrict__ w) {
    __shared__ XT prod[CAP];
    __shared__ XT wbuf[W > 0 ? W : 1];
    const int32_t task = tasks[xcd_block(blockIdx.x, gridDim.x)];
    if (task < 0) {
        gather_item(items[~task], idx, v, xdst);
        return;
    }
    const int2 wn = W > 0 ? win[task] : make_int2(0, 0);
    product_block<VT, XT, CAP, W, false>(rowblk[task], rowblk[task + 1], blkptr[task],
                                         blkptr[task + 1], wn, rowptr, col, val, v, w, prod, wbuf);
}

// Second launch: the off-process product, added into the partial w.
template <typename VT, typename XT, int CAP>
__global__ __launch_bounds__(kBlock) void k_remote(
    const int32_t *__restrict__ rowblk, const int32_t *__restrict__ blkptr,
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const VT *__restrict__ val, const XT *__restrict__ ghost, XT *__restrict__ w) {
    __shared__ XT prod[CAP];
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    product_block<VT, XT, CAP, 0, true>(rowblk[b], rowblk[b + 1], blkptr[b], blkptr[b + 1],
                                        make_int2(0, 0), rowptr, col, val, ghost, w, prod,
                                        nullptr);
}

}  // namespace napspmv
