// gfx950 kernels of the apply path: index gathers and scatters that carry
// the plan's messages, and the split CSR product.
//
// Every kernel is memory-bound (the product does 2 flops per 12-16 bytes),
// so the design is about bytes and latency, not arithmetic: 256-thread
// blocks of four wave64s, one load per element with no reuse, and an
// XCD-aware block order for the product so that the eight L2 caches each see
// a contiguous range of rows (the vector window and ghost segment of the few
// processes an XCD is working on stay in that XCD's L2).
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

// Widening loads of a stored value of A into the accumulation type.
__device__ __forceinline__ double load_val(const double *p, int32_t k) { return p[k]; }
__device__ __forceinline__ float load_val(const float *p, int32_t k) { return p[k]; }
__device__ __forceinline__ float load_val(const uint16_t *p, int32_t k) {
    return __uint_as_float((uint32_t)p[k] << 16);   // bfloat16 -> float32 is exact
}

// dst[k] = src[idx[k]] for k < n: the pack loop of a phase (every message of
// the phase concatenated), or the standard ghost gather.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int32_t n, const int32_t *__restrict__ idx,
                                                   const T *__restrict__ src, T *__restrict__ dst) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k < (uint32_t)n) dst[k] = src[idx[k]];
}

// Two indexed copies in one launch: ghost[d1[k]] = s1v[s1[k]] (received
// inter-node values, to their users on the node) for the first nb1 blocks,
// ghost[d2[k]] = s2v[s2[k]] (fully local on-node values) for the rest.  Each
// ghost slot appears in exactly one of the two lists, once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter2(
    int32_t n1, const int32_t *__restrict__ s1, const int32_t *__restrict__ d1,
    const T *__restrict__ s1v, int32_t n2, const int32_t *__restrict__ s2,
    const int32_t *__restrict__ d2, const T *__restrict__ s2v, T *__restrict__ ghost,
    uint32_t nb1) {
    if (blockIdx.x < nb1) {
        const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
        if (k < (uint32_t)n1) ghost[d1[k]] = s1v[s1[k]];
    } else {
        const uint32_t k = (blockIdx.x - nb1) * kBlock + threadIdx.x;
        if (k < (uint32_t)n2) ghost[d2[k]] = s2v[s2[k]];
    }
}

// dst[k] = src[k]: the explicit inter-node hop (send buffer -> receive buffer).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int32_t n, const T *__restrict__ src,
                                                 T *__restrict__ dst) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k < (uint32_t)n) dst[k] = src[k];
}

// Split CSR product, S lanes per row (a subwave), 256/S rows per block:
//   w[i] = sum over the row's entries of a * x,  x = v[c] (c >= 0, on-process)
//                                                 or ghost[c & 0x7fffffff] (off-process).
// VT: stored value type (double, float, uint16 bfloat16 bits); XT: vector
// type; the accumulator is XT (double for float64 plans, float otherwise).
template <typename VT, typename XT, int S>
__global__ __launch_bounds__(kBlock) void k_spmv(int32_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const VT *__restrict__ val,
                                                 const XT *__restrict__ v,
                                                 const XT *__restrict__ ghost,
                                                 XT *__restrict__ w) {
    constexpr int kRows = kBlock / S;
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t row = b * kRows + threadIdx.x / S;
    const int lane = threadIdx.x % S;
    if (row >= (uint32_t)n) return;     // whole subwaves leave together
    const int32_t beg = rowptr[row], end = rowptr[row + 1];
    XT sum = 0;
    for (int32_t k = beg + lane; k < end; k += S) {
        const int32_t c = col[k];
        const XT a = (XT)load_val(val, k);
        const XT *p = c >= 0 ? v + c : ghost + (c & 0x7fffffff);
        sum = fma(a, *p, sum);
    }
#pragma unroll
    for (int o = S / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, S);
    if (lane == 0) w[row] = sum;
}

}  // namespace napspmv
