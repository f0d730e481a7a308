// Device-wide exclusive scan (int32) of a functor over [0, n): three passes
// (tile reduce, scan of tile sums, tile scan + offset).  256-thread blocks,
// 16 items per thread, 4096 items per tile.
#pragma once

#include "common.h"

namespace cpd {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Inclusive scan of v across the 256 threads of a block; returns the inclusive
// value, and the block total in *tot.  smem: >= 4 ints.
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t v, int32_t *smem, int32_t *tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) smem[wave] = v;
    __syncthreads();
    int32_t off = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
        int32_t x = smem[w];
        if (w < wave) off += x;
        all += x;
    }
    __syncthreads();
    *tot = all;
    return v + off;
}

template <typename F>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(F f, int64_t n, int32_t *partial) {
    __shared__ int32_t smem[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (i < n) s += f(i);
    }
    int32_t tot;
    block_inclusive_scan(s, smem, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block scans nb tile sums in place (exclusive) and writes the grand total.
static __global__ void __launch_bounds__(SCAN_THREADS) k_scan_partials(int32_t *partial, int64_t nb,
                                                                 int32_t *total) {
    __shared__ int32_t smem[4];
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_THREADS) {
        int64_t i = b0 + threadIdx.x;
        int32_t v = i < nb ? partial[i] : 0;
        int32_t tot;
        int32_t inc = block_inclusive_scan(v, smem, &tot);
        if (i < nb) partial[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename F>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(F f, int64_t n, const int32_t *partial,
                                                            int32_t *out) {
    __shared__ int32_t smem[4];
    __shared__ int32_t tile[SCAN_TILE + SCAN_TILE / 32];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // coalesced evaluation into LDS (padded by one slot every 32 to spread banks)
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int p = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + p;
        tile[p + (p >> 5)] = i < n ? f(i) : 0;
    }
    __syncthreads();
    int32_t loc[SCAN_ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int p = threadIdx.x * SCAN_ITEMS + j;
        loc[j] = s;
        s += tile[p + (p >> 5)];
    }
    int32_t tot;
    int32_t inc = block_inclusive_scan(s, smem, &tot);
    int32_t off = partial[blockIdx.x] + inc - s;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int p = threadIdx.x * SCAN_ITEMS + j;
        tile[p + (p >> 5)] = off + loc[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int p = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + p;
        if (i < n) out[i] = tile[p + (p >> 5)];
    }
}

template <typename F>
cpd_status exclusive_scan(F f, int64_t n, int32_t *out, int32_t *total, hipStream_t s) {
    int64_t nb = ceil_div(n, SCAN_TILE);
    if (nb == 0) {
        if (total) CPD_HIP(hipMemsetAsync(total, 0, sizeof(int32_t), s));
        return CPD_OK;
    }
    DevBuf<int32_t> partial;
    CPD_TRY(partial.alloc(nb, s));
    hipLaunchKernelGGL(k_scan_reduce<F>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, f, n,
                       partial.p);
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, partial.p, nb, total);
    CPD_LAUNCH_CHECK();
    if (out) {
        hipLaunchKernelGGL(k_scan_down<F>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, f, n,
                           (const int32_t *)partial.p, out);
        CPD_LAUNCH_CHECK();
    }
    return CPD_OK;
}

}  // namespace cpd
