// Shared host/device helpers of libcpd (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string>

#include "../../include/cpd.h"

namespace cpd {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

// Keep memory returned to the current device's stream-ordered pool cached in
// the pool (release threshold raised once per device), so repeated builds and
// solves reuse it instead of mapping fresh pages.
void keep_pool_memory();

#define CPD_FAIL(code, ...)              \
    do {                                 \
        ::cpd::set_error(__VA_ARGS__);   \
        return (code);                   \
    } while (0)

#define CPD_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::cpd::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                             __FILE__, __LINE__);                                       \
            return (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)        \
                       ? CPD_ENOMEM                                                     \
                       : CPD_EHIP;                                                      \
        }                                                                               \
    } while (0)

#define CPD_TRY(expr)                     \
    do {                                  \
        cpd_status s_ = (expr);           \
        if (s_ != CPD_OK) return s_;      \
    } while (0)

#define CPD_LAUNCH_CHECK() CPD_HIP(hipGetLastError())

// Scratch blocks for stream-ordered use on stream s: reused from a cache of
// blocks released on the same stream, else taken from the stream-ordered pool.
cpd_status scratch_get(size_t bytes, hipStream_t s, void **p);
// Every device allocation of the library (stream-ordered): CPD_ENOMEM when
// the runtime refuses it or when it exceeds the limit cpd_set_alloc_limit set.
cpd_status device_alloc(void **p, size_t bytes, hipStream_t s);
void scratch_put(void *p, size_t bytes, hipStream_t s);

// Stream-ordered scratch buffer that returns itself to the scratch cache on
// scope exit.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    cpd_status alloc(size_t count, hipStream_t stream) {
        release();
        s = stream;
        n = count;
        if (count == 0) return CPD_OK;
        void *q = nullptr;
        cpd_status st = scratch_get(count * sizeof(T), stream, &q);
        p = static_cast<T *>(q);
        return st;
    }
    void release() {
        if (p) scratch_put(p, n * sizeof(T), s);
        p = nullptr;
        n = 0;
    }
    T *detach() {
        T *q = p;
        p = nullptr;
        n = 0;
        return q;
    }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------- device side
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// A load of data each launch reads once (a tree's leaf stream): the
// nontemporal hint streams it through the caches, so that it does not evict
// the factor rows the gathers reuse.
template <typename T>
__device__ __forceinline__ T stream_load(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Block-wide helpers for 256-thread blocks (4 waves of 64).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace cpd
