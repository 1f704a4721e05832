// hbm_device.h -- device-side helpers for gfx950 kernels (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hbm {

constexpr int WAVE = 64;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // each product as one 32x32->64 multiply (one v_mad_u64_u32 instead of a low and a high
        // multiply)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u, p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t pick4(const uint4 &y, uint32_t q) {
    return q == 0 ? y.x : q == 1 ? y.y : q == 2 ? y.z : y.w;
}

// Uniform root of RR set j: floor(x * n / 2^64), x the first 64 bits of the tag-0 draw.
__device__ __forceinline__ uint32_t rr_root(uint64_t seed, uint64_t j, uint32_t n) {
    const uint4 y = philox10((uint32_t)j, (uint32_t)(j >> 32), 0u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t x = (uint64_t)y.x | ((uint64_t)y.y << 32);
    return (uint32_t)__umul64hi(x, (uint64_t)n);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Order LDS traffic between the lanes of one wave (single-wave workgroups need no s_barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes of a wave.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const unsigned l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(v, d, WAVE);
        if (l >= (unsigned)d) v += o;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        uint64_t o = __shfl_xor(v, d, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// Read 32 bits of an MSB-first bit stream starting at bit `pos` (buffer padded by one word).
__device__ __forceinline__ uint32_t peek32(const uint32_t *__restrict__ buf, uint64_t pos) {
    const uint64_t w = pos >> 5;
    const uint32_t sh = (uint32_t)(pos & 31);
    const uint64_t two = ((uint64_t)buf[w] << 32) | (uint64_t)buf[w + 1];
    return (uint32_t)((two << sh) >> 32);
}

// Binary search: first index in [lo, hi) with a[i] > key (a non-decreasing).
template <class T, class I>
__device__ __forceinline__ I upper_bound_dev(const T *__restrict__ a, I lo, I hi, T key) {
    while (lo < hi) {
        I mid = lo + (hi - lo) / 2;
        if (a[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace hbm

namespace hbm {

// ---------------------------------------------------------------- grouped launches
// One launch serves many independent jobs: job i owns blocks [boff[i], boff[i+1]) of
// the grid and reads its own argument block args[i].  A kernel body takes its block
// position within its job explicitly, so the same body runs as a plain kernel (one job,
// arguments by value) or as a grouped one.
template <class Args>
struct GroupArgs {
    const Args *args;
    const uint32_t *boff;  // count + 1 block offsets
    uint32_t count;
    int x;                 // extra scalar shared by all jobs (e.g. the selection iteration)
};

__device__ __forceinline__ uint32_t group_of(const uint32_t *boff, uint32_t count, uint32_t b) {
    uint32_t lo = 0, hi = count - 1;  // last job whose first block is <= b
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The root a store leaves out of set j under implicit roots (~0u: every member is stored).
__device__ __forceinline__ uint32_t dropped_root(int implicit, uint64_t seed, uint64_t j, uint32_t n) {
    return implicit ? rr_root(seed, j, n) : 0xFFFFFFFFu;
}

// Plain ids of a store: [0, split) in device memory, [split, ...) in pinned host memory that
// the GPU reads over the bus (split is a multiple of 4, so 16-byte loads never straddle it).
__device__ __forceinline__ int32_t raw_id(const int32_t *dev, const int32_t *host, int64_t split, int64_t i) {
    return i < split ? dev[i] : host[i - split];
}
__device__ __forceinline__ uint4 raw_id4(const int32_t *dev, const int32_t *host, int64_t split, int64_t q) {
    const int64_t i = q * 4;
    return i < split ? reinterpret_cast<const uint4 *>(dev)[q] : reinterpret_cast<const uint4 *>(host + (i - split))[0];
}

#define HBM_KERNEL(NAME, ARGS, THREADS)                                                              \
    __device__ void NAME##_body(const ARGS &A, uint32_t bid, uint32_t nblk, int x);                  \
    __global__ __launch_bounds__(THREADS) void NAME(ARGS A, int x) { NAME##_body(A, blockIdx.x, gridDim.x, x); } \
    __global__ __launch_bounds__(THREADS) void NAME##_g(GroupArgs<ARGS> G) {                         \
        const uint32_t i = group_of(G.boff, G.count, blockIdx.x);                                     \
        const ARGS a_ = G.args[i]; /* uniform: held in scalar registers, not re-read */              \
        NAME##_body(a_, blockIdx.x - G.boff[i], G.boff[i + 1] - G.boff[i], G.x);                      \
    }                                                                                                \
    __device__ void NAME##_body(const ARGS &A, uint32_t bid, uint32_t nblk, int x)

}  // namespace hbm
