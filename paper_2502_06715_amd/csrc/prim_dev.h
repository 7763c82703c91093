// Device building blocks shared by the build and join kernels: wave64 scans and
// reductions, and a reduce-then-scan exclusive prefix sum with pluggable loads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hc_internal.h"

namespace hc {

constexpr int kBlock = 256;           // threads per workgroup: 4 wave64
constexpr int kWaves = kBlock / 64;

__device__ inline uint64_t lanemask_lt() { return __lanemask_lt(); }

__device__ inline uint64_t wave_inclusive_sum(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ inline uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline uint64_t wave_xor(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v ^= __shfl_xor(v, d, 64);
    return v;
}

// Exclusive scan of one value per thread across a 256-thread block; returns the
// exclusive prefix and writes the block total to *total.  Uses 4 u64 of LDS.
__device__ inline uint64_t block_exclusive_sum(uint64_t v, uint64_t* lds4, uint64_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_inclusive_sum(v);
    if (lane == 63) lds4[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        uint64_t s = lds4[k];
        if (k < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---------------------------------------------------------------- reduce-then-scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;   // 2048 items per workgroup

template <class Load>
__device__ inline void scan_reduce_tile(Load ld, int64_t n, uint64_t* partial) {
    __shared__ uint64_t lds4[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) s += ld(i);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int k = 0; k < kWaves; ++k) t += lds4[k];
        partial[blockIdx.x] = t;
    }
}

// out[i] = (partial ? partial[block] : 0) + sum of ld(j) for tile_base <= j < i;
// the block with writes_total set also writes out[n] = grand total.
template <class Load>
__device__ inline void scan_down_tile(Load ld, int64_t n, const uint64_t* partial, uint64_t* out,
                                      bool writes_total) {
    __shared__ uint64_t tile[kScanTile];
    __shared__ uint64_t lds4[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        tile[k * kBlock + threadIdx.x] = i < n ? ld(i) : 0;
    }
    __syncthreads();
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[threadIdx.x * kScanItems + k];
        s += v[k];
    }
    uint64_t total;
    uint64_t off = block_exclusive_sum(s, lds4, &total);
    const uint64_t pb = partial ? partial[blockIdx.x] : 0;
    off += pb;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + threadIdx.x * kScanItems + k;
        if (i < n) out[i] = off;
        off += v[k];
    }
    if (writes_total && threadIdx.x == 0) out[n] = pb + total;
}

template <class Load>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(Load ld, int64_t n, uint64_t* partial) {
    scan_reduce_tile(ld, n, partial);
}
template <class Load>
__global__ __launch_bounds__(kBlock) void k_scan_down(Load ld, int64_t n, const uint64_t* partial,
                                                      uint64_t* out) {
    scan_down_tile(ld, n, partial, out, blockIdx.x == gridDim.x - 1);
}

// Device-sized variants: the element count is read from device memory, so the
// launch sequence does not depend on it (a captured graph); the grid covers a
// fixed capacity, and blocks past the count write zero partials or leave.  The
// block holding position n writes out[n].
template <class Load>
__global__ __launch_bounds__(kBlock) void k_scan_reduce_dn(Load ld, const uint64_t* n_dev, uint64_t* partial) {
    scan_reduce_tile(ld, (int64_t)*n_dev, partial);
}
template <class Load>
__global__ __launch_bounds__(kBlock) void k_scan_down_dn(Load ld, const uint64_t* n_dev, const uint64_t* partial,
                                                         uint64_t* out) {
    const int64_t n = (int64_t)*n_dev;
    if ((int64_t)blockIdx.x * kScanTile > n) return;   // block-uniform
    scan_down_tile(ld, n, partial, out, (int64_t)blockIdx.x == n / kScanTile);
}

struct LoadU32 {
    const uint32_t* p;
    __device__ uint64_t operator()(int64_t i) const { return p[i]; }
};
struct LoadU64 {
    const uint64_t* p;
    __device__ uint64_t operator()(int64_t i) const { return p[i]; }
};
struct LoadPopc {
    const uint64_t* p;
    __device__ uint64_t operator()(int64_t i) const { return (uint64_t)__popcll(p[i]); }
};

template <class Load>
void scan_exclusive(const Alloc& a, Load ld, uint64_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) {
        HC_HIP(hipMemsetAsync(out, 0, sizeof(uint64_t), s));
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_scan_down<Load><<<1, kBlock, 0, s>>>(ld, n, nullptr, out);
        HC_HIP(hipGetLastError());
        return;
    }
    DevBuf<uint64_t> part(a, nb + 1);
    k_scan_reduce<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n, part.p);
    HC_HIP(hipGetLastError());
    scan_exclusive(a, LoadU64{part.p}, part.p, nb, s);   // in place: each tile is staged in LDS first
    k_scan_down<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n, part.p, out);
    HC_HIP(hipGetLastError());
}

// Workspace (u64 values) of scan_exclusive_ws over n elements: the partial sums of
// every level of the reduce-then-scan recursion.
inline int64_t scan_ws_size(int64_t n) {
    if (n <= kScanTile) return 0;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return nb + 1 + scan_ws_size(nb);
}
// scan_exclusive with its partial sums in a caller-provided workspace (no
// allocation, so it can be captured in a graph); n > 0.
template <class Load>
void scan_exclusive_ws(Load ld, uint64_t* out, int64_t n, uint64_t* ws, hipStream_t s) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) {
        k_scan_down<Load><<<1, kBlock, 0, s>>>(ld, n, nullptr, out);
        HC_HIP(hipGetLastError());
        return;
    }
    k_scan_reduce<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n, ws);
    HC_HIP(hipGetLastError());
    scan_exclusive_ws(LoadU64{ws}, ws, nb, ws + nb + 1, s);
    k_scan_down<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n, ws, out);
    HC_HIP(hipGetLastError());
}
// Workspace of scan_exclusive_dn for counts up to cap.
inline int64_t scan_dn_ws_size(int64_t cap) {
    const int64_t nb = cap / kScanTile + 1;
    return nb + 1 + scan_ws_size(nb);
}
// Exclusive scan of *n_dev <= cap elements (out has cap + 1 entries) with a launch
// sequence fixed by cap alone.
template <class Load>
void scan_exclusive_dn(Load ld, uint64_t* out, const uint64_t* n_dev, int64_t cap, uint64_t* ws, hipStream_t s) {
    const int64_t nb = cap / kScanTile + 1;
    k_scan_reduce_dn<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n_dev, ws);
    HC_HIP(hipGetLastError());
    scan_exclusive_ws(LoadU64{ws}, ws, nb, ws + nb + 1, s);
    k_scan_down_dn<Load><<<(unsigned)nb, kBlock, 0, s>>>(ld, n_dev, ws, out);
    HC_HIP(hipGetLastError());
}

// Binary search helpers over sorted uint32 arrays.
__device__ inline int64_t lower_bound_u32(const uint32_t* a, int64_t lo, int64_t hi, uint32_t v) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ inline int64_t lower_bound_u64key(const uint64_t* a, int64_t lo, int64_t hi, uint64_t v) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace hc
