// Prefix sums and the LSD radix sort used to build CoCo (Section 4: the index
// is built by sorting each relation lexicographically in the variable order).
//
// Radix sort: least-significant-digit first, 8-bit digits, reduce-then-scan
// per pass (Merrill and Grimshaw, "High performance and scalable radix sorting",
// 2011): (1) every 4096-key tile counts its digits in LDS, (2) an exclusive scan
// over the digit-major count matrix gives each (digit, tile) its output start,
// (3) every tile ranks its keys stably with wave64 ballots (keys whose digit
// bits all agree form one match mask; the rank is the popcount of earlier
// lanes), stages them in LDS grouped by digit, and writes each digit's run
// contiguously to HBM.
#include "prim_dev.h"

namespace hc {

constexpr int kRsRows = 16;                       // rows of 64 keys per wave
constexpr int kRsWaveKeys = kRsRows * 64;          // 1024
constexpr int kRsTile = kWaves * kRsWaveKeys;      // 4096 keys per workgroup

// Mask of the lanes holding the same 8-bit digit as this lane (valid lanes only).
__device__ inline uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ in, int64_t n, int shift,
                                                       uint32_t* __restrict__ counts, int64_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * kRsWaveKeys;
    for (int r = 0; r < kRsRows; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)(in[i] >> shift) & 255u : 0u;
        const uint64_t m = match_digit(d, valid);
        if (valid && (m & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                          int64_t n, int shift, const uint64_t* __restrict__ offs,
                                                          int64_t ntiles) {
    __shared__ uint64_t s_keys[kRsTile];
    __shared__ uint32_t s_wcnt[kWaves][256];
    __shared__ uint32_t s_dstart[256];
    __shared__ uint64_t s_gbase[256];
    __shared__ uint64_t lds4[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kRsTile + (int64_t)w * kRsWaveKeys;
    for (int d = tid; d < kWaves * 256; d += kBlock) (&s_wcnt[0][0])[d] = 0;
    __syncthreads();
    uint64_t key[kRsRows];
    uint32_t rank[kRsRows];
#pragma unroll
    for (int r = 0; r < kRsRows; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? in[i] : 0;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        const uint32_t pre = (uint32_t)__popcll(m & lanemask_lt());
        uint32_t before = 0;
        if (valid) before = s_wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && pre == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        rank[r] = before + pre;
    }
    __syncthreads();
    {
        const int d = tid;
        const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint64_t blk_total;
        const uint64_t start = block_exclusive_sum(tot, lds4, &blk_total);
        s_wcnt[0][d] = 0;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
        s_dstart[d] = (uint32_t)start;
        s_gbase[d] = offs[(int64_t)d * ntiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRows; ++r) {
        const int64_t i = base + r * 64 + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            s_keys[s_dstart[d] + s_wcnt[w][d] + rank[r]] = key[r];
        }
    }
    __syncthreads();
    const int64_t rem = n - tile * kRsTile;
    const int tile_n = rem < kRsTile ? (int)rem : kRsTile;
    for (int j = tid; j < tile_n; j += kBlock) {
        const uint64_t k = s_keys[j];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        out[s_gbase[d] + (uint64_t)(j - (int)s_dstart[d])] = k;
    }
}

void radix_sort_u64(const Alloc& a, DevBuf<uint64_t>& keys, DevBuf<uint64_t>& tmp, int64_t n, int bits,
                    hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t ntiles = (n + kRsTile - 1) / kRsTile;
    DevBuf<uint32_t> counts(a, (size_t)ntiles * 256);
    DevBuf<uint64_t> offs(a, (size_t)ntiles * 256 + 1);
    for (int shift = 0; shift < bits; shift += 8) {
        k_radix_hist<<<(unsigned)ntiles, kBlock, 0, s>>>(keys.p, n, shift, counts.p, ntiles);
        HC_HIP(hipGetLastError());
        scan_exclusive(a, LoadU32{counts.p}, offs.p, ntiles * 256, s);
        k_radix_scatter<<<(unsigned)ntiles, kBlock, 0, s>>>(keys.p, tmp.p, n, shift, offs.p, ntiles);
        HC_HIP(hipGetLastError());
        std::swap(keys.p, tmp.p);
    }
}

void scan_u32_to_u64(const Alloc& a, const uint32_t* in, uint64_t* out, int64_t n, hipStream_t s) {
    scan_exclusive(a, LoadU32{in}, out, n, s);
}
void scan_u64(const Alloc& a, const uint64_t* in, uint64_t* out, int64_t n, hipStream_t s) {
    scan_exclusive(a, LoadU64{in}, out, n, s);
}
void scan_popc(const Alloc& a, const uint64_t* words, uint64_t* out, int64_t n, hipStream_t s) {
    scan_exclusive(a, LoadPopc{words}, out, n, s);
}

}  // namespace hc
