// Lexicographic order of emitted rows (hc_join_emit with HC_EMIT_SORTED).
//
// The output of a join is a set of head-order tuples of raw ids below 2^b
// (Section 2, Eq. (1): Q(D) is a set).  When a whole row fits one 64-bit word
// (n_vars * b <= 64) the row itself is the sort key: rows are packed with the
// first column in the high bits, radix sorted on their n_vars * b significant
// bits and unpacked in place.  Otherwise the rows are ordered by a stable LSD
// pass per column, last column first, each pass sorting (row index, column
// value) pairs on the value's b bits; a final gather writes the rows in order.
#include "prim_dev.h"

namespace hc {

template <class T>
__global__ void k_pack_rows(const T* __restrict__ rows, int64_t n, int nv, int b, uint64_t* __restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = 0;
        for (int v = 0; v < nv; ++v) k = (k << b) | (uint64_t)(uint32_t)rows[i * nv + v];
        keys[i] = k;
    }
}

template <class T>
__global__ void k_unpack_rows(const uint64_t* __restrict__ keys, int64_t n, int nv, int b, T* __restrict__ rows) {
    const uint64_t mask = b >= 64 ? ~0ull : (1ull << b) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        for (int v = nv - 1; v >= 0; --v) {
            rows[i * nv + v] = (T)(uint32_t)(k & mask);
            k >>= b;
        }
    }
}

// keys[i] = (row index of position i) << 32 | column c of that row
template <class T>
__global__ void k_column_keys(const T* __restrict__ rows, const uint32_t* __restrict__ perm, int64_t n, int nv,
                              int c, uint64_t* __restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = perm ? perm[i] : (uint32_t)i;
        keys[i] = ((uint64_t)r << 32) | (uint64_t)(uint32_t)rows[(int64_t)r * nv + c];
    }
}

__global__ void k_keys_to_perm(const uint64_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ perm) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        perm[i] = (uint32_t)(keys[i] >> 32);
}

template <class T>
__global__ void k_gather_rows(const T* __restrict__ src, const uint32_t* __restrict__ perm, int64_t n, int nv,
                              T* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * nv;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / nv, v = i - row * nv;
        dst[i] = src[(int64_t)perm[row] * nv + v];
    }
}

static unsigned grid_rows(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

template <class T>
static void sort_rows_t(const Alloc& a, T* rows, int64_t n, int nv, int b, hipStream_t s) {
    DevBuf<uint64_t> keys(a, (size_t)n), tmp(a, (size_t)n);
    if ((int64_t)nv * b <= 64) {
        k_pack_rows<T><<<grid_rows(n), kBlock, 0, s>>>(rows, n, nv, b, keys.p);
        HC_HIP(hipGetLastError());
        radix_sort_u64(a, keys, tmp, n, nv * b, s);
        k_unpack_rows<T><<<grid_rows(n), kBlock, 0, s>>>(keys.p, n, nv, b, rows);
        HC_HIP(hipGetLastError());
        return;
    }
    HC_REQUIRE(n < ((int64_t)1 << 32), HC_ERR_UNSUPPORTED, "sorted emit of 2^32 rows or more");
    DevBuf<uint32_t> perm(a, (size_t)n);
    for (int c = nv - 1; c >= 0; --c) {
        k_column_keys<T><<<grid_rows(n), kBlock, 0, s>>>(rows, c == nv - 1 ? nullptr : perm.p, n, nv, c, keys.p);
        HC_HIP(hipGetLastError());
        radix_sort_u64(a, keys, tmp, n, b, s);   // stable: equal values keep the previous passes' order
        k_keys_to_perm<<<grid_rows(n), kBlock, 0, s>>>(keys.p, n, perm.p);
        HC_HIP(hipGetLastError());
    }
    keys.reset();
    tmp.reset();
    DevBuf<T> copy(a, (size_t)(n * nv));
    HC_HIP(hipMemcpyAsync(copy.p, rows, sizeof(T) * (size_t)(n * nv), hipMemcpyDeviceToDevice, s));
    k_gather_rows<T><<<grid_rows(n * nv), kBlock, 0, s>>>(copy.p, perm.p, n, nv, rows);
    HC_HIP(hipGetLastError());
}

void sort_rows(const Alloc& a, void* rows, int64_t n, int nv, int b, bool i64, hipStream_t s) {
    if (n <= 1) return;
    HC_REQUIRE(b >= 1 && b <= 32 && nv >= 1, HC_ERR_INVALID, "sort_rows: bad row shape");
    if (i64) sort_rows_t<int64_t>(a, (int64_t*)rows, n, nv, b, s);
    else sort_rows_t<int32_t>(a, (int32_t*)rows, n, nv, b, s);
}

}  // namespace hc
