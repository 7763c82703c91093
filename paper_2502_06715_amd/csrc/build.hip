// CoCo construction (Section 4, "Compressed Column layout").
//
// A relation R(X_1..X_k) is turned into k levels.  Level r lists, once per
// distinct prefix (x_1..x_{r+1}) in sorted order, the value x_{r+1} (V_r), and
// where that entry's children start in level r+1 (O_r, l_r + 1 entries; the
// last entry closes the last range).  The relation is a set, so the deepest
// level keeps no offsets.
//
// The paper builds the levels with two scans over the sorted rows (count the
// distinct prefixes, then fill top-down using the first differing column of
// adjacent rows).  Here the same quantities come from data-parallel steps:
//   1. pack: each row becomes one u64 key, the mixed values H_b(x) of its
//      columns in level order, b bits each (so sorting the keys is the
//      lexicographic sort of the mixed rows);
//   2. LSD radix sort of the keys (prim.hip);
//   3. flags: row i opens a new level-r entry iff its key differs from row
//      i-1 and its (r+1)-column prefix differs too; an exclusive scan of the
//      flags gives every new entry its index (two levels per u64 scan);
//   4. scatter: V_r[index] = column r of the row, O_r[index] = the index the
//      same row gets in level r+1.
#include "prim_dev.h"

namespace hc {

Mixer make_mixer(int b, uint64_t seed, int kb) {
    Mixer m{};
    m.b = b;
    m.kb = kb;
    m.kmask = kb >= 32 ? 0xFFFFFFFFu : ((1u << kb) - 1u);
    m.mask = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    m.seed = (uint32_t)seed & m.mask;
    const uint32_t h = (uint32_t)(b + 1) / 2;
    m.s1 = h;
    m.s2 = h > 1 ? h - 1 : 1;
    m.s3 = h;
    m.c1 = 0x7FEB352Du & m.mask;
    m.c2 = 0x846CA68Bu & m.mask;
    auto inv = [](uint32_t c) {   // inverse of an odd number modulo 2^32 (Newton iteration)
        uint32_t x = c;
        for (int k = 0; k < 5; ++k) x *= 2u - c * x;
        return x;
    };
    m.c1inv = inv(0x7FEB352Du) & m.mask;
    m.c2inv = inv(0x846CA68Bu) & m.mask;
    return m;
}

struct ColOrder {
    int32_t c[4];
};

template <class T>
__global__ void k_max_id(const T* __restrict__ t, int64_t count, unsigned long long* mx, int* bad) {
    unsigned long long local = 0;
    int neg = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = t[i];
        if (v < 0) neg = 1;
        else if ((unsigned long long)v > local) local = (unsigned long long)v;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned long long o = __shfl_xor(local, d, 64);
        local = o > local ? o : local;
        neg |= __shfl_xor(neg, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(mx, local);
        if (neg) atomicOr(bad, 1);
    }
}

template <class T>
__global__ void k_pack(const T* __restrict__ t, int64_t n, int arity, ColOrder co, Mixer m,
                       uint64_t* __restrict__ keys, int* bad) {
    int err = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key = 0;
        for (int c = 0; c < arity; ++c) {
            const T v = t[i * arity + co.c[c]];
            if (v < 0 || (unsigned long long)v > (unsigned long long)m.kmask) err = 1;
            key = (key << m.kb) | mix_key((uint32_t)v, m);
        }
        keys[i] = key;
    }
    if (err) atomicOr(bad, 1);
}

// Flags of row i: bit r set iff row i opens a new entry of level r.
__device__ inline uint32_t level_flags(const uint64_t* K, int64_t i, int arity, int b) {
    const uint32_t all = (1u << arity) - 1u;
    if (i == 0) return all;
    const uint64_t k = K[i], p = K[i - 1];
    if (k == p) return 0;
    uint32_t f = 0;
    for (int r = 0; r < arity; ++r) {
        const int sh = (arity - 1 - r) * b;
        if ((k >> sh) != (p >> sh)) f |= 1u << r;
    }
    return f;
}

struct LoadLevelPair {
    const uint64_t* K;
    int arity, b, pair;
    __device__ uint64_t operator()(int64_t i) const {
        const uint32_t f = level_flags(K, i, arity, b);
        const uint64_t lo = (f >> (2 * pair)) & 1u;
        const uint64_t hi = (f >> (2 * pair + 1)) & 1u;
        return lo | (hi << 32);
    }
};

struct LevelPtrs {
    uint32_t* V[4];
    int32_t* O[4];
};

__device__ inline uint32_t pos_of(const uint64_t* P0, const uint64_t* P1, int64_t i, int r) {
    const uint64_t p = r < 2 ? P0[i] : P1[i];
    return (r & 1) ? (uint32_t)(p >> 32) : (uint32_t)p;
}

__global__ void k_coco_scatter(const uint64_t* __restrict__ K, int64_t n, int arity, int b,
                               const uint64_t* __restrict__ P0, const uint64_t* __restrict__ P1, LevelPtrs L) {
    const uint64_t mask = b >= 32 ? 0xFFFFFFFFull : ((1ull << b) - 1ull);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t f = level_flags(K, i, arity, b);
        if (!f) continue;
        const uint64_t k = K[i];
        for (int r = 0; r < arity; ++r) {
            if (!((f >> r) & 1u)) continue;
            const uint32_t pr = pos_of(P0, P1, i, r);
            L.V[r][pr] = (uint32_t)((k >> ((arity - 1 - r) * b)) & mask);
            if (r + 1 < arity) L.O[r][pr] = (int32_t)pos_of(P0, P1, i, r + 1);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int r = 0; r + 1 < arity; ++r) {
            const uint32_t lr = pos_of(P0, P1, n, r), lr1 = pos_of(P0, P1, n, r + 1);
            L.O[r][lr] = (int32_t)lr1;
        }
    }
}

// Largest child list: a maximum per block, then one atomic per block (one address
// takes every atomic, so there are few).
__global__ void k_max_children(const int32_t* __restrict__ O, int64_t l, unsigned long long* out) {
    __shared__ unsigned long long wmax[kWaves];
    unsigned long long local = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = (unsigned long long)(O[e + 1] - O[e]);
        local = d > local ? d : local;
    }
    for (int dd = 32; dd >= 1; dd >>= 1) {
        unsigned long long o = __shfl_xor(local, dd, 64);
        local = o > local ? o : local;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) local = wmax[w] > local ? wmax[w] : local;
        atomicMax(out, local);
    }
}

// Distinct values of a level with wide keys: one bit per value.
__global__ void k_bitmap_mark(const uint32_t* __restrict__ V, int64_t l, uint32_t* bitmap) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = V[e];
        const uint32_t bit = 1u << (v & 31u);
        // most values repeat: test first, so that only the first few setters of a bit
        // contend for its word (a stale read only costs one redundant atomic)
        if (!(__atomic_load_n(&bitmap[v >> 5], __ATOMIC_RELAXED) & bit)) atomicOr(&bitmap[v >> 5], bit);
    }
}

// Distinct values of a level: one byte flag per value, set by plain stores (setting
// a flag twice is harmless, so no atomics and no test read), then counted.
__global__ void k_flag_mark(const uint32_t* __restrict__ V, int64_t l, uint8_t* __restrict__ flags) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x)
        flags[V[e]] = 1;
}

// Adds the set flags of words[0 .. n) (byte flags of 0 or 1, or bitmap bits) to *out.
__global__ void k_flag_count(const uint32_t* __restrict__ words, int64_t n, unsigned long long* out) {
    __shared__ unsigned long long wsum[kWaves];
    unsigned long long local = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        local += (unsigned long long)__popc(words[e]);
    local = wave_sum(local);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) local += wsum[w];
        atomicAdd(out, local);
    }
}

// Symmetry check of a binary relation: every key (x, y) must have (y, x).
__global__ void k_check_symmetric(const uint64_t* __restrict__ K, int64_t n, int b, int* bad) {
    const uint64_t mask = b >= 32 ? 0xFFFFFFFFull : ((1ull << b) - 1ull);
    int err = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = K[i];
        const uint64_t t = ((k & mask) << b) | (k >> b);
        const int64_t p = lower_bound_u64key(K, 0, n, t);
        if (p >= n || K[p] != t) err = 1;
    }
    if (err) atomicOr(bad, 1);
}

static unsigned grid_for(int64_t n, int cap = 8192) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void build_coco(hc_ctx* ctx, const void* tuples, int64_t n, int arity, hc_dtype dtype,
                const int32_t* col_order, int key_bits, int mix_bits, uint64_t seed, uint32_t flags,
                hc_coco* out) {
    const Alloc& A = ctx->alloc;
    hipStream_t s = ctx->stream;
    ColOrder co{};
    for (int c = 0; c < 4; ++c) co.c[c] = c < arity ? col_order[c] : 0;

    DevBuf<unsigned long long> scal(A, 8);   // [0] max id, [1] max children, [2] popcount
    DevBuf<int> bad(A, 2);
    HC_HIP(hipMemsetAsync(scal.p, 0, sizeof(unsigned long long) * 8, s));
    HC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int) * 2, s));

    int b = key_bits;
    if (n > 0 && b == 0) {
        if (dtype == HC_I32)
            k_max_id<int32_t><<<grid_for(n * arity), kBlock, 0, s>>>((const int32_t*)tuples, n * arity, scal.p, bad.p);
        else
            k_max_id<int64_t><<<grid_for(n * arity), kBlock, 0, s>>>((const int64_t*)tuples, n * arity, scal.p, bad.p);
        HC_HIP(hipGetLastError());
        unsigned long long mx = 0;
        int badh = 0;
        HC_HIP(hipMemcpyAsync(&mx, scal.p, sizeof(mx), hipMemcpyDeviceToHost, s));
        HC_HIP(hipMemcpyAsync(&badh, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HC_HIP(hipStreamSynchronize(s));
        HC_REQUIRE(!badh, HC_ERR_INVALID, "hc_build_coco: negative id");
        HC_REQUIRE(mx <= 0xFFFFFFFFull, HC_ERR_UNSUPPORTED, "hc_build_coco: ids must be below 2^32");
        b = 1;
        while (b < 32 && (mx >> b) != 0) ++b;
    }
    if (b == 0) b = 1;
    HC_REQUIRE(b >= 1 && b <= 32, HC_ERR_INVALID, "hc_build_coco: key_bits must be 0..32");
    HC_REQUIRE(arity * b <= 64, HC_ERR_UNSUPPORTED, "hc_build_coco: arity * key_bits must be <= 64");
    const int mb = mix_bits > 0 ? mix_bits : b;
    HC_REQUIRE(mb >= 1 && mb <= b, HC_ERR_INVALID, "hc_build_coco: mixed bits must be 1..key_bits");
    const Mixer mx = make_mixer(mb, seed, b);
    out->mix_bits = mb;

    out->arity = arity;
    out->key_bits = b;
    out->mix_seed = seed;
    for (int c = 0; c < 4; ++c) out->col_order[c] = c < arity ? col_order[c] : c;
    out->dtype = dtype;
    out->n_input = n;

    DevBuf<uint64_t> keys(A, (size_t)n + 1), tmp(A, (size_t)n + 1);
    if (n > 0) {
        if (dtype == HC_I32)
            k_pack<int32_t><<<grid_for(n), kBlock, 0, s>>>((const int32_t*)tuples, n, arity, co, mx, keys.p, bad.p);
        else
            k_pack<int64_t><<<grid_for(n), kBlock, 0, s>>>((const int64_t*)tuples, n, arity, co, mx, keys.p, bad.p);
        HC_HIP(hipGetLastError());
        radix_sort_u64(A, keys, tmp, n, arity * b, s);
    }
    // entry indices of every level (two levels per u64 scan)
    DevBuf<uint64_t> P0(A, (size_t)n + 1), P1;
    scan_exclusive(A, LoadLevelPair{keys.p, arity, b, 0}, P0.p, n, s);
    if (arity > 2) {
        P1 = DevBuf<uint64_t>(A, (size_t)n + 1);
        scan_exclusive(A, LoadLevelPair{keys.p, arity, b, 1}, P1.p, n, s);
    }
    uint64_t tot[2] = {0, 0};
    int badh = 0;
    HC_HIP(hipMemcpyAsync(&tot[0], P0.p + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    if (arity > 2) HC_HIP(hipMemcpyAsync(&tot[1], P1.p + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HC_HIP(hipMemcpyAsync(&badh, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HC_HIP(hipStreamSynchronize(s));
    HC_REQUIRE(!badh, HC_ERR_INVALID, "hc_build_coco: id negative or not below 2^key_bits");
    for (int r = 0; r < arity; ++r) {
        const uint64_t p = r < 2 ? tot[0] : tot[1];
        out->level_len[r] = (int64_t)((r & 1) ? (p >> 32) : (p & 0xFFFFFFFFull));
    }
    out->n_unique = out->level_len[arity - 1];
    // allocate the levels (owned by the CoCo)
    out->alloc = A;
    LevelPtrs L{};
    int64_t bytes = 0;
    for (int r = 0; r < arity; ++r) {
        out->V[r] = (uint32_t*)A.get(sizeof(uint32_t) * (size_t)(out->level_len[r] + 1));
        L.V[r] = out->V[r];
        bytes += sizeof(uint32_t) * (out->level_len[r] + 1);
        if (r + 1 < arity) {
            out->O[r] = (int32_t*)A.get(sizeof(int32_t) * (size_t)(out->level_len[r] + 2));
            L.O[r] = out->O[r];
            bytes += sizeof(int32_t) * (out->level_len[r] + 2);
        }
    }
    out->bytes = bytes;
    if (n > 0) {
        k_coco_scatter<<<grid_for(n), kBlock, 0, s>>>(keys.p, n, arity, b, P0.p, arity > 2 ? P1.p : P0.p, L);
        HC_HIP(hipGetLastError());
    } else {
        for (int r = 0; r + 1 < arity; ++r) HC_HIP(hipMemsetAsync(out->O[r], 0, sizeof(int32_t), s));
    }
    // statistics: largest child list per level (scal[1 + r]), distinct values per
    // column (scal[4 + r]), the symmetry check (bad[1]); read back together
    HC_REQUIRE(!(flags & HC_BUILD_SYMMETRIC) || arity == 2, HC_ERR_INVALID,
               "hc_build_coco: HC_BUILD_SYMMETRIC needs a binary relation");
    for (int r = 0; r + 1 < arity; ++r)
        if (out->level_len[r] > 0) {
            k_max_children<<<grid_for(out->level_len[r]), kBlock, 0, s>>>(out->O[r], out->level_len[r], scal.p + 1 + r);
            HC_HIP(hipGetLastError());
        }
    bool counted[4] = {false, false, false, false};
    DevBuf<uint8_t> fl;
    for (int r = 1; r < arity; ++r) {
        // the first level's values are distinct; wide keys get the level length as an
        // upper bound; a symmetric binary relation holds the same values in both
        // columns (the symmetry itself is verified below, failing the build otherwise)
        if (out->level_len[r] == 0 || b > 30 || ((flags & HC_BUILD_SYMMETRIC) && arity == 2)) continue;
        // byte flags (plain stores) up to 2^26 values, a bitmap (atomics) above
        const bool bytes_ = b <= 26;
        const int64_t nfl = bytes_ ? ((int64_t)1 << b) : ((int64_t)1 << b) / 8;
        if (!fl.p) fl = DevBuf<uint8_t>(A, (size_t)nfl + 4);
        HC_HIP(hipMemsetAsync(fl.p, 0, (size_t)nfl + 4, s));
        if (bytes_)
            k_flag_mark<<<grid_for(out->level_len[r]), kBlock, 0, s>>>(out->V[r], out->level_len[r], fl.p);
        else
            k_bitmap_mark<<<grid_for(out->level_len[r]), kBlock, 0, s>>>(out->V[r], out->level_len[r],
                                                                         (uint32_t*)fl.p);
        HC_HIP(hipGetLastError());
        // a set byte flag and a set bitmap bit both count one (popcount of the words)
        k_flag_count<<<grid_for(nfl / 4 + 1), kBlock, 0, s>>>((const uint32_t*)fl.p, nfl / 4 + 1, scal.p + 4 + r);
        HC_HIP(hipGetLastError());
        counted[r] = true;
    }
    if ((flags & HC_BUILD_SYMMETRIC) && n > 0) {
        k_check_symmetric<<<grid_for(n), kBlock, 0, s>>>(keys.p, n, b, bad.p + 1);
        HC_HIP(hipGetLastError());
    }
    unsigned long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int sb[2] = {0, 0};
    HC_HIP(hipMemcpyAsync(st, scal.p, sizeof(st), hipMemcpyDeviceToHost, s));
    HC_HIP(hipMemcpyAsync(sb, bad.p, sizeof(sb), hipMemcpyDeviceToHost, s));
    HC_HIP(hipStreamSynchronize(s));
    for (int r = 0; r + 1 < arity; ++r) out->max_children[r] = (int64_t)st[1 + r];
    for (int r = 0; r < arity; ++r)
        out->distinct[out->col_order[r]] = counted[r] ? (int64_t)st[4 + r] : out->level_len[r];
    if ((flags & HC_BUILD_SYMMETRIC) && arity == 2) out->distinct[out->col_order[1]] = out->level_len[0];
    if (flags & HC_BUILD_SYMMETRIC) {
        HC_REQUIRE(!sb[1], HC_ERR_INVALID, "hc_build_coco: relation is not symmetric");
        out->symmetric = 1;
    }
}

// ---------------------------------------------------------------- partition sizes
struct PartArgs {
    const uint32_t* V[4];
    const int32_t* O[4];
    int64_t len[4];
    int32_t arity, b;
    int32_t shift_of_level[4];   // bit position of the level's column id in the flat cell id
    int32_t k_of_level[4];
};

__global__ void k_partition_hist(PartArgs a, unsigned long long* B) {
    const int64_t nleaf = a.len[a.arity - 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nleaf; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t cell = 0;
        int64_t idx = i;
        for (int r = a.arity - 1; r >= 0; --r) {
            const uint32_t v = a.V[r][idx];
            if (a.k_of_level[r] > 0) cell |= (uint64_t)(v >> (a.b - a.k_of_level[r])) << a.shift_of_level[r];
            if (r > 0) {   // parent: last entry e of level r-1 with O[e] <= idx
                int64_t lo = 0, hi = a.len[r - 1];
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a.O[r - 1][mid] <= idx) lo = mid + 1; else hi = mid;
                }
                idx = lo - 1;
            }
        }
        atomicAdd(&B[cell], 1ull);
    }
}

void partition_sizes(hc_ctx* ctx, const hc_coco* c, const int32_t* log2_shares, int64_t* Bh, int64_t* Bpref) {
    int total = 0;
    for (int col = 0; col < c->arity; ++col) {
        HC_REQUIRE(log2_shares[col] >= 0 && log2_shares[col] <= c->key_bits, HC_ERR_INVALID,
                   "hc_partition_sizes: share exceeds key_bits");
        total += log2_shares[col];
    }
    HC_REQUIRE(total <= 24, HC_ERR_INVALID, "hc_partition_sizes: more than 2^24 partitions");
    PartArgs a{};
    a.arity = c->arity;
    a.b = c->key_bits;
    // flat id: original column 0 most significant
    int shift_of_col[4] = {0, 0, 0, 0};
    int acc = 0;
    for (int col = c->arity - 1; col >= 0; --col) {
        shift_of_col[col] = acc;
        acc += log2_shares[col];
    }
    for (int r = 0; r < c->arity; ++r) {
        a.V[r] = c->V[r];
        a.O[r] = c->O[r];
        a.len[r] = c->level_len[r];
        a.shift_of_level[r] = shift_of_col[c->col_order[r]];
        a.k_of_level[r] = log2_shares[c->col_order[r]];
    }
    const int64_t ncell = (int64_t)1 << total;
    DevBuf<unsigned long long> B(ctx->alloc, (size_t)ncell);
    HC_HIP(hipMemsetAsync(B.p, 0, sizeof(unsigned long long) * ncell, ctx->stream));
    if (c->n_unique > 0) {
        k_partition_hist<<<grid_for(c->n_unique), kBlock, 0, ctx->stream>>>(a, B.p);
        HC_HIP(hipGetLastError());
    }
    std::vector<unsigned long long> h((size_t)ncell);
    HC_HIP(hipMemcpyAsync(h.data(), B.p, sizeof(unsigned long long) * ncell, hipMemcpyDeviceToHost, ctx->stream));
    HC_HIP(hipStreamSynchronize(ctx->stream));
    int64_t run = 0;
    for (int64_t i = 0; i < ncell; ++i) {
        Bh[i] = (int64_t)h[i];
        Bpref[i] = run;   // exclusive: start of partition i in the partitioned array
        run += (int64_t)h[i];
    }
}

}  // namespace hc
