// C-ABI entry points: argument validation, error capture, allocation.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>

#include "hc_internal.h"

namespace hc {

void fail(hc_status st, const std::string& msg) { throw Error{st, msg}; }

void* Alloc::get(size_t bytes) const {
    void* p = nullptr;
    if (alloc) {
        p = alloc(bytes, user);
        if (!p) fail(HC_ERR_OOM, "allocator refused " + std::to_string(bytes) + " bytes");
        return p;
    }
    hipError_t e = hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        fail(HC_ERR_OOM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void Alloc::put(void* p) const {
    if (!p) return;
    if (free_) free_(p, user);
    else (void)hipFreeAsync(p, stream);
}

}  // namespace hc

namespace {

template <class F>
hc_status guarded(hc_ctx* ctx, F&& f) {
    try {
        if (ctx) {
            ctx->err.clear();
            HC_HIP(hipSetDevice(ctx->device));
        }
        f();
        return HC_OK;
    } catch (const hc::Error& e) {
        if (ctx) ctx->err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->err = "host allocation failed";
        return HC_ERR_OOM;
    } catch (const std::exception& e) {
        if (ctx) ctx->err = e.what();
        return HC_ERR_DEVICE;
    } catch (...) {
        if (ctx) ctx->err = "unknown error";
        return HC_ERR_DEVICE;
    }
}

// Flags each entry point takes; any other bit is rejected.
constexpr uint32_t kJoinFlags = HC_NO_REWRITE | HC_FORCE_MERGE | HC_FORCE_GALLOP | HC_SEARCH_MASK;
constexpr uint32_t kShareFlags = HC_NO_REWRITE | HC_KEEP_ORDER | HC_JOINT_SEARCH | HC_PESSIMISTIC | HC_CACHE_SHARES;

void check_flags(uint32_t flags, uint32_t allowed, const char* call) {
    HC_REQUIRE((flags & ~allowed) == 0, HC_ERR_INVALID,
               std::string(call) + ": unknown flag bits 0x" + [&] {
                   char b[16];
                   std::snprintf(b, sizeof(b), "%x", flags & ~allowed);
                   return std::string(b);
               }());
}

void check_query_ptrs(const hc_query* q) {
    HC_REQUIRE(q != nullptr, HC_ERR_INVALID, "query is NULL");
    HC_REQUIRE(q->n_vars >= 1 && q->n_vars <= hc::kMaxVars, HC_ERR_INVALID, "n_vars must be 1..8");
    HC_REQUIRE(q->n_atoms >= 1 && q->n_atoms <= hc::kMaxAtoms, HC_ERR_INVALID, "n_atoms must be 1..16");
    HC_REQUIRE(q->atom_arity && q->atom_vars, HC_ERR_INVALID, "query arrays are NULL");
    HC_REQUIRE((q->var_lo == nullptr) == (q->var_hi == nullptr), HC_ERR_INVALID, "var_lo/var_hi: both or neither");
}

}  // namespace

extern "C" {

hc_status hc_ctx_create(int device, void* hip_stream, hc_alloc_fn alloc, hc_free_fn free_, void* user,
                        hc_ctx** out) {
    if (!out) return HC_ERR_INVALID;
    *out = nullptr;
    if ((alloc == nullptr) != (free_ == nullptr)) return HC_ERR_INVALID;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return HC_ERR_DEVICE;
    if (device < 0 || device >= n) return HC_ERR_INVALID;
    hc_ctx* c = new (std::nothrow) hc_ctx();
    if (!c) return HC_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->alloc.alloc = alloc;
    c->alloc.free_ = free_;
    c->alloc.user = user;
    c->alloc.stream = c->stream;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return HC_ERR_DEVICE;
    }
    c->num_cus = prop.multiProcessorCount;
    // The cancel word lives in coherent pinned host memory: the host sets it with a
    // plain store while kernels run (no stream operation that would queue behind them).
    if (hipHostMalloc((void**)&c->h_cancel, sizeof(int), hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->d_cancel, c->h_cancel, 0) != hipSuccess) {
        (void)hipGetLastError();
        hc_ctx_destroy(c);
        return HC_ERR_DEVICE;
    }
    __atomic_store_n(c->h_cancel, 0, __ATOMIC_SEQ_CST);
    // the device address of this device's scratch array (hc_join_count_noalloc)
    try {
        hc::scratch_setup(device);
    } catch (const hc::Error& e) {
        hc_ctx_destroy(c);
        return e.st;
    }
    *out = c;
    return HC_OK;
}

void hc_ctx_destroy(hc_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->h_cancel) (void)hipHostFree(ctx->h_cancel);
    delete ctx;
}

hc_status hc_ctx_cancel(hc_ctx* ctx, int32_t on) {
    if (!ctx) return HC_ERR_INVALID;
    ctx->cancel.store(on ? 1 : 0);
    __atomic_store_n(ctx->h_cancel, on ? 1 : 0, __ATOMIC_SEQ_CST);
    return HC_OK;
}

const char* hc_last_error(const hc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static hc_status build_any(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity, hc_dtype dtype,
                           const int32_t* col_order, int32_t key_bits, int32_t mix_bits, uint64_t mix_seed,
                           uint32_t flags, hc_coco** out);

hc_status hc_build_coco(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity, hc_dtype dtype,
                        const int32_t* col_order, int32_t key_bits, uint64_t mix_seed, uint32_t flags,
                        hc_coco** out) {
    return build_any(ctx, tuples, n, arity, dtype, col_order, key_bits, 0, mix_seed, flags, out);
}

hc_status hc_build_coco_segmented(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity, hc_dtype dtype,
                                  const int32_t* col_order, int32_t mix_bits, int32_t segment_bits,
                                  uint64_t mix_seed, uint32_t flags, hc_coco** out) {
    if (!ctx) return HC_ERR_INVALID;
    if (mix_bits < 1 || segment_bits < 0 || mix_bits + segment_bits > 32) {
        ctx->err = "hc_build_coco_segmented: need mix_bits >= 1, segment_bits >= 0, sum <= 32";
        return HC_ERR_INVALID;
    }
    return build_any(ctx, tuples, n, arity, dtype, col_order, mix_bits + segment_bits, mix_bits, mix_seed, flags,
                     out);
}

static hc_status build_any(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity, hc_dtype dtype,
                           const int32_t* col_order, int32_t key_bits, int32_t mix_bits, uint64_t mix_seed,
                           uint32_t flags, hc_coco** out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        HC_REQUIRE(out != nullptr, HC_ERR_INVALID, "out is NULL");
        *out = nullptr;
        HC_REQUIRE(arity >= 1 && arity <= 4, HC_ERR_INVALID, "arity must be 1..4");
        HC_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), HC_ERR_INVALID, "n must be in [0, 2^31)");
        HC_REQUIRE(n == 0 || tuples != nullptr, HC_ERR_INVALID, "tuples is NULL");
        HC_REQUIRE(dtype == HC_I32 || dtype == HC_I64, HC_ERR_INVALID, "bad dtype");
        HC_REQUIRE(col_order != nullptr, HC_ERR_INVALID, "col_order is NULL");
        HC_REQUIRE(key_bits >= 0 && key_bits <= 32, HC_ERR_INVALID, "key_bits must be 0..32");
        HC_REQUIRE((flags & ~HC_BUILD_SYMMETRIC) == 0, HC_ERR_INVALID, "unknown build flag");
        int seen[4] = {0, 0, 0, 0};
        for (int c = 0; c < arity; ++c) {
            HC_REQUIRE(col_order[c] >= 0 && col_order[c] < arity && !seen[col_order[c]], HC_ERR_INVALID,
                       "col_order must be a permutation of 0..arity-1");
            seen[col_order[c]] = 1;
        }
        hc_coco* c = new hc_coco();
        try {
            hc::build_coco(ctx, tuples, n, arity, dtype, col_order, key_bits, mix_bits, mix_seed, flags, c);
        } catch (...) {
            hc_coco_free(c);
            throw;
        }
        *out = c;
    });
}

void hc_coco_free(hc_coco* c) {
    if (!c) return;
    for (int r = 0; r < 4; ++r) {
        c->alloc.put(c->V[r]);
        c->alloc.put(c->O[r]);
    }
    delete c;
}

hc_status hc_coco_get_info(const hc_coco* c, hc_coco_info* info) {
    if (!c || !info) return HC_ERR_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->n_input = c->n_input;
    info->n_unique = c->n_unique;
    info->arity = c->arity;
    info->key_bits = c->key_bits;
    info->mix_bits = c->mix_bits;
    info->mix_seed = c->mix_seed;
    for (int r = 0; r < 4; ++r) {
        info->col_order[r] = c->col_order[r];
        info->level_len[r] = c->level_len[r];
        info->max_children[r] = c->max_children[r];
        info->distinct[r] = c->distinct[r];
    }
    info->symmetric = c->symmetric;
    info->dtype = c->dtype;
    info->bytes = c->bytes;
    return HC_OK;
}

hc_status hc_coco_copy_level(hc_ctx* ctx, const hc_coco* c, int32_t level, uint32_t* values_host,
                             int32_t* offsets_host) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        HC_REQUIRE(c != nullptr, HC_ERR_INVALID, "coco is NULL");
        HC_REQUIRE(level >= 0 && level < c->arity, HC_ERR_INVALID, "level out of range");
        const int64_t l = c->level_len[level];
        if (values_host && l > 0)
            HC_HIP(hipMemcpyAsync(values_host, c->V[level], sizeof(uint32_t) * l, hipMemcpyDeviceToHost, ctx->stream));
        if (offsets_host && level + 1 < c->arity)
            HC_HIP(hipMemcpyAsync(offsets_host, c->O[level], sizeof(int32_t) * (l + 1), hipMemcpyDeviceToHost,
                                  ctx->stream));
        HC_HIP(hipStreamSynchronize(ctx->stream));
    });
}

hc_status hc_partition_sizes(hc_ctx* ctx, const hc_coco* c, const int32_t* log2_shares, int64_t* B_host,
                             int64_t* Bpref_host) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        HC_REQUIRE(c && log2_shares && B_host && Bpref_host, HC_ERR_INVALID, "NULL argument");
        hc::partition_sizes(ctx, c, log2_shares, B_host, Bpref_host);
    });
}

static std::vector<hc::AtomStats> stats_of_info(const hc_query* q, const hc_coco_info* infos) {
    std::vector<hc::AtomStats> st((size_t)q->n_atoms);
    for (int j = 0; j < q->n_atoms; ++j) {
        HC_REQUIRE(infos[j].arity == q->atom_arity[j], HC_ERR_INVALID, "info arity does not match its atom");
        st[j].rows = (double)infos[j].n_unique;
        st[j].arity = infos[j].arity;
        st[j].dom_bits = infos[j].key_bits;
        for (int k = 0; k < 4; ++k) {
            st[j].distinct[k] = (double)infos[j].distinct[k];
            st[j].maxdeg[k] = (double)infos[j].max_children[k];
        }
    }
    return st;
}

static std::vector<hc::AtomStats> stats_of(const hc_query* q, const hc_coco* const* atoms) {
    std::vector<hc::AtomStats> st((size_t)q->n_atoms);
    for (int j = 0; j < q->n_atoms; ++j) {
        HC_REQUIRE(atoms[j] != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        const hc_coco* c = atoms[j];
        HC_REQUIRE(c->arity == q->atom_arity[j], HC_ERR_INVALID, "CoCo arity does not match its atom");
        st[j].rows = (double)c->n_unique;
        st[j].arity = c->arity;
        st[j].dom_bits = c->key_bits;
        for (int k = 0; k < 4; ++k) {
            st[j].distinct[k] = (double)c->distinct[k];
            st[j].maxdeg[k] = (double)c->max_children[k];
        }
    }
    return st;
}

hc_status hc_compute_shares(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                            int32_t log2_total_P, uint32_t flags, int32_t* var_order_inout,
                            int32_t* log2_shares_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order_inout && log2_shares_out, HC_ERR_INVALID, "NULL argument");
        HC_REQUIRE(log2_total_P >= 0 && log2_total_P <= 24, HC_ERR_INVALID, "log2_total_P must be 0..24");
        check_flags(flags, kShareFlags, "hc_compute_shares");
        hc::validate_query(q, 4);
        auto st = stats_of(q, atom_index);
        hc::choose_shares(q, st, log2_total_P, flags, var_order_inout, log2_shares_out);
    });
}

hc_status hc_compute_shares_from_info(const hc_query* q, const hc_coco_info* infos, int32_t log2_total_P,
                                      uint32_t flags, int32_t* var_order_inout, int32_t* log2_shares_out) {
    try {
        check_query_ptrs(q);
        HC_REQUIRE(infos && var_order_inout && log2_shares_out, HC_ERR_INVALID, "NULL argument");
        HC_REQUIRE(log2_total_P >= 0 && log2_total_P <= 24, HC_ERR_INVALID, "log2_total_P must be 0..24");
        check_flags(flags, kShareFlags, "hc_compute_shares_from_info");
        hc::validate_query(q, 4);
        hc::choose_shares(q, stats_of_info(q, infos), log2_total_P, flags, var_order_inout, log2_shares_out);
        return HC_OK;
    } catch (const hc::Error& e) {
        return e.st;
    } catch (...) {
        return HC_ERR_INVALID;
    }
}

hc_status hc_plan_cost_from_info(const hc_query* q, const hc_coco_info* infos, const int32_t* var_order,
                                 const int32_t* log2_shares, uint32_t flags, double* per_level_out,
                                 double* total_out) {
    try {
        check_query_ptrs(q);
        HC_REQUIRE(infos && var_order && total_out, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, HC_NO_REWRITE | HC_PESSIMISTIC, "hc_plan_cost_from_info");
        *total_out = hc::plan_cost(q, stats_of_info(q, infos), var_order, log2_shares, flags, per_level_out);
        return HC_OK;
    } catch (const hc::Error& e) {
        return e.st;
    } catch (...) {
        return HC_ERR_INVALID;
    }
}

hc_status hc_join_count(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                        const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                        uint64_t* count_out, uint64_t* digest_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && count_out, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, kJoinFlags, "hc_join_count");
        // A count without shares whose first variable is restricted to a narrow id
        // range is a batch of one request: its first level then searches the
        // range's mixed ids instead of walking the whole top level.
        if (!digest_out && q->var_lo && q->n_vars > 1 && atom_index[0]) {
            bool no_shares = true;
            for (int v = 0; v < q->n_vars && log2_shares; ++v) no_shares = no_shares && log2_shares[v] == 0;
            const int v0 = var_order[0];
            const hc_coco* c0 = atom_index[0];
            const bool v0_ok = v0 >= 0 && v0 < q->n_vars;
            const int64_t lo = v0_ok ? std::max<int64_t>(q->var_lo[v0], 0) : 0, hi = v0_ok ? q->var_hi[v0] : 0;
            const bool one_segment = c0->key_bits == c0->mix_bits || hi <= lo ||
                                     (lo >> c0->mix_bits) == ((hi - 1) >> c0->mix_bits);
            if (no_shares && v0_ok && hi - lo <= ((int64_t)1 << 16) && one_segment) {
                const int64_t rng[2] = {lo, hi};
                uint64_t per = 0, total = 0;
                hc::join_run(ctx, q, atom_index, var_order, nullptr, flags, false, &total, nullptr, nullptr, 0,
                             nullptr, &per, 1, rng);
                *count_out = per;
                return;
            }
        }
        // small joins: the device-sized sequence, no read-back between the levels
        if (!digest_out && hc::join_small_device_sized(ctx, q, atom_index, var_order, log2_shares, flags, -1, nullptr,
                                                       0, count_out, nullptr, nullptr))
            return;
        hc::join_run(ctx, q, atom_index, var_order, log2_shares, flags, false, count_out, digest_out, nullptr, 0,
                     nullptr);
    });
}

hc_status hc_join_count_noalloc(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                                uint64_t* count_out, uint64_t* digest_out, uint64_t* scratch_used) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && count_out, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, kJoinFlags, "hc_join_count_noalloc");
        for (int j = 0; j < q->n_atoms; ++j) HC_REQUIRE(atom_index[j] != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        // the largest chunking cap whose workspace bound fits the array (smaller caps
        // split the frontiers into more, smaller chunks)
        int64_t cap = hc::kDefaultCap;
        uint64_t need = 0;
        for (;; cap >>= 2) {
            need = hc::join_workspace_bound(q, atom_index, var_order, log2_shares, flags, 0, 0, cap, false);
            if (need <= hc::scratch_bytes() || cap <= ((int64_t)1 << 12)) break;
        }
        HC_REQUIRE(need <= hc::scratch_bytes(), HC_ERR_UNSUPPORTED,
                   "hc_join_count_noalloc: the call may need " + std::to_string(need) +
                       " bytes of device scratch even in chunks of " + std::to_string(cap) +
                       " entries, more than the fixed " + std::to_string(hc::scratch_bytes()) +
                       " bytes it has; use hc_join_count");
        void* base = hc::scratch_ptr(ctx->device);
        HC_REQUIRE(base != nullptr, HC_ERR_DEVICE, "scratch array of this device was not set up");
        hc::ScratchArena arena(base, hc::scratch_bytes());
        hc::Alloc a;
        a.alloc = hc::ScratchArena::alloc_cb;
        a.free_ = hc::ScratchArena::free_cb;
        a.user = &arena;
        a.stream = ctx->stream;
        // no timing events either: profiling is off for this call
        const int prof = ctx->profiling;
        ctx->profiling = 0;
        try {
            hc::join_run(ctx, q, atom_index, var_order, log2_shares, flags, false, count_out, digest_out, nullptr, 0,
                         nullptr, nullptr, 0, nullptr, &a, cap);
        } catch (...) {
            ctx->profiling = prof;
            HC_HIP(hipStreamSynchronize(ctx->stream));   // nothing may still use the arena's ranges
            throw;
        }
        ctx->profiling = prof;
        if (scratch_used) *scratch_used = arena.high_water();
    });
}

hc_status hc_join_count_cells(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                              const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                              uint64_t* cell_counts, uint64_t* count_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && cell_counts && count_out, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, kJoinFlags, "hc_join_count_cells");
        if (hc::join_small_device_sized(ctx, q, atom_index, var_order, log2_shares, flags, 0, nullptr, 0, count_out,
                                        cell_counts, nullptr))
            return;
        hc::join_run(ctx, q, atom_index, var_order, log2_shares, flags, false, count_out, nullptr, nullptr, 0,
                     nullptr, cell_counts);
    });
}

hc_status hc_join_count_segments(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                 const int32_t* var_order, int32_t log2_extra, uint32_t flags,
                                 uint64_t* segment_counts, uint64_t* count_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && segment_counts && count_out, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, kJoinFlags, "hc_join_count_segments");
        HC_REQUIRE(atom_index[0] != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        const int seg = atom_index[0]->key_bits - atom_index[0]->mix_bits;
        HC_REQUIRE(seg >= 1, HC_ERR_INVALID, "hc_join_count_segments needs segmented CoCos");
        HC_REQUIRE(log2_extra >= 0 && seg + log2_extra <= 24, HC_ERR_INVALID, "log2_extra out of range");
        HC_REQUIRE(var_order[0] >= 0 && var_order[0] < q->n_vars, HC_ERR_INVALID, "bad var_order");
        std::vector<int32_t> shares((size_t)q->n_vars, 0);
        shares[(size_t)var_order[0]] = seg + log2_extra;
        // the cell id is the first variable's coordinate (segment above the extra split)
        if (hc::join_small_device_sized(ctx, q, atom_index, var_order, shares.data(), flags, log2_extra, nullptr, 0,
                                        count_out, segment_counts, nullptr))
            return;
        hc::join_run(ctx, q, atom_index, var_order, shares.data(), flags, false, count_out, nullptr, nullptr, 0,
                     nullptr, segment_counts, 0, nullptr, nullptr, 0, log2_extra);
    });
}

hc_status hc_join_workspace_bound(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                  const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                                  int64_t n_queries, int64_t first_width, uint64_t* bytes_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && bytes_out, HC_ERR_INVALID, "NULL argument");
        HC_REQUIRE(n_queries >= 0 && first_width >= 0, HC_ERR_INVALID, "negative n_queries or first_width");
        check_flags(flags, kJoinFlags, "hc_join_workspace_bound");
        for (int j = 0; j < q->n_atoms; ++j) HC_REQUIRE(atom_index[j] != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        *bytes_out = hc::join_workspace_bound(q, atom_index, var_order, log2_shares, flags, n_queries, first_width);
    });
}

hc_status hc_join_count_multi(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                              const int32_t* var_order, uint32_t flags, int64_t n_queries,
                              const int64_t* first_var_ranges, uint64_t* counts_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && first_var_ranges && counts_out, HC_ERR_INVALID, "NULL argument");
        HC_REQUIRE(n_queries >= 0, HC_ERR_INVALID, "negative n_queries");
        check_flags(flags, kJoinFlags, "hc_join_count_multi");
        if (n_queries == 0) return;
        uint64_t total = 0;
        hc::join_run(ctx, q, atom_index, var_order, nullptr, flags, false, &total, nullptr, nullptr, 0, nullptr,
                     counts_out, n_queries, first_var_ranges);
    });
}

hc_status hc_join_emit(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                       const int32_t* var_order, const int32_t* log2_shares, uint32_t flags, void* out,
                       int64_t capacity, int64_t* n_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && n_out, HC_ERR_INVALID, "NULL argument");
        HC_REQUIRE(capacity >= 0, HC_ERR_INVALID, "capacity must be >= 0");
        HC_REQUIRE(capacity == 0 || out != nullptr, HC_ERR_INVALID, "out is NULL");
        check_flags(flags, kJoinFlags | HC_EMIT_SORTED, "hc_join_emit");
        uint64_t count = 0;
        if (!(out != nullptr && hc::join_small_device_sized(ctx, q, atom_index, var_order, log2_shares,
                                                             flags & ~HC_EMIT_SORTED, -1, out, capacity, &count,
                                                             nullptr, n_out)))
            hc::join_run(ctx, q, atom_index, var_order, log2_shares, flags & ~HC_EMIT_SORTED, true, &count, nullptr,
                         out, capacity, n_out);
        *n_out = (int64_t)count;
        if ((int64_t)count > capacity)
            hc::fail(HC_ERR_OVERFLOW, "hc_join_emit: " + std::to_string(count) + " rows exceed capacity " +
                                          std::to_string(capacity));
        if ((flags & HC_EMIT_SORTED) && count > 1) {
            // rows of raw ids below 2^key_bits (the build rejects larger ids)
            const hc_coco* c0 = atom_index[0];
            hc::sort_rows(ctx->alloc, out, (int64_t)count, q->n_vars, c0->key_bits, c0->dtype == HC_I64,
                          ctx->stream);
            HC_HIP(hipStreamSynchronize(ctx->stream));
        }
    });
}

hc_status hc_join_graph_create(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                               const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                               int32_t cell_group, void* out, int64_t capacity, int64_t frontier_cap,
                               int64_t item_cap, hc_join_graph** graph_out) {
    if (!ctx) return HC_ERR_INVALID;
    return guarded(ctx, [&] {
        check_query_ptrs(q);
        HC_REQUIRE(atom_index && var_order && graph_out, HC_ERR_INVALID, "NULL argument");
        *graph_out = nullptr;
        check_flags(flags, kJoinFlags, "hc_join_graph_create");
        HC_REQUIRE((flags & ~HC_NO_REWRITE) == 0, HC_ERR_UNSUPPORTED, "captured joins use the default search");
        HC_REQUIRE(capacity >= 0 && frontier_cap >= 0 && item_cap >= 0, HC_ERR_INVALID, "negative capacity");
        HC_REQUIRE(out != nullptr || capacity == 0, HC_ERR_INVALID, "capacity without out");
        for (int j = 0; j < q->n_atoms; ++j) HC_REQUIRE(atom_index[j] != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        *graph_out = hc::join_graph_create(ctx, q, atom_index, var_order, log2_shares, flags, cell_group, out, capacity,
                                           frontier_cap, item_cap);
    });
}

hc_status hc_join_graph_launch(hc_join_graph* g) {
    if (!g) return HC_ERR_INVALID;
    hc_ctx* ctx = hc::join_graph_ctx(g);
    return guarded(ctx, [&] { hc::join_graph_launch(g); });
}

hc_status hc_join_graph_result(hc_join_graph* g, uint64_t* count_out, uint64_t* cell_counts, int64_t* n_out,
                               int32_t* replayed) {
    if (!g || !count_out) return HC_ERR_INVALID;
    hc_ctx* ctx = hc::join_graph_ctx(g);
    int64_t no = 0;
    const hc_status st = guarded(ctx, [&] { hc::join_graph_result(g, count_out, cell_counts, &no, replayed); });
    if (n_out) *n_out = no;
    return st;
}

void hc_join_graph_destroy(hc_join_graph* g) { hc::join_graph_destroy(g); }

hc_status hc_plan_describe(const hc_query* q, const int32_t* var_order, uint32_t flags, char* buf, size_t cap) {
    try {
        check_query_ptrs(q);
        HC_REQUIRE(var_order && buf, HC_ERR_INVALID, "NULL argument");
        check_flags(flags, HC_NO_REWRITE, "hc_plan_describe");
        hc::Plan p = hc::compile_plan(q, var_order, !(flags & HC_NO_REWRITE));
        std::string s = hc::describe_plan(p);
        if (s.size() + 1 > cap) return HC_ERR_OVERFLOW;
        std::memcpy(buf, s.c_str(), s.size() + 1);
        return HC_OK;
    } catch (const hc::Error& e) {
        return e.st;
    } catch (...) {
        return HC_ERR_INVALID;
    }
}

hc_status hc_ctx_set_grid_limit(hc_ctx* ctx, int32_t max_workgroups) {
    if (!ctx || max_workgroups < 0) return HC_ERR_INVALID;
    ctx->grid_limit = max_workgroups;
    return HC_OK;
}

hc_status hc_ctx_set_profiling(hc_ctx* ctx, int on) {
    if (!ctx) return HC_ERR_INVALID;
    ctx->profiling = on ? 1 : 0;
    return HC_OK;
}

hc_status hc_ctx_get_timing(const hc_ctx* ctx, hc_timing* t) {
    if (!ctx || !t) return HC_ERR_INVALID;
    *t = ctx->timing;
    return HC_OK;
}

}  // extern "C"
