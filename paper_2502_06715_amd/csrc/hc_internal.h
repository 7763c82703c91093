// Internal declarations of the gfx950 Generic Join library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "hc.h"

namespace hc {

// ---------------------------------------------------------------- errors
struct Error {
    hc_status st;
    std::string msg;
};
[[noreturn]] void fail(hc_status st, const std::string& msg);
#define HC_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::hc::fail(HC_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define HC_REQUIRE(cond, st, msg) \
    do {                          \
        if (!(cond)) ::hc::fail((st), (msg)); \
    } while (0)

// ---------------------------------------------------------------- bijective b-bit mixer
// H_b: Wellons' lowbias32 (xorshift, odd multiply, xorshift, odd multiply, xorshift)
// restricted to b-bit words; shifts ceil(b/2), max(1, ceil(b/2)-1), ceil(b/2).
// Keys are kb >= b bits wide: the low b bits are mixed, the kb-b bits above them
// (a segment number, e.g. the query of a batch) pass through unchanged.
struct Mixer {
    uint32_t mask, seed;          // mask of the b mixed bits
    uint32_t s1, s2, s3;
    uint32_t c1, c2, c1inv, c2inv;
    int32_t b;                    // mixed bits
    int32_t kb;                   // key bits
    uint32_t kmask;               // mask of the kb key bits
};
Mixer make_mixer(int b, uint64_t seed, int kb);

__host__ __device__ inline uint32_t mix_key(uint32_t x, const Mixer& m) {
    const uint32_t hi = x & ~m.mask;
    x = (x ^ m.seed) & m.mask;
    x ^= x >> m.s1;
    x = (x * m.c1) & m.mask;
    x ^= x >> m.s2;
    x = (x * m.c2) & m.mask;
    x ^= x >> m.s3;
    return hi | x;
}
__host__ __device__ inline uint32_t unxorshift(uint32_t y, uint32_t s, int b) {
    uint32_t x = y;
    for (int k = (int)s; k < b; k += (int)s) x ^= y >> k;
    return x;
}
__host__ __device__ inline uint32_t unmix_key(uint32_t y, const Mixer& m) {
    const uint32_t hi = y & ~m.mask;
    uint32_t x = unxorshift(y & m.mask, m.s3, m.b);
    x = (x * m.c2inv) & m.mask;
    x = unxorshift(x, m.s2, m.b);
    x = (x * m.c1inv) & m.mask;
    x = unxorshift(x, m.s1, m.b);
    return hi | ((x ^ m.seed) & m.mask);
}

// ---------------------------------------------------------------- memory
struct Alloc {
    hc_alloc_fn alloc = nullptr;
    hc_free_fn free_ = nullptr;
    void* user = nullptr;
    hipStream_t stream = nullptr;
    void* get(size_t bytes) const;
    void put(void* p) const;
};

template <class T>
struct DevBuf {
    const Alloc* a = nullptr;
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const Alloc& al, size_t count) : a(&al), n(count) {
        p = static_cast<T*>(al.get(sizeof(T) * (count ? count : 1)));
    }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : a(o.a), p(o.p), n(o.n) { o.p = nullptr; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        reset();
        a = o.a; p = o.p; n = o.n; o.p = nullptr;
        return *this;
    }
    void reset() {
        if (p && a) a->put(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { reset(); }
};

// First-fit arena over the per-device scratch array (noalloc.hip): hands out
// 256-byte aligned ranges, host-side bookkeeping only.
class ScratchArena {
public:
    ScratchArena(void* base, size_t size);
    void* get(size_t bytes);
    void put(void* p);
    size_t high_water() const { return high_; }
    static void* alloc_cb(size_t bytes, void* user);
    static void free_cb(void* p, void* user);

private:
    struct Range {
        size_t off, len;
    };
    char* base_;
    size_t size_;
    size_t high_ = 0;
    std::vector<Range> free_, used_;
};
// Look up the device address of this device's scratch array (the device must be
// current); idempotent.  scratch_ptr returns it (null before set-up).
void scratch_setup(int device);
void* scratch_ptr(int device);
size_t scratch_bytes();

}  // namespace hc

// ---------------------------------------------------------------- handles
struct hc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hc::Alloc alloc;
    std::string err;
    int profiling = 0;
    hc_timing timing{};
    int num_cus = 256;
    int grid_limit = 0;                    // workgroups of a persistent launch at most (0: default)
    std::atomic<int> cancel{0};            // cancel request (host view)
    int* h_cancel = nullptr;               // the same request in coherent pinned host memory,
    int* d_cancel = nullptr;               // read by kernels through this device address
};

struct hc_coco {
    hc::Alloc alloc;
    int32_t arity = 0;
    int32_t key_bits = 0;
    int32_t mix_bits = 0;         // low bits mixed; the bits above are a segment number
    uint64_t mix_seed = 0;
    int32_t col_order[4] = {0, 1, 2, 3};
    hc_dtype dtype = HC_I32;
    int64_t n_input = 0, n_unique = 0;
    int64_t level_len[4] = {0, 0, 0, 0};
    int64_t max_children[4] = {0, 0, 0, 0};
    int64_t distinct[4] = {0, 0, 0, 0};
    int32_t symmetric = 0;
    uint32_t* V[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t* O[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t bytes = 0;
};

namespace hc {

// ---------------------------------------------------------------- primitives (prim.hip)
// Exclusive prefix sum of u32 counts into u64 (out has n+1 entries; out[n] = total).
void scan_u32_to_u64(const Alloc& a, const uint32_t* in, uint64_t* out, int64_t n, hipStream_t s);
void scan_u64(const Alloc& a, const uint64_t* in, uint64_t* out, int64_t n, hipStream_t s);
// Exclusive prefix of popcounts of 64-bit words (out has n+1 entries).
void scan_popc(const Alloc& a, const uint64_t* words, uint64_t* out, int64_t n, hipStream_t s);
// LSD radix sort of u64 keys over their low `bits` bits; result in *keys (buffers swapped).
void radix_sort_u64(const Alloc& a, DevBuf<uint64_t>& keys, DevBuf<uint64_t>& tmp, int64_t n, int bits,
                    hipStream_t s);

// Sort n emitted head-order rows (nv columns of raw ids below 2^b, int32 or int64)
// lexicographically, in place (rows.hip).
void sort_rows(const Alloc& a, void* rows, int64_t n, int nv, int b, bool i64, hipStream_t s);

// ---------------------------------------------------------------- build (build.hip)
void build_coco(hc_ctx* ctx, const void* tuples, int64_t n, int arity, hc_dtype dtype,
                const int32_t* col_order, int key_bits, int mix_bits, uint64_t seed, uint32_t flags,
                hc_coco* out);
void partition_sizes(hc_ctx* ctx, const hc_coco* c, const int32_t* log2_shares, int64_t* B,
                     int64_t* Bpref);

// ---------------------------------------------------------------- plan (plan.cpp)
constexpr int kMaxVars = 8;
constexpr int kMaxAtoms = 16;
constexpr int kMaxOps = 8;      // operands of one level intersection
constexpr int kMaxGroups = 8;

enum OpKind : int32_t { OP_V0 = 0, OP_CHILD = 1, OP_TMP = 2 };

struct PlanOp {
    int32_t kind;
    int32_t atom;     // atom index (V0 / CHILD)
    int32_t group;    // lifted group (TMP)
    int32_t lvl;      // CoCo level of the operand (V0: 0; CHILD: 1 .. arity-1)
};

struct PlanGroup {           // a lifted intersection (Section 6.1)
    int32_t var;
    int32_t consumer;        // level (0-based) whose loop consumes it
    int32_t lift;            // computed on frontier F_lift (lift vars bound)
    int32_t n_ops;
    PlanOp ops[kMaxOps];     // V0 / CHILD operands only
};

struct PlanLevel {
    int32_t var;
    int32_t n_ops;
    PlanOp ops[kMaxOps];     // after lifting: V0 / CHILD / TMP
    int32_t n_new_nodes;     // atoms whose first variable is bound here and which have a child level
    int32_t new_node_atom[kMaxAtoms];
};

struct Plan {
    int32_t n_vars = 0, n_atoms = 0;
    int32_t order[kMaxVars];
    int32_t pos[kMaxVars];           // level of each variable
    int32_t atom_arity[kMaxAtoms];
    int32_t atom_first[kMaxAtoms];   // variable at CoCo level 0
    int32_t atom_second[kMaxAtoms];  // variable at CoCo level 1 (-1 for unary)
    int32_t atom_lvl_var[kMaxAtoms][4];   // variable at every CoCo level (columns in variable order)
    int32_t n_groups = 0;
    PlanGroup groups[kMaxGroups];
    PlanLevel levels[kMaxVars];
};

// Validates q and order; builds the per-level plan with (optionally) the lift rule.
// Intersections that would be lifted to a frontier below min_lift stay where they are.
Plan compile_plan(const hc_query* q, const int32_t* order, bool rewrite, int min_lift = 0);
std::string describe_plan(const Plan& p);
// Validate the query alone (variables covered, arities, repeated variables).
void validate_query(const hc_query* q, int max_arity);

struct AtomStats {
    double rows;           // |R_j| (unique)
    double distinct[4];    // distinct values per original column
    double maxdeg[4];      // longest child list below CoCo level r (0 if unknown)
    int32_t arity;
    int32_t dom_bits;
};
void choose_shares(const hc_query* q, const std::vector<AtomStats>& st, int K, uint32_t flags,
                   int32_t* order_inout, int32_t* shares_out);
// Cost of one (order, shares) plan under the model: per-level costs (n entries,
// already multiplied by the replication of Eq. (total cost)) and their sum.
double plan_cost(const hc_query* q, const std::vector<AtomStats>& st, const int32_t* order, const int32_t* shares,
                 uint32_t flags, double* per_level);

// ---------------------------------------------------------------- join (join.hip)
// Chunking cap: frontier entries, lifted-pool elements and elements per expand /
// emit chunk below F_0 (a single entry larger than the cap still goes whole).
constexpr int64_t kDefaultCap = (int64_t)1 << 27;
// alloc: where the call's device buffers come from (null: the context's allocator);
// cap_entries: the chunking cap (0: kDefaultCap); cell_group: cell_counts holds one
// count per group of 2^cell_group consecutive cells.
void join_run(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
              const int32_t* shares, uint32_t flags, bool emit, uint64_t* count, uint64_t* digest,
              void* out, int64_t capacity, int64_t* n_out, uint64_t* cell_counts = nullptr,
              int64_t n_multi = 0, const int64_t* multi_ranges = nullptr, const Alloc* alloc = nullptr,
              int64_t cap_entries = 0, int cell_group = 0);
// with_small_path: also cover the device-sized sequence a small count takes
// (hc_join_count, hc_join_count_cells); false for calls that always run eagerly.
uint64_t join_workspace_bound(const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                              const int32_t* shares, uint32_t flags, int64_t n_queries, int64_t first_width,
                              int64_t cap_entries = kDefaultCap, bool with_small_path = true);

// Device-sized joins captured in a HIP graph (join.hip).
hc_join_graph* join_graph_create(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                                 const int32_t* shares, uint32_t flags, int32_t cell_group, void* out,
                                 int64_t capacity, int64_t frontier_cap, int64_t item_cap);
void join_graph_launch(hc_join_graph* g);
void join_graph_result(hc_join_graph* g, uint64_t* count, uint64_t* cell_counts, int64_t* n_out, int32_t* replayed);
void join_graph_destroy(hc_join_graph* g);
hc_ctx* join_graph_ctx(const hc_join_graph* g);
// A join that its CoCo statistics bound to small frontiers (at most 2^20 entries
// and 2^23 elements per level), run as the device-sized launch sequence directly on
// the context's stream: no host read-back between the levels.  Returns false, having
// done nothing, when the join is not such a join (the caller then runs the eager
// path); results as join_run's.
bool join_small_device_sized(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                             const int32_t* shares, uint32_t flags, int32_t cell_group, void* out, int64_t capacity,
                             uint64_t* count, uint64_t* cell_counts, int64_t* n_out);

}  // namespace hc
