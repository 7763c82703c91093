/*
 * hc.h -- C-ABI of the MI355X (gfx950) Generic Join library.
 *
 * The library evaluates a full conjunctive query (Section 2, Eq. (1)):
 *     Q(X_1..X_n) <- R_1(X_1) AND ... AND R_m(X_m)
 * under set semantics, by Generic Join (Section 2, "Generic Join Algorithm")
 * over the CoCo index (Section 4), with the domain of every variable
 * HyperCube-partitioned by power-of-two shares (Section 2, "HyperCube
 * Algorithm"; Section 5), and with the lifted-intersection rewriting of
 * Section 6.1.  Shares and the variable order can be chosen by the cost model
 * of Sections 6.2-6.3.
 *
 * Conventions shared by every call
 *  - Device pointers point to memory of the context's device; host pointers to
 *    ordinary host memory.  Every call names which one each argument is.
 *  - Calls are ordered on the context's HIP stream and return after the work
 *    they launched has completed, so results are valid on return.
 *  - No call aborts or throws across the ABI.  A non-HC_OK status leaves a
 *    message retrievable with hc_last_error(ctx); outputs are then unspecified
 *    unless stated otherwise.
 *  - Ids are non-negative integers.  Values are mapped to b-bit keys by a
 *    bijective mixer H_b (b = key_bits) fixed per CoCo; a share 2^k of a
 *    variable selects the top k bits of H_b(x) (the paper leaves the hash open;
 *    any deterministic map partitions the output correctly).  All CoCos used
 *    by one join must share b and the mixer seed.
 *  - Scratch device memory comes from the allocator given to hc_ctx_create.
 *  - A context is not thread-safe (hc_ctx_cancel excepted); use one context
 *    per host thread.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_ERR_INVALID = 1,      /* malformed argument or query */
    HC_ERR_OOM = 2,          /* the allocator refused a request */
    HC_ERR_OVERFLOW = 3,     /* emit: more result rows than the capacity */
    HC_ERR_DEVICE = 4,       /* a HIP runtime call or a device-side check failed */
    HC_ERR_UNSUPPORTED = 5,  /* valid but outside what the library implements */
    HC_ERR_CANCELLED = 6     /* the context's cancel request stopped the call */
} hc_status;

typedef enum { HC_I32 = 0, HC_I64 = 1 } hc_dtype;

typedef struct hc_ctx hc_ctx;
typedef struct hc_coco hc_coco;
typedef struct hc_join_graph hc_join_graph;

/*
 * A full conjunctive query (Section 2, Eq. (1)).  Variables are 0..n_vars-1,
 * which is also the head (output column) order.  Atom j has atom_arity[j]
 * variables, listed consecutively in atom_vars.  Every variable must occur in
 * some atom (Section 2).  A variable repeated inside one atom is unsupported.
 * var_lo/var_hi (host, nullable, both or neither): a range predicate
 * var_lo[v] <= x_v < var_hi[v] on raw ids pushed down into the atoms
 * (Section 2 treats predicates this way); used to emit outputs in chunks.
 */
typedef struct {
    int32_t n_vars;
    int32_t n_atoms;
    const int32_t* atom_arity;   /* host, [n_atoms] */
    const int32_t* atom_vars;    /* host, [sum of arities] */
    const int64_t* var_lo;       /* host, [n_vars] or NULL */
    const int64_t* var_hi;       /* host, [n_vars] or NULL */
} hc_query;

typedef void* (*hc_alloc_fn)(size_t bytes, void* user);
typedef void (*hc_free_fn)(void* ptr, void* user);

/* Flags of hc_build_coco */
#define HC_BUILD_SYMMETRIC 0x1u   /* binary relation claimed symmetric: verified on the
                                     device; the CoCo then serves both column orders */

/* Flags of hc_compute_shares / hc_join_count / hc_join_emit.  Every call rejects
 * (HC_ERR_INVALID) a bit it does not take: the joins take HC_NO_REWRITE,
 * HC_FORCE_MERGE, HC_FORCE_GALLOP, an HC_SEARCH_* method and (hc_join_emit only)
 * HC_EMIT_SORTED; hc_compute_shares takes HC_NO_REWRITE, HC_KEEP_ORDER,
 * HC_JOINT_SEARCH, HC_PESSIMISTIC and HC_CACHE_SHARES. */
#define HC_NO_REWRITE     0x1u    /* disable the Section 6.1 lift */
/* The two forced intersection methods of Section 5: every operand a level does
 * not iterate is searched from its cursor by a linear scan (the multiway merge,
 * HC_FORCE_MERGE, the same as HC_SEARCH_LINEAR) or by galloping (exponential
 * search, HC_FORCE_GALLOP, the same as HC_SEARCH_EXPONENTIAL).  Setting both,
 * or one with an HC_SEARCH_* method other than its own, is HC_ERR_INVALID. */
#define HC_FORCE_MERGE    0x2u
#define HC_FORCE_GALLOP   0x4u
/* hc_join_emit: the rows come out in lexicographic order of the head-order tuple
 * (raw ids compared as unsigned integers), sorted on the device. */
#define HC_EMIT_SORTED    0x80u
/* hc_join_*: how the operands a level does not iterate are searched (Section 5).
 * HC_SEARCH_WINDOW (0, default): wave-cooperative -- the step's candidate range
 * is staged in LDS and searched there.  The others are the paper's per-element
 * methods, one search per lane: exponential (galloping), quadratic (fixed jumps
 * of a 128-byte line, applied at two levels, then a scan), linear (a scan), or
 * chosen per step by the candidate range's size (<= 32: linear, <= 4096:
 * quadratic, else exponential).  Results do not depend on the method. */
#define HC_SEARCH_SHIFT       8
#define HC_SEARCH_MASK        0x700u
#define HC_SEARCH_WINDOW      0x000u
#define HC_SEARCH_EXPONENTIAL 0x100u
#define HC_SEARCH_QUADRATIC   0x200u
#define HC_SEARCH_LINEAR      0x300u
#define HC_SEARCH_BY_SIZE     0x400u
#define HC_KEEP_ORDER     0x8u    /* hc_compute_shares: use var_order_inout as given */
#define HC_JOINT_SEARCH   0x10u   /* hc_compute_shares: search orders and shares jointly */
#define HC_PESSIMISTIC    0x20u   /* cost model: upper-bound cardinality estimator */
#define HC_CACHE_SHARES   0x40u   /* hc_compute_shares: cheapest vector whose cells fit an L2 */

/*
 * Create a context on HIP device `device`, ordering work on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  alloc/free_ (nullable, both or
 * neither) supply device memory, e.g. from a framework's caching allocator;
 * alloc returns NULL to refuse (reported as HC_ERR_OOM).  Without them the
 * library uses stream-ordered hipMallocAsync/hipFreeAsync.
 * Errors: HC_ERR_INVALID (bad device, out == NULL), HC_ERR_DEVICE.
 */
hc_status hc_ctx_create(int device, void* hip_stream, hc_alloc_fn alloc, hc_free_fn free_,
                        void* user, hc_ctx** out);
void hc_ctx_destroy(hc_ctx* ctx);
/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char* hc_last_error(const hc_ctx* ctx);

/*
 * Build the CoCo index of one relation (Section 4, "Compressed Column
 * layout"): the tuples are mapped to mixed keys, sorted lexicographically in
 * column order col_order (the order of the atom's variables in the variable
 * order), deduplicated (set semantics: the last level keeps no offsets), and
 * split into levels V_r (values, one per distinct prefix) and O_r (offsets of
 * each entry's children in level r+1; l_r + 1 entries).
 *   tuples     device, row-major [n][arity] of dtype; borrowed for the call
 *   n          rows, 0 <= n < 2^31
 *   arity      1..4
 *   col_order  host, permutation of 0..arity-1
 *   key_bits   b in 1..32, or 0 = smallest b covering the largest id;
 *              arity * b <= 64 is required
 *   mix_seed   seed of the mixer (its low b bits are used)
 *   flags      HC_BUILD_SYMMETRIC or 0
 *   out        receives a library-owned handle (free with hc_coco_free, not
 *              while a join that uses it runs)
 * Errors: HC_ERR_INVALID (negative id, id >= 2^b, bad col_order, symmetry claim
 * false), HC_ERR_UNSUPPORTED (arity*b > 64), HC_ERR_OOM, HC_ERR_DEVICE.
 */
hc_status hc_build_coco(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity, hc_dtype dtype,
                        const int32_t* col_order, int32_t key_bits, uint64_t mix_seed,
                        uint32_t flags, hc_coco** out);
void hc_coco_free(hc_coco* coco);

/*
 * Segmented build, for many independent relations fused into one index (one
 * query per segment of a batch): ids are seg * 2^mix_bits + x with x < 2^mix_bits
 * and seg < 2^segment_bits; only the low mix_bits are mixed, so every segment
 * occupies one contiguous key range.  key_bits = mix_bits + segment_bits <= 32.
 * A join over segmented CoCos must give the first variable of the order a share
 * of at least segment_bits (its coordinate names the segment) and no share to
 * the other variables; every operand then stays inside the segment of its cell,
 * so one cell never mixes two relations.  Other arguments as hc_build_coco.
 */
hc_status hc_build_coco_segmented(hc_ctx* ctx, const void* tuples, int64_t n, int32_t arity,
                                  hc_dtype dtype, const int32_t* col_order, int32_t mix_bits,
                                  int32_t segment_bits, uint64_t mix_seed, uint32_t flags,
                                  hc_coco** out);

/* Statistics of a built CoCo (host struct, filled by hc_coco_get_info). */
typedef struct {
    int64_t n_input;            /* rows given */
    int64_t n_unique;           /* rows after deduplication */
    int32_t arity;
    int32_t key_bits;
    uint64_t mix_seed;
    int32_t col_order[4];
    int64_t level_len[4];       /* l_r: entries of level r */
    int64_t max_children[4];    /* largest child list below level r (r < arity-1) */
    int64_t distinct[4];        /* distinct values of input column c (original order) */
    int32_t symmetric;          /* verified symmetric binary relation */
    int32_t dtype;              /* hc_dtype of the input ids (also of emitted rows) */
    int64_t bytes;              /* device bytes held by the index */
    int32_t mix_bits;           /* low key bits that are mixed (= key_bits unless segmented) */
    int32_t reserved;
} hc_coco_info;

hc_status hc_coco_get_info(const hc_coco* coco, hc_coco_info* info);

/*
 * Copy level r of a CoCo to host memory: values (uint32 mixed keys,
 * level_len[r] entries) and, for r < arity-1, offsets (int32, level_len[r]+1
 * entries).  Either pointer may be NULL to skip it.
 */
hc_status hc_coco_copy_level(hc_ctx* ctx, const hc_coco* coco, int32_t level,
                             uint32_t* values_host, int32_t* offsets_host);

/*
 * Partition sizes of a relation under per-column shares (Section 4): tuple
 * (x_1..x_k) belongs to partition (s_1..s_k), s_c = top log2_shares[c] bits of
 * H_b(x_c) (columns in the relation's original order).  B[s] counts the unique
 * tuples of partition s and Bpref[s] is the exclusive prefix sum of B in
 * lexicographic order of s, i.e. the start of partition s in the partitioned
 * array.  B_host/Bpref_host: host, 2^(sum log2_shares) entries each.
 * Errors: HC_ERR_INVALID if a share exceeds b or the total exceeds 2^24.
 */
hc_status hc_partition_sizes(hc_ctx* ctx, const hc_coco* coco, const int32_t* log2_shares,
                             int64_t* B_host, int64_t* Bpref_host);

/*
 * Choose the variable order and the shares (Sections 6.2-6.3).  P = 2^K cells
 * (K = log2_total_P, 0..24) are split as P = prod 2^k_v.  The cost of an order
 * sums, over the levels, |S| * min N * log2(1 + max N / min N) bounded with the
 * statistics of the CoCos (Lemma of Section 6.2), the rewriting moving lifted
 * operands to their lift level; a share vector costs sum_i (prod_{j>i} P_j) *
 * C_i (Eq. (total cost)).  Vectors costing more than twice the unpartitioned
 * cost, or with a share P_v such that |Dom(X_v)| < 3 P_v ln P_v, are pruned;
 * the minimum evenness E = sum_i P_sigma(i) * max(1 - i/100, 3/4) wins.
 * With HC_JOINT_SEARCH (and not HC_KEEP_ORDER) orders and share vectors are
 * searched together: a vector of any order is feasible when it costs at most
 * twice the best unpartitioned cost over all orders.  HC_PESSIMISTIC bounds
 * the prefix bindings from above (longest lists, whole atoms inside the
 * prefix) instead of chaining average list sizes.
 * HC_CACHE_SHARES replaces the evenness rule, which balances one cell per CPU
 * thread, with the GPU's concern: the work queue balances the cells, and a
 * cell's CoCo slices should fit the 4 MB L2 of the XCD that sweeps it.  Among
 * the vectors passing the domain rule, those whose every atom slice (4 bytes
 * per tuple divided by the shares of the atom's variables) fits 4 MB compete
 * on Eq. (total cost) alone; if none fits, the smallest largest slice wins,
 * then the lower cost.  Only the order given or chosen as above is searched.
 *   atom_index       host array of n_atoms CoCo handles (may repeat)
 *   var_order_inout  host [n_vars]; if HC_KEEP_ORDER is set it is the order to
 *                    use, else it receives the chosen order
 *   log2_shares_out  host [n_vars], indexed by variable id
 * Host-only: launches nothing.  Errors: HC_ERR_INVALID.
 */
hc_status hc_compute_shares(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                            int32_t log2_total_P, uint32_t flags, int32_t* var_order_inout,
                            int32_t* log2_shares_out);

/*
 * Same decision from statistics only (host-only, needs no context or GPU):
 * infos[j] describes the CoCo of atom j as hc_coco_get_info would.
 */
hc_status hc_compute_shares_from_info(const hc_query* q, const hc_coco_info* infos, int32_t log2_total_P,
                                      uint32_t flags, int32_t* var_order_inout, int32_t* log2_shares_out);

/*
 * The cost model's figure for one plan (host-only, from statistics): Eq. (total
 * cost) of Section 6.3 for the order var_order and the shares log2_shares
 * (NULL: all zero) -- the per-level costs of Section 6.2 bounded with the
 * Lemma, each multiplied by the product of the shares of the later variables.
 * flags: HC_NO_REWRITE, HC_PESSIMISTIC.  per_level_out (host [n_vars] in
 * level order, may be NULL) receives the replicated per-level costs,
 * total_out (host) their sum.  Errors: HC_ERR_INVALID.
 */
hc_status hc_plan_cost_from_info(const hc_query* q, const hc_coco_info* infos, const int32_t* var_order,
                                 const int32_t* log2_shares, uint32_t flags, double* per_level_out,
                                 double* total_out);

/*
 * Count |Q(D)| (Section 5): every HyperCube cell (s_1..s_n), s_v in
 * [0, 2^log2_shares[v]), runs Generic Join restricted to the key ranges of its
 * coordinates; cells have disjoint outputs whose union is Q(D), so the count
 * does not depend on the shares, the order or the rewriting.
 *   atom_index   host array of n_atoms CoCo handles; the CoCo of atom j must
 *                have its columns ordered by the positions of atom j's
 *                variables in var_order (or be symmetric, for binary atoms)
 *   var_order    host [n_vars], a permutation of the variables
 *   log2_shares  host [n_vars] indexed by variable id, each 0..b, sum <= 24;
 *                NULL = all zero
 *   count_out    host, receives the count
 *   digest_out   host [2] or NULL: order-independent digest of the output set
 *                (sum and xor over the rows t, in head order with raw ids, of
 *                h(t) = F(...F(F(c ^ (t_0 + G)) ^ (t_1 + 2G))...), F the
 *                SplitMix64 finaliser, c = 0x6A09E667F3BCC909, G = 0x9E3779B97F4A7C15)
 * flags: HC_NO_REWRITE, HC_SEARCH_*.
 * A join whose CoCo statistics bound every frontier below 2^20 entries and every
 * level below 2^23 elements (entries times the longest list of the level's
 * shortest operand), with the default search and no digest, runs the
 * captured joins' device-sized launch sequence directly (no host read-back
 * between the levels; see hc_join_graph_create); likewise hc_join_emit,
 * hc_join_count_cells and hc_join_count_segments.  Results do not depend on it.
 * Errors: HC_ERR_INVALID (bad query, order, shares, or CoCos that do not
 * match), HC_ERR_UNSUPPORTED (a frontier entry wider than the engine's limit),
 * HC_ERR_OOM, HC_ERR_CANCELLED (hc_ctx_cancel), HC_ERR_DEVICE.
 */
hc_status hc_join_count(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                        const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                        uint64_t* count_out, uint64_t* digest_out);

/*
 * hc_join_count for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same count and digest, with every device buffer of the call carved out of a
 * fixed scratch array of 256 MiB that the library holds on each GPU it runs on
 * (set up when the first context on that GPU is created, kept until the process
 * ends).  The call makes no hipMalloc or hipFree and never calls the context's
 * allocator; profiling events are not recorded.  The call's inputs (the CoCos)
 * and outputs are the caller's as for hc_join_count.
 *   scratch_used  host, nullable: receives the bytes of the array the call used
 * Every call on one GPU shares that GPU's array and leaves its contents behind
 * (the call clears what it needs): calls that overlap on one GPU -- from two
 * contexts or threads -- race and must not be issued.
 * Errors: HC_ERR_UNSUPPORTED when hc_join_workspace_bound of the call exceeds
 * the array (use hc_join_count then); HC_ERR_OOM if the array's free ranges
 * cannot hold a buffer; otherwise as hc_join_count.
 */
hc_status hc_join_count_noalloc(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                                uint64_t* count_out, uint64_t* digest_out, uint64_t* scratch_used);

/*
 * Count per HyperCube cell (the output of each of the paper's threads, Section
 * 5): cell_counts (host, 2^(sum of log2_shares) entries) receives the number of
 * result tuples of every cell; the cell id packs the coordinates of the
 * variables in order, the first variable of the order in the lowest bits, each
 * taking log2_shares[v] bits.  count_out receives the total.  With segmented
 * CoCos and only the first variable split by exactly segment_bits, cell c is
 * segment c, i.e. one query of a batch.  Errors as hc_join_count.
 */
hc_status hc_join_count_cells(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                              const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                              uint64_t* cell_counts, uint64_t* count_out);

/*
 * Count per segment of segmented CoCos (the batched workload: one independent
 * query per segment, all fused into one join; Section 5's cells partition the
 * output, so a segment's cells add up to its query's count).  The first variable
 * of the order takes the share segment_bits + log2_extra (every segment split into
 * 2^log2_extra cells, the per-query split the batch autotuner chooses), the others
 * none; the per-cell counts are summed per segment on the device.
 *   segment_counts  host, 2^segment_bits entries: the count of each segment
 *   count_out       host: the total
 * Errors: HC_ERR_INVALID (CoCos not segmented, segment_bits + log2_extra > 24, bad
 * query or order); otherwise as hc_join_count.
 */
hc_status hc_join_count_segments(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                 const int32_t* var_order, int32_t log2_extra, uint32_t flags,
                                 uint64_t* segment_counts, uint64_t* count_out);

/*
 * Many instances of one query in one pass (the served workload fuses the
 * queued requests of one shape over one resident CoCo set): instance t is q
 * with its first variable (var_order[0]) restricted to raw ids in
 * [first_var_ranges[2t], first_var_ranges[2t+1]) (an empty or inverted range
 * selects nothing); any var_lo/var_hi of q apply to every instance.  Frontier
 * F_0 of Generic Join (Section 5) holds one entry per instance instead of one
 * per HyperCube cell; no shares are taken.  counts_out (host, n_queries
 * entries) receives each instance's count, equal to hc_join_count of that
 * instance alone.  first_var_ranges is host memory, [n_queries][2] int64.
 * Errors: HC_ERR_INVALID for a bad query, order, NULL argument, negative
 * n_queries, more than 2^24 instances or segmented CoCos; otherwise as
 * hc_join_count.
 */
hc_status hc_join_count_multi(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                              const int32_t* var_order, uint32_t flags, int64_t n_queries,
                              const int64_t* first_var_ranges, uint64_t* counts_out);

/*
 * Memory estimate for admission control (the served workload keeps CoCos
 * resident and admits work while its estimate fits the free budget): an upper
 * bound, in bytes, of the device memory one call allocates through the
 * context's allocator -- hc_join_count / hc_join_count_cells with these
 * arguments when n_queries = 0, or hc_join_count_multi with n_queries
 * instances whose first-variable ranges are at most first_width ids wide
 * (0: unbounded; log2_shares is then ignored).  Host-only: it reads the CoCos'
 * statistics (level lengths, longest child list) and launches nothing.  The
 * bound follows the level-by-level frontiers of Generic Join (Section 5):
 * entries of F_{i+1} are at most those of F_i times the longest list of level
 * i's shortest operand (an id range on the variable caps it by the range
 * width), and each frontier chunk, pool and table by the library's chunking
 * cap of 2^27 entries; a count call bounded to small frontiers (see
 * hc_join_count) is charged the fixed capacities it then takes, when those are
 * larger.  bytes_out (host) receives it.  Errors: HC_ERR_INVALID
 * for a bad query, order, NULL argument or negative count or width.
 */
hc_status hc_join_workspace_bound(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                                  const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                                  int64_t n_queries, int64_t first_width, uint64_t* bytes_out);

/*
 * Materialise Q(D) (Section 5: each cell writes its own outputs, then they are
 * concatenated).  out: device, row-major [capacity][n_vars] in head order,
 * raw ids, same dtype as the CoCos' input.  n_out (host) always receives the
 * exact number of result rows; if it exceeds capacity the call returns
 * HC_ERR_OVERFLOW and the contents of out are unspecified.  Row order is
 * deterministic for given inputs, order and shares, but otherwise unspecified,
 * unless flags has HC_EMIT_SORTED: then the rows are in lexicographic order.
 * Other arguments and errors as hc_join_count.
 */
hc_status hc_join_emit(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                       const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                       void* out, int64_t capacity, int64_t* n_out);

/*
 * A Generic Join (Sections 5 and 6) recorded once as a fixed launch sequence in a
 * HIP graph and replayed: every kernel reads the frontier sizes the kernel before
 * it wrote in device memory, so a replay makes no host round trip between the
 * levels (the eager calls read each level's sizes back to size the next).  The
 * frontiers below F_0 hold at most frontier_cap entries and every level that
 * materialises (all but a counting deepest level) at most item_cap elements
 * (0: 2^20 and 2^22); a replay whose data exceeds them raises a device flag, and
 * hc_join_graph_result then computes that call's result with the eager path, so
 * results are always exact.  The graph is bound to the CoCo handles, their
 * contents, the query, order and shares it was created with, and to ctx (all must
 * outlive it); replays run on ctx's stream.
 *   cell_group  < 0: a count; >= 0: per-cell counts as hc_join_count_cells, summed
 *               over groups of 2^cell_group consecutive cells (with segmented
 *               CoCos and the first variable's share segment_bits + extra,
 *               cell_group = extra gives per-segment counts as
 *               hc_join_count_segments)
 *   out         device, nullable: emit the rows as hc_join_emit (unsorted) into
 *               capacity rows; then cell_group must be < 0
 * Lifted intersections (Section 6.1) run on the frontier they are lifted to, each
 * with at most item_cap elements per call, into a pool of item_cap elements.
 * Supported plans: at most 4 operands per level and per lifted intersection, the
 * default search (flags take HC_NO_REWRITE only).
 * Errors: HC_ERR_INVALID (as hc_join_count; capacities above 2^28 entries or
 * 2^30 elements), HC_ERR_UNSUPPORTED (plans outside the above), HC_ERR_OOM,
 * HC_ERR_DEVICE.
 */
hc_status hc_join_graph_create(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atom_index,
                               const int32_t* var_order, const int32_t* log2_shares, uint32_t flags,
                               int32_t cell_group, void* out, int64_t capacity, int64_t frontier_cap,
                               int64_t item_cap, hc_join_graph** graph_out);
/* Enqueue one replay on ctx's stream (asynchronous). */
hc_status hc_join_graph_launch(hc_join_graph* g);
/*
 * Wait for the last replay and return its result: count_out (host) the count, or
 * the rows emitted; cell_counts (host, nullable; 2^(K - cell_group) entries) the
 * per-cell counts; n_out (host, nullable) the rows; replayed (host, nullable) 1
 * when the replay's own result was used, 0 when a capacity was exceeded and the
 * eager path computed it.  Errors: HC_ERR_INVALID (no replay launched),
 * HC_ERR_OVERFLOW (emit: more rows than the capacity; n_out holds the total),
 * HC_ERR_CANCELLED, HC_ERR_DEVICE.
 */
hc_status hc_join_graph_result(hc_join_graph* g, uint64_t* count_out, uint64_t* cell_counts, int64_t* n_out,
                               int32_t* replayed);
/* Wait for every replay on ctx's stream, then release the graph and its buffers. */
void hc_join_graph_destroy(hc_join_graph* g);

/*
 * Describe the compiled Generic Join plan (per level: operands and the lifted
 * intersections of Section 6.1) as JSON text into buf (host, cap bytes,
 * NUL-terminated).  Host-only.  Errors: HC_ERR_INVALID, HC_ERR_OVERFLOW if
 * cap is too small.
 */
hc_status hc_plan_describe(const hc_query* q, const int32_t* var_order, uint32_t flags,
                           char* buf, size_t cap);

/*
 * Timing of the most recent join call on ctx, measured with HIP events on the
 * context stream when profiling is on (hc_ctx_set_profiling): total
 * milliseconds and launch count of the kernel that runs the deepest level of
 * Generic Join, and of the whole call.
 */
typedef struct {
    double leaf_ms;
    int64_t leaf_launches;
    double total_ms;
    uint64_t leaf_items;        /* smallest-operand elements visited at the deepest level */
} hc_timing;
hc_status hc_ctx_set_profiling(hc_ctx* ctx, int on);

/*
 * Device share of the context's calls (for callers that run several calls at once
 * on one GPU, e.g. the slots of a serving loop): the persistent intersection
 * kernels launch at most max_workgroups workgroups (rounded down to a multiple of
 * 8, at least 8) instead of 8 per compute unit, so that a long call does not hold
 * every compute unit while others wait.  0 restores the default.  Results do not
 * depend on it.  Errors: HC_ERR_INVALID (NULL ctx, negative limit).
 */
hc_status hc_ctx_set_grid_limit(hc_ctx* ctx, int32_t max_workgroups);

/*
 * Cancel request (for callers that bound a request's time, e.g. a serving loop):
 * on != 0 raises it, on = 0 withdraws it.  While it is raised, every join call on
 * this context returns HC_ERR_CANCELLED: a call already running notices it
 * between its launches and inside the intersection kernels, where the wave that
 * takes every 64th work chunk reads the request (a word of pinned host memory the
 * context owns) and, finding it raised, empties the work queues so that every
 * wave leaves at its next chunk; the call's outputs are then unspecified.  Safe to call from
 * another thread while a join runs on ctx: it is a plain store, no stream
 * operation.  Errors: HC_ERR_INVALID (NULL ctx).
 */
hc_status hc_ctx_cancel(hc_ctx* ctx, int32_t on);
hc_status hc_ctx_get_timing(const hc_ctx* ctx, hc_timing* t);

#ifdef __cplusplus
}
#endif
#endif /* HC_H */
