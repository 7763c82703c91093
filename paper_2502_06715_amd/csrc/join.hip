// Generic Join over CoCo with HyperCube cells (Sections 2, 5, 6.1).
//
// Execution model.  A frontier F_i holds one entry per binding of the first i
// variables of the order, tagged with the HyperCube cell it belongs to:
//   word 0          cell id (coordinates of every variable packed together)
//   words 1..i      the bound values (mixed keys)
//   node words      for every atom and CoCo level r whose variable is bound
//                   while the variable of level r+1 is not: the index of the
//                   bound prefix in level r (its child list is
//                   O_r[node]..O_r[node+1] in level r+1)
//   tmp words       (offset, length) of the lifted intersections that are live
// F_0 holds one entry per cell, so every cell runs its own Generic Join
// restricted to the key range of its coordinates (Section 5); the key range of
// coordinate s of a variable with share 2^k is [s << (b-k), (s+1) << (b-k)),
// which is a contiguous sub-range of every sorted CoCo array.
//
// Level i expands F_i into F_{i+1}: for every entry it intersects the level's
// operands (Section 5, "multiway intersection"; Section 2: iterate the
// smallest set, probe the others).  On the GPU the iteration elements of all
// entries are flattened into one index space by a prefix sum over the
// per-entry sizes, so every wave64 gets 64 consecutive elements whatever the
// skew (the load balancing the paper gets from work stealing); each lane
// probes the other operands by binary search, and a ballot gives one 64-bit
// match word per wave.  A scan over the match words' popcounts gives every
// match its output slot, so frontiers, temporary results and emitted rows are
// compact, ordered and deterministic.  The deepest level only counts (or
// digests, or writes rows).
//
// Lifted intersections (Section 6.1) are computed the same way on the frontier
// where they are lifted to, stored as sorted arrays in a pool together with
// the top-level positions of their sources, and referenced by (offset, length)
// from the entries until the consuming level.
#include <algorithm>
#include <cstddef>
#include <memory>

#include "prim_dev.h"

namespace hc {

constexpr int kMaxW = 32;   // words per frontier entry

struct DAtom {
    const uint32_t* V[4];   // CoCo levels: keys
    const int32_t* O[3];    // child offsets of levels 0..arity-2
    int64_t len[4];         // level lengths
};

struct KData {
    DAtom atoms[kMaxAtoms];
    const uint32_t* tmp_val[kMaxGroups];
    const int32_t* tmp_src[kMaxGroups][kMaxOps];
    Mixer mix;
    int32_t b;
    int32_t dtype64;
    const int* cancel;   // nonzero: the caller cancelled the call (polled between work chunks)
    int32_t cell_group;  // per-cell counts are accumulated per group of 2^cell_group consecutive cells
    int32_t grid_limit;  // host only: workgroups of a persistent launch at most (0: kPersistBlocks)
};

struct KOp {
    int32_t kind;
    int32_t atom;
    int32_t word;     // CHILD: entry word of the parent node; TMP: entry word of (offset, length)
    int32_t group;    // TMP
    int32_t lvl;      // CoCo level read (V0: 0; CHILD: the children's level)
    const int2* v0_range;   // V0 restricted by the cell: table indexed by the coordinate (or null)
    int32_t rng_shift, rng_k;     // coordinate = (src >> rng_shift) & (2^rng_k - 1), src = the cell id
    int32_t rng_word;             // or, when >= 0, this word of the entry (a bound key, a query's id range)
    const int32_t* child_range;   // CHILD: per node, start of every coordinate's sub-range (or null)
    int32_t child_stride;         // 2^k + 1 entries per node
};

struct KStep {
    int32_t n_ops;
    KOp ops[kMaxOps];
    int32_t W_in;
    int32_t k_share;          // log2 share of the variable bound by this step
    int32_t cell_shift;       // bit position of its coordinate in the cell id
    int32_t has_pred;
    int64_t pred_lo, pred_hi;     // id range of the variable bound here (all entries)
    int32_t pred_word;            // >= 0: each entry also carries its own range (lo, hi inclusive) there
    int32_t search;               // SEARCH_*: how the other operands are searched
    // EXPAND output
    int32_t W_out;
    int32_t n_copy;
    int8_t copy_from[kMaxW], copy_to[kMaxW];
    int32_t val_word;
    int32_t n_new;
    int8_t new_word[kMaxAtoms], new_op[kMaxAtoms], new_src[kMaxAtoms];
    int32_t n_zero;
    int8_t zero_word[kMaxW];
    // TMP output
    int32_t group;
    int32_t n_src;
    int8_t src_op[kMaxOps];
    // EMIT / DIGEST
    int32_t n_vars;
    int8_t head_word[kMaxVars];   // entry word of each head variable, -1 = the value bound here
};

enum Mode { M_COUNT = 0, M_DIGEST = 1, M_BITMAP = 2, M_EXPAND = 3, M_TMPW = 4, M_EMIT = 5, M_CELLS = 6 };
// How a step searches the operands it does not iterate: wave-cooperative LDS
// windows (the default), or one of the per-element methods of Section 5.
enum Search { SEARCH_WINDOW = 0, SEARCH_EXPONENTIAL = 1, SEARCH_QUADRATIC = 2, SEARCH_LINEAR = 3, SEARCH_BY_SIZE = 4 };
// modes that write every match at its rank (from the match words and their prefix)
constexpr bool mat_mode(int m) { return m == M_EXPAND || m == M_TMPW || m == M_EMIT; }

struct Seg {
    int32_t* seg;      // [2*n_ops][stride]: begin, end per operand
    int32_t* iter;     // operand iterated
    uint32_t* m;       // its length (0 if any operand is empty)
    int64_t stride;
};

// Sizes of one level in a device-sized launch sequence (a captured graph): each
// kernel reads the counts the one before it wrote, instead of the host reading
// them back between launches.
struct DevSizes {
    uint64_t n;          // entries of the level's frontier
    uint64_t total;      // elements of the level (the prefix sum of the entry lengths)
    uint64_t n_chunks;   // work-queue chunks of the next pass (0: the pass does nothing)
    uint64_t chunk_sz;   // elements per chunk
    uint64_t nw;         // match words of the bitmap pass
    uint64_t got;        // matches
    unsigned long long queue[8];   // per-XCD work-queue counters
    uint64_t pad[2];
};
static_assert(sizeof(DevSizes) == 128, "DevSizes is two 64-byte lines");

// Id predicate on the value bound by a step: the raw id (the key unmixed) must lie
// in the step's range and, for entries that carry one, in the entry's own range.
__device__ inline bool pred_ok(const KStep& S, const int32_t* ent, uint32_t key, const Mixer& mix) {
    const int64_t raw = (int64_t)unmix_key(key, mix);
    bool ok = raw >= S.pred_lo && raw < S.pred_hi;
    if (S.pred_word >= 0)
        ok = ok && raw >= (int64_t)(uint32_t)ent[S.pred_word] && raw <= (int64_t)(uint32_t)ent[S.pred_word + 1];
    return ok;
}

__device__ inline const uint32_t* op_array(const KData& D, const KOp& o) {
    if (o.kind == OP_V0) return D.atoms[o.atom].V[0];
    if (o.kind == OP_CHILD) return D.atoms[o.atom].V[o.lvl];
    return D.tmp_val[o.group];
}

// Per-cell match counts of one wave (M_CELLS).  Frontier entries are in cell order,
// so a wave sees long runs of one cell: it accumulates the run in a wave-uniform
// counter and issues one atomic per run, not one per match or per step.
struct CellAcc {
    uint32_t cell = 0xFFFFFFFFu;
    uint64_t n = 0;
};
__device__ inline void cell_flush(unsigned long long* cells, CellAcc& ca, int lane) {
    if (ca.n && lane == 0) atomicAdd(&cells[ca.cell], (unsigned long long)ca.n);
    ca.n = 0;
}
// Add n matches (wave-uniform) of one cell (wave-uniform).
__device__ inline void cell_add(unsigned long long* cells, CellAcc& ca, uint32_t cell, uint64_t n, int lane) {
    if (n == 0) return;
    if (cell != ca.cell) {
        cell_flush(cells, ca, lane);
        ca.cell = cell;
    }
    ca.n += n;
}
// Add one match per lane with found set, each of the lane's own cell cl.
__device__ inline void cell_add_lanes(unsigned long long* cells, CellAcc& ca, bool found, uint32_t cl, int lane) {
    const uint64_t bal = __ballot(found);
    if (bal == 0) return;
    const int lead = __ffsll((long long)bal) - 1;
    const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)__shfl(cl, lead, 64));
    const bool other = found && cl != c0;
    const uint64_t ob = __ballot(other);
    cell_add(cells, ca, c0, (uint64_t)__popcll(bal & ~ob), lane);
    if (other) atomicAdd(&cells[cl], 1ull);
}

__global__ void k_init_cells(int32_t* F, int64_t n, int W) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        F[e * W] = (int32_t)e;
        for (int w = 1; w < W; ++w) F[e * W + w] = 0;
    }
}

// Key ranges of a top level, one per coordinate value of a share 2^k.
__global__ void k_v0_ranges(const uint32_t* V0, int64_t l0, int b, int k, int2* out) {
    const int64_t ncoord = (int64_t)1 << k;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ncoord; s += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t lo = (uint64_t)s << (b - k), hi = (uint64_t)(s + 1) << (b - k);
        const int64_t a = lower_bound_u32(V0, 0, l0, (uint32_t)lo);
        const int64_t z = hi >= (1ull << 32) ? l0 : lower_bound_u32(V0, a, l0, (uint32_t)hi);
        out[s] = make_int2((int)a, (int)z);
    }
}

// For every top-level entry of a binary atom and every coordinate s of a share 2^k
// on its second variable: the first child whose key is >= s << (b-k); entry 2^k
// closes the list.  Row `node` of the table has 2^k + 1 entries.
__global__ void k_child_ranges(const int32_t* __restrict__ O0, const uint32_t* __restrict__ V1, int64_t l0, int b,
                               int k, int32_t* __restrict__ out) {
    const int64_t stride = ((int64_t)1 << k) + 1;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < l0 * stride;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = idx / stride, s = idx - node * stride;
        const int64_t beg = O0[node], end = O0[node + 1];
        if (s == stride - 1) out[idx] = (int32_t)end;
        else out[idx] = (int32_t)lower_bound_u32(V1, beg, end, (uint32_t)((uint64_t)s << (b - k)));
    }
}

// Range of a top-level operand for one entry: the whole level, or the key range of
// the coordinate (of a share, or of the segment) that the cell or an entry word names.
__device__ inline void v0_bounds(const KData& D, const KOp& op, const int32_t* ent, uint32_t cell, int64_t& beg,
                                 int64_t& end) {
    if (op.v0_range) {
        const uint32_t src = op.rng_word >= 0 ? (uint32_t)ent[op.rng_word] : cell;
        const int2 r = op.v0_range[(src >> op.rng_shift) & ((1u << op.rng_k) - 1u)];
        beg = r.x;
        end = r.y;
    } else {
        beg = 0;
        end = D.atoms[op.atom].len[0];
    }
}

// Resolve every operand of every entry to a [begin, end) range, restricted to the cell.
// n_dev, when set, holds the entry count instead of n (device-sized sequences).
__global__ __launch_bounds__(kBlock) void k_prep(KData D, KStep S, const int32_t* __restrict__ F, int64_t e0,
                                                 int64_t n, Seg G, const uint64_t* __restrict__ n_dev) {
    if (n_dev) n = (int64_t)*n_dev;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + t;
        const int32_t* ent = F + e * S.W_in;
        const uint32_t cell = (uint32_t)ent[0];
        const bool restrict_ = S.k_share > 0;
        const uint32_t coord = restrict_ ? (cell >> S.cell_shift) & ((1u << S.k_share) - 1u) : 0u;
        const uint64_t lo = (uint64_t)coord << (D.b - S.k_share);
        const uint64_t hi = (uint64_t)(coord + 1) << (D.b - S.k_share);
        uint32_t best_len = 0xFFFFFFFFu;
        int best = 0;
        bool empty = false;
        for (int o = 0; o < S.n_ops; ++o) {
            const KOp& op = S.ops[o];
            int64_t beg, end;
            if (op.kind == OP_V0) {
                v0_bounds(D, op, ent, cell, beg, end);
            } else if (op.kind == OP_CHILD) {
                const int32_t node = ent[op.word];
                const int32_t* O = D.atoms[op.atom].O[op.lvl - 1];
                beg = O[node];
                end = O[node + 1];
                if (restrict_ && op.child_range) {
                    const int32_t* cr = op.child_range + (int64_t)node * op.child_stride + coord;
                    beg = cr[0];
                    end = cr[1];
                } else if (restrict_) {
                    const uint32_t* A = D.atoms[op.atom].V[op.lvl];
                    const int64_t b2 = lower_bound_u32(A, beg, end, (uint32_t)lo);
                    end = hi >= (1ull << 32) ? end : lower_bound_u32(A, b2, end, (uint32_t)hi);
                    beg = b2;
                }
            } else {
                beg = ent[op.word];
                end = beg + ent[op.word + 1];
            }
            G.seg[(2 * o) * G.stride + e] = (int32_t)beg;
            G.seg[(2 * o + 1) * G.stride + e] = (int32_t)end;
            const uint32_t len = (uint32_t)(end - beg);
            if (len == 0) empty = true;
            if (len < best_len) {
                best_len = len;
                best = o;
            }
        }
        G.iter[e] = best;
        G.m[e] = empty ? 0u : best_len;
    }
}

// Largest e in [lo, hi) with prefix[e] <= g (prefix[lo] <= g is required).
__device__ inline int64_t find_entry(const uint64_t* __restrict__ prefix, int64_t lo, int64_t hi, uint64_t g) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ inline uint64_t fmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Probe {
    bool found;
    uint32_t a;
    int64_t e;
    int64_t pos[kMaxOps];
};

// Evaluate flattened element g: entry, value, and whether every operand holds it.
__device__ inline void probe_item(const KData& D, const KStep& S, const int32_t* F, const Seg& G,
                                  const uint64_t* prefix, int64_t e,
                                  uint64_t g, Probe& P) {
    P.e = e;
    const int it = G.iter[e];
    const int64_t ib = G.seg[(2 * it) * G.stride + e];
    const int64_t ipos = ib + (int64_t)(g - prefix[e]);
    const uint32_t a = op_array(D, S.ops[it])[ipos];
    P.a = a;
    bool found = true;
#pragma unroll
    for (int o = 0; o < kMaxOps; ++o) {
        if (o >= S.n_ops) break;
        if (o == it) {
            P.pos[o] = ipos;
            continue;
        }
        if (!found) continue;
        const uint32_t* arr = op_array(D, S.ops[o]);
        const int64_t beg = G.seg[(2 * o) * G.stride + e];
        const int64_t end = G.seg[(2 * o + 1) * G.stride + e];
        const int64_t p = lower_bound_u32(arr, beg, end, a);
        P.pos[o] = p;
        found = p < end && arr[p] == a;
    }
    if (found && S.has_pred) found = pred_ok(S, F + e * S.W_in, a, D.mix);
    P.found = found;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_probe(KData D, KStep S, const int32_t* __restrict__ F, Seg G,
                                                  const uint64_t* __restrict__ prefix, int64_t e_begin,
                                                  int64_t e_end, uint64_t item_begin, uint64_t n_items,
                                                  uint64_t* __restrict__ words, unsigned long long* acc,
                                                  unsigned long long* cells) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n_words = (int64_t)((n_items + 63) / 64);
    uint64_t cnt = 0, dsum = 0, dxor = 0;
    CellAcc ca;
    for (int64_t w = wave; w < n_words; w += nwaves) {
        const uint64_t rel = (uint64_t)w * 64 + lane;
        const bool valid = rel < n_items;
        const uint64_t g_first = item_begin + (uint64_t)w * 64;
        const uint64_t last_rel = ((uint64_t)w * 64 + 63 < n_items) ? (uint64_t)w * 64 + 63 : n_items - 1;
        const int64_t e_lo = find_entry(prefix, e_begin, e_end, g_first);
        const int64_t e_hi = find_entry(prefix, e_lo, e_end, item_begin + last_rel);
        Probe P;
        P.found = false;
        if (valid) {
            const uint64_t g = item_begin + rel;
            probe_item(D, S, F, G, prefix, find_entry(prefix, e_lo, e_hi + 1, g), g, P);
        }
        const uint64_t bal = __ballot(P.found);
        if (MODE == M_BITMAP) {
            if (lane == 0) words[w] = bal;
        } else {
            cnt += (uint64_t)__popcll(bal);
            if (MODE == M_CELLS)
                cell_add_lanes(cells, ca, P.found, P.found ? (uint32_t)F[P.e * S.W_in] >> D.cell_group : 0u, lane);
            if (MODE == M_DIGEST && P.found) {
                const int32_t* ent = F + P.e * S.W_in;
                uint64_t h = 0x6A09E667F3BCC909ull;
                for (int v = 0; v < S.n_vars; ++v) {
                    const int hw = S.head_word[v];
                    const uint32_t key = hw < 0 ? P.a : (uint32_t)ent[hw];
                    const uint64_t raw = (uint64_t)unmix_key(key, D.mix);
                    h = fmix64(h ^ (raw + (uint64_t)(v + 1) * 0x9E3779B97F4A7C15ull));
                }
                dsum += h;
                dxor ^= h;
            }
        }
    }
    if (MODE == M_CELLS) cell_flush(cells, ca, lane);
    if (MODE != M_BITMAP) {
        // cnt is wave-uniform (sum of ballots); digest terms are per lane
        if (MODE == M_DIGEST) {
            dsum = wave_sum(dsum);
            dxor = wave_xor(dxor);
        }
        if (lane == 0) {
            if (cnt) atomicAdd(&acc[0], (unsigned long long)cnt);
            if (MODE == M_DIGEST) {
                atomicAdd(&acc[1], (unsigned long long)dsum);
                atomicXor(&acc[2], (unsigned long long)dxor);
            }
        }
    }
}

struct MatOut {
    int32_t* F;            // next frontier
    uint32_t* tval;        // lifted intersection values
    int32_t* tsrc[kMaxOps];
    void* rows;            // emitted rows
    unsigned long long* cells;   // per-cell counts
    int64_t row_base, row_cap;
    // [n_ops][n_items] positions found in the probed operands, element by element:
    // the bitmap pass writes them, the materialising pass that follows reads them
    // instead of searching again (null: search)
    int32_t* pos;
};

// Write one match at its slot: a frontier entry (bound values, node indices of
// the atoms whose first variable was just bound, live temporary references), a
// lifted-intersection element with its source positions, or an output row.
__device__ inline void write_item(int mode, const KData& D, const KStep& S, const int32_t* ent, uint32_t a,
                                  const int64_t* pos, int64_t rank, const MatOut& out) {
    if (mode == M_EXPAND) {
        int32_t* o = out.F + rank * S.W_out;
        for (int c = 0; c < S.n_copy; ++c) o[S.copy_to[c]] = ent[S.copy_from[c]];
        o[S.val_word] = (int32_t)a;
        for (int t = 0; t < S.n_new; ++t) {
            const int op = S.new_op[t];
            const int64_t p = pos[op];
            o[S.new_word[t]] = S.ops[op].kind == OP_TMP ? D.tmp_src[S.ops[op].group][S.new_src[t]][p] : (int32_t)p;
        }
        for (int z = 0; z < S.n_zero; ++z) o[S.zero_word[z]] = 0;
    } else if (mode == M_TMPW) {
        out.tval[rank] = a;
        for (int t = 0; t < S.n_src; ++t) out.tsrc[t][rank] = (int32_t)pos[S.src_op[t]];
    } else {
        const int64_t row = out.row_base + rank;
        if (row < out.row_cap) {
            for (int v = 0; v < S.n_vars; ++v) {
                const int hw = S.head_word[v];
                const uint32_t key = hw < 0 ? a : (uint32_t)ent[hw];
                const uint32_t raw = unmix_key(key, D.mix);
                if (D.dtype64) ((int64_t*)out.rows)[row * S.n_vars + v] = (int64_t)raw;
                else ((int32_t*)out.rows)[row * S.n_vars + v] = (int32_t)raw;
            }
        }
    }
}

// ---------------------------------------------------------------- cursor-based intersection
// The deepest (hottest) level.  Each wave owns one contiguous range of the
// flattened elements, so it visits its entries in order and keeps, per entry,
// one cursor per probed operand.  While the next elements stay inside one entry
// they are consecutive elements of the iterated operand: the wave takes up to
// 4 x 64 of them at once (4 per lane, coalesced loads) and looks them up in
// every other operand.  A short operand list is staged whole in an LDS region
// and stays there while consecutive entries probe the same list (an operand
// bound at a shallower level repeats over long runs of entries).  A long one is
// searched from its cursor (the galloping search of Section 5, here 64-ary
// across the wave's lanes), the window that can hold the step's value range is
// staged in LDS with coalesced loads and searched there, and values beyond it
// are binary-searched in place.  Stretches where one 64-element chunk spans
// several small entries fall back to one search per lane.
constexpr int kWin = 1024;      // LDS window per wave (elements)
constexpr int kSub = 4;         // 64-element chunks per cursor step
constexpr int kTiny = 48;       // counting modes: entries shorter than this take the per-lane path
constexpr uint64_t kChunk = 4096;       // elements per work-queue chunk (one queue atomic each)
constexpr uint64_t kMinChunk = 256;     // smallest chunk, for launches with few elements
constexpr int kXcd = 8;                 // XCDs of an MI355X
constexpr uint64_t kPersistBlocks = 2048;   // 8 workgroups of 4 waves per CU: 8 waves per SIMD

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Load through the constant address space: a wave-uniform address then becomes a
// scalar load into SGPRs (no vector load, no readfirstlane).  Only for data that no
// kernel running concurrently writes (the step's prepared arrays).
template <class T>
__device__ inline T sload(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// First p in [c, end) with B[p] >= v (end if none), all 64 lanes cooperating: one
// probe of the 64 elements at the cursor, then 64-ary narrowing, so a long jump
// costs about log64 of its length in dependent loads (wave-uniform result).  Lanes
// past the end reload the last element instead of branching around their load.
__device__ inline uint64_t probe_lt(const uint32_t* __restrict__ Bc, int32_t n, uint32_t v, uint32_t lane4) {
    const uint32_t n4 = (uint32_t)((n < 64 ? n : 64) - 1) * 4u;   // n >= 1; only 64 lanes
    const uint32_t x = *(const uint32_t*)((const char*)Bc + (lane4 < n4 ? lane4 : n4));
    return __ballot(lane4 <= n4) & __ballot(x < v);   // ballots of single compares
}
__device__ inline int32_t wave_search(const uint32_t* __restrict__ B, int32_t c, int32_t end, uint32_t v,
                                      int lane) {
    if (c >= end) return c;
    const uint32_t lane4 = (uint32_t)lane * 4u;
    {
        const int k = __popcll(probe_lt(B + c, end - c, v, lane4));
        if (k < 64) return c + k;
    }
    int32_t lo = c + 64, hi = end;   // the answer lies in [lo, hi]
    while (hi - lo > 64) {
        const int32_t step = (hi - lo + 63) >> 6;
        const int32_t p = lo + lane * step;
        const bool lt = p < hi && B[p < hi ? p : hi - 1] < v;
        const int k = __popcll(__ballot(lt));
        if (k == 0) return lo;
        const int32_t nlo = lo + (k - 1) * step + 1;
        const int32_t nhi = lo + k * step < hi ? lo + k * step : hi;
        lo = nlo;
        hi = nhi;
    }
    if (lo >= hi) return lo;
    return lo + __popcll(probe_lt(B + lo, hi - lo, v, lane4));
}

// The same when the answer is expected about `hint` elements past c: the first round
// probes 64 positions hint/32 apart (the expected answer falls in the first half of
// them), then the found stride is searched as above.
__device__ inline int32_t wave_search_hint(const uint32_t* __restrict__ B, int32_t c, int32_t end, uint32_t v,
                                           int lane, uint32_t hint) {
    if (c >= end) return c;
    // stride: hint / 32, at most (end - c) / 63 + 1 (so c + 63 * st stays near end)
    const int32_t st = (int32_t)min(hint >> 5, (uint32_t)(end - c) / 63u + 1u);
    if (st <= 1) return wave_search(B, c, end, v, lane);
    const int32_t p = c + lane * st;
    const uint64_t in = __ballot(p < end);
    const uint64_t lt = __ballot(B[p < end ? p : end - 1] < v) & in;
    const int k = __popcll(lt);   // probes below v: a prefix of the lanes
    if (k == 0) return c;
    const int32_t lo = c + (k - 1) * st + 1;
    const int32_t hi = (k == 64 || c + k * st >= end) ? end : c + k * st;   // B[hi] >= v when hi < end
    return wave_search(B, lo, hi, v, lane);
}

// Stage B[base, base + len_al) in an LDS region with 16-byte loads (gfx950 takes
// them at any 4-byte-aligned address): the first sh slots are zeroed (they hold
// keys before the list's start, so the region stays sorted) and slots
// len_al .. p2-1 hold the largest key, which no searched value exceeds.
__device__ inline void stage_window(uint32_t* rw, const uint32_t* __restrict__ B, int32_t base, int32_t sh,
                                    int32_t len_al, int32_t p2, int lane) {
    // all loads first, then the LDS stores: the loads of one lane overlap
    constexpr int kMaxQ = 4;   // p2 <= 1024 keys = 4 x 64 lanes x 16 bytes
    const int nq = p2 >> 2;
    uint4 val[kMaxQ];
#pragma unroll
    for (int i = 0; i < kMaxQ; ++i) {
        const int k0 = 4 * (lane + 64 * i);
        val[i] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        if (k0 + 4 <= len_al) {
            __builtin_memcpy(&val[i], B + base + k0, 16);   // 16-byte load, any 4-byte-aligned base
        } else if (k0 < len_al) {
            val[i].x = B[base + k0];
            if (k0 + 1 < len_al) val[i].y = B[base + k0 + 1];
            if (k0 + 2 < len_al) val[i].z = B[base + k0 + 2];
        }
    }
#pragma unroll
    for (int i = 0; i < kMaxQ; ++i) {
        const int q = lane + 64 * i;
        if (q >= nq) continue;
        if (q == 0) {
            if (sh > 0) val[i].x = 0u;
            if (sh > 1) val[i].y = 0u;
            if (sh > 2) val[i].z = 0u;
        }
        *reinterpret_cast<uint4*>(rw + 4 * q) = val[i];
    }
}

// The same when B[base, base + p2) lies inside the list: the quads that hold the
// window are copied whole (the last one's extra elements are later elements of the
// list, no smaller than any searched value) and the rest of the p2 slots get the
// largest key, without the per-element tail handling.
__device__ inline void stage_window_inlist(uint32_t* rw, const uint32_t* __restrict__ B, int32_t base, int32_t sh,
                                           int32_t len_al, int32_t p2, int lane) {
    const uint4* src = reinterpret_cast<const uint4*>(B + base);
    uint4* dst = reinterpret_cast<uint4*>(rw);
    const int nl = (len_al + 3) >> 2;   // quads holding the window
    const int nq = p2 >> 2;
    uint4 val[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        val[i] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        if (lane + 64 * i < nl) val[i] = src[lane + 64 * i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (lane + 64 * i < nq) dst[lane + 64 * i] = val[i];
    if (lane < sh) rw[lane] = 0u;
}

// The same when all of B[base, base + p2) lies inside the list (p2 a power of two,
// 64 <= p2 <= 1024): it is copied whole, later list elements past the window being
// no smaller than any searched value; whole rows of 64 quads need no lane test.
__device__ inline void stage_full(uint32_t* rw, const uint32_t* __restrict__ B, int32_t base, int32_t sh, int32_t p2,
                                  int lane) {
    const uint32_t* src = B + base + 4 * lane;   // 16-byte loads at any 4-byte-aligned base
    uint4* dst = reinterpret_cast<uint4*>(rw);
    const int nq = p2 >> 2;
    uint4 v0, v1, v2, v3;
    if (nq >= 256) {
        __builtin_memcpy(&v0, src, 16);
        __builtin_memcpy(&v1, src + 256, 16);
        __builtin_memcpy(&v2, src + 512, 16);
        __builtin_memcpy(&v3, src + 768, 16);
        dst[lane] = v0;
        dst[lane + 64] = v1;
        dst[lane + 128] = v2;
        dst[lane + 192] = v3;
    } else if (nq == 128) {
        __builtin_memcpy(&v0, src, 16);
        __builtin_memcpy(&v1, src + 256, 16);
        dst[lane] = v0;
        dst[lane + 64] = v1;
    } else if (nq == 64 || lane < nq) {
        __builtin_memcpy(&v0, src, 16);
        dst[lane] = v0;
    }
    if (lane < sh) rw[lane] = 0u;
}

// nsc * rem_b / rem_a, approximately (a window size estimate: single precision is
// plenty), wave-uniform.
__device__ inline uint32_t est_cover(uint32_t nsc, uint32_t rem_b, uint32_t rem_a) {
    const float r = (float)rem_b * __builtin_amdgcn_rcpf((float)rem_a);
    const int32_t e = (int32_t)fminf((float)nsc * r, 1.0e9f);
    return (uint32_t)__builtin_amdgcn_readfirstlane(e);
}

// Largest e' in [e, e_end) with prefix[e'] <= g, given prefix[e] <= g: exponential
// search forward from e (the next entries are usually close).
__device__ inline int64_t advance_entry(const uint64_t* __restrict__ prefix, int64_t e, int64_t e_end, uint64_t g) {
    int64_t lo = e, step = 1;   // prefix[lo] <= g
    while (lo + step < e_end && prefix[lo + step] <= g) {
        lo += step;
        step <<= 1;
    }
    const int64_t hi = lo + step < e_end ? lo + step : e_end;
    return find_entry(prefix, lo, hi, g);
}

template <int MODE>
__device__ inline void digest_add(const KData& D, const KStep& S, const int32_t* ent, uint32_t a, uint64_t& dsum,
                                  uint64_t& dxor) {
    uint64_t h = 0x6A09E667F3BCC909ull;
    for (int v = 0; v < S.n_vars; ++v) {
        const int hw = S.head_word[v];
        const uint32_t key = hw < 0 ? a : (uint32_t)ent[hw];
        const uint64_t raw = (uint64_t)unmix_key(key, D.mix);
        h = fmix64(h ^ (raw + (uint64_t)(v + 1) * 0x9E3779B97F4A7C15ull));
    }
    dsum += h;
    dxor ^= h;
}

__device__ inline int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
// Smallest power of two >= max(x, lo) (lo a power of two, x <= 2^30): a count of
// leading zeros instead of a doubling loop.
__device__ inline int32_t pow2_at_least(int32_t x, int32_t lo) {
    return x <= lo ? lo : (int32_t)(1u << (32 - __builtin_clz((uint32_t)(x - 1))));
}

__device__ inline uint64_t uni64(uint64_t v) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32)) << 32) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
}

// Branch-free lower bounds of kSub values in one sorted LDS array of p2 (a power of
// two, at most 1024) keys.  Every level first issues the kSub reads, then compares,
// so the four searches' LDS latencies overlap instead of queueing one after another.
// The cursors are LDS pointers and the levels are unrolled, so each read takes its
// level's distance as the instruction's constant offset: a level costs a compare, a
// select and an add per value, with no address arithmetic.
typedef const __attribute__((address_space(3))) uint32_t* lds_cptr;   // 32-bit LDS address

template <int KS, int S>
__device__ inline void lds_level(int32_t p2, const uint32_t (&a)[KS], lds_cptr (&q)[KS]) {
    if (p2 < 2 * S) return;   // wave-uniform
    uint32_t x[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) x[k] = q[k][S - 1];
#pragma unroll
    for (int k = 0; k < KS; ++k) q[k] += x[k] < a[k] ? S : 0;
}

// p[k] is the lower bound of a[k] (p2 if every key is smaller) and x[k] the key at
// min(p[k], p2 - 1): the key at the lower bound whenever it lies in the window.
template <int KS>
__device__ inline void lds_search(const uint32_t* w, int32_t p2, const uint32_t (&a)[KS], int32_t (&p)[KS],
                                  uint32_t (&x)[KS]) {
    const lds_cptr w3 = (lds_cptr)w;
    lds_cptr q[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) q[k] = w3;
    lds_level<KS, 512>(p2, a, q);
    lds_level<KS, 256>(p2, a, q);
    lds_level<KS, 128>(p2, a, q);
    lds_level<KS, 64>(p2, a, q);
    lds_level<KS, 32>(p2, a, q);
    lds_level<KS, 16>(p2, a, q);
    lds_level<KS, 8>(p2, a, q);
    lds_level<KS, 4>(p2, a, q);
    lds_level<KS, 2>(p2, a, q);
    lds_level<KS, 1>(p2, a, q);
#pragma unroll
    for (int k = 0; k < KS; ++k) x[k] = q[k][0];
#pragma unroll
    for (int k = 0; k < KS; ++k) p[k] = (int32_t)(q[k] - w3) + (x[k] < a[k] ? 1 : 0);
}

__device__ inline int32_t lower_bound32(const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v) {
    while (l < h) {
        const int32_t mid = (l + h) >> 1;
        if (B[mid] < v) l = mid + 1; else h = mid;
    }
    return l;
}

// Lower bound of v in a sorted list given B[lo] = blo < v <= bhi = B[hi] (lo < hi):
// interpolation probes (the keys are hashed, so they spread evenly over the key
// range and the guess lands near the bound), each reading the 8 keys around its
// guess in one round trip, which usually hold the bound; near the array's start
// single-key probes narrow [lo, hi] instead and, once at most 4 keys remain, the up
// to 3 between lo and hi are read together and counted.  Returns the bound and, in
// key, the key there (bhi when it is hi).
__device__ inline int32_t interp_lb_between(const uint32_t* __restrict__ B, int32_t lo, uint32_t blo, int32_t hi,
                                            uint32_t bhi, uint32_t v, uint32_t& key) {
    {
        // 8 keys per probe (two unaligned 16-byte loads in one round trip): a window
        // [s, s + 8) inside [0, hi] around the interpolated position, or ending at hi
        // once it covers every key between lo and hi (slots up to lo then belong to
        // another list and count as below).  The keys below the value in it give the
        // bound unless they are none (bound below s) or all (bound above s + 7) of a
        // window that does not reach lo or hi.  Every window starts at or above 0: a
        // window below the value lowers hi, and the windows stop once hi is below 8.
#pragma unroll 1
        for (int it = 0; it < 8 && hi - lo > 1 && hi >= 8; ++it) {   // (hi drops on a window below)
            int32_t s = hi - 8;
            if (hi - lo > 9) {
                const float f = (float)(v - blo) * __builtin_amdgcn_rcpf((float)(bhi - blo));
                const int32_t p = lo + (int32_t)(f * (float)(hi - lo));
                s = min(max(p - 4, lo + 1), hi - 8);
            }
            uint4 w0, w1;
            __builtin_memcpy(&w0, B + s, 16);
            __builtin_memcpy(&w1, B + s + 4, 16);
            const uint32_t k[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
            int32_t c = 0;
#pragma unroll
            for (int t = 0; t < 8; ++t) c += (s + t <= lo || k[t] < v) ? 1 : 0;
            const bool below = c == 0 && s > lo + 1;
            const bool above = c == 8 && s + 8 < hi;
            if (!below && !above) {
                uint32_t kc = bhi;   // c = 8: the bound is hi
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (t == c) kc = k[t];
                key = kc;
                return s + c;
            }
            if (below) {
                hi = s;
                bhi = k[0];
            } else {
                lo = s + 7;
                blo = k[7];
            }
        }
        if (hi - lo == 1) {
            key = bhi;
            return hi;
        }
    }
#pragma unroll 1
    for (int it = 0; it < 8 && hi - lo > 4; ++it) {
        const float f = (float)(v - blo) * __builtin_amdgcn_rcpf((float)(bhi - blo));
        int32_t p = lo + (int32_t)(f * (float)(hi - lo));
        p = min(max(p, lo + 1), hi - 1);
        const uint32_t bp = B[p];
        if (bp < v) {
            lo = p;
            blo = bp;
        } else {
            hi = p;
            bhi = bp;
        }
    }
    if (hi - lo > 4) {   // (keys far from even: finish by bisection)
        const int32_t q = lower_bound32(B, lo + 1, hi, v);
        key = q < hi ? B[q] : bhi;
        return q;
    }
    // positions lo+1 .. lo+3 clamped to hi (whose key is known to be >= v)
    const uint32_t k1 = lo + 1 < hi ? B[lo + 1] : bhi;
    const uint32_t k2 = lo + 2 < hi ? B[lo + 2] : bhi;
    const uint32_t k3 = lo + 3 < hi ? B[lo + 3] : bhi;
    const int32_t nb = (k1 < v ? 1 : 0) + (k2 < v ? 1 : 0) + (k3 < v ? 1 : 0);
    key = nb == 0 ? k1 : (nb == 1 ? k2 : (nb == 2 ? k3 : bhi));
    return min(lo + 1 + nb, hi);
}

// First p in [l, h) with B[p] >= v (h if none) by interpolation from the range's
// ends; key receives B[p] when p < h.
__device__ inline int32_t interp_lb(const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v, uint32_t& key) {
    if (l >= h) return l;
    const uint32_t b0 = B[l], b1 = B[h - 1];
    key = b0;
    if (v <= b0) return l;
    if (v > b1) return h;
    return interp_lb_between(B, l, b0, h - 1, b1, v, key);
}

// ---- the per-element search methods of Section 5 (one search per lane), each
// returning the first p in [l, h) with B[p] >= v (h if none):
//   exponential: jumps of 1, 2, 4, ... from l until one overshoots, then binary search;
//   quadratic:   fixed jumps of 32 elements (one 128-byte line) from l, applied at two
//                levels (32 lines, then one line), then a scan of the last line;
//   linear:      a scan from l.
// SEARCH_BY_SIZE picks linear / quadratic / exponential from the candidate range's
// length (at most 32, at most 4096, more), the size-based reading of Section 5.
__device__ inline int32_t exp_search32(const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v) {
    if (l >= h || B[l] >= v) return l;
    int32_t lo = l, step = 1;   // B[lo] < v
    while (lo + step < h && B[lo + step] < v) {
        lo += step;
        step <<= 1;
    }
    return lower_bound32(B, lo + 1, lo + step < h ? lo + step : h, v);
}
__device__ inline int32_t quad_search32(const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v) {
    constexpr int32_t kLine = 32, kBig = 32 * kLine;
    int32_t p = l;   // invariant: every position below p holds a value < v
    while (p + kBig < h && B[p + kBig - 1] < v) p += kBig;
    while (p + kLine < h && B[p + kLine - 1] < v) p += kLine;
    while (p < h && B[p] < v) ++p;
    return p;
}
__device__ inline int32_t lin_search32(const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v) {
    while (l < h && B[l] < v) ++l;
    return l;
}
__device__ inline int32_t lane_search(int method, const uint32_t* __restrict__ B, int32_t l, int32_t h, uint32_t v) {
    if (method == SEARCH_BY_SIZE) method = h - l <= 32 ? SEARCH_LINEAR : (h - l <= 4096 ? SEARCH_QUADRATIC
                                                                                      : SEARCH_EXPONENTIAL);
    if (method == SEARCH_LINEAR) return lin_search32(B, l, h, v);
    if (method == SEARCH_QUADRATIC) return quad_search32(B, l, h, v);
    if (method == SEARCH_EXPONENTIAL) return exp_search32(B, l, h, v);
    return lower_bound32(B, l, h, v);
}

// SM = 0: the window method only (the default; the per-element methods are compiled
// out, which keeps their registers out of the hot loop); SM = 1: the method S.search.
// DEV: the entry and element counts, the chunk count and size come from dsz (a
// device-sized sequence) instead of the arguments.
template <int MODE, int NOPS, int SM, bool DEV = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_probe2(KData D, KStep S, const int32_t* __restrict__ F, Seg G,
                                                   const uint64_t* __restrict__ prefix, int64_t e_begin,
                                                   int64_t e_end, uint64_t item_begin, uint64_t n_items,
                                                   const int64_t* __restrict__ chunk_entry,
                                                   unsigned long long* queue, uint64_t n_chunks, uint32_t chunk_sz,
                                                   uint64_t* __restrict__ words, unsigned long long* acc,
                                                   const uint64_t* __restrict__ wprefix, MatOut out,
                                                   const DevSizes* __restrict__ dsz = nullptr) {
    if constexpr (DEV) {
        e_end = (int64_t)sload(&dsz->n);
        n_items = sload(&dsz->total);
        n_chunks = sload(&dsz->n_chunks);
        chunk_sz = (uint32_t)sload(&dsz->chunk_sz);
    }
    constexpr bool kMat = mat_mode(MODE);
    constexpr bool kPos = kMat || MODE == M_BITMAP;   // positions in the probed operands are needed
    const int search = SM ? S.search : (int)SEARCH_WINDOW;
    __shared__ __attribute__((aligned(16))) uint32_t win_all[kWaves][kWin];
    __shared__ uint64_t ps_all[kWaves][64];   // entry starts of a per-lane chunk
    const int lane = threadIdx.x & 63;
    const uint32_t lane4 = (uint32_t)lane * 4u;
    uint32_t* win = win_all[threadIdx.x >> 6];
    // Counting with two operands: every entry is rearranged so that operand 0 is the
    // one it iterates (arrays, ranges and cursors swapped), which makes the roles
    // static in the step.  arr0 keeps the operands in plan order.
    constexpr bool kCanon = NOPS == 2 && (MODE == M_COUNT || MODE == M_DIGEST || MODE == M_CELLS);
    const uint32_t* arr0[NOPS];
    const uint32_t* arr[NOPS];
#pragma unroll
    for (int o = 0; o < NOPS; ++o) arr[o] = arr0[o] = op_array(D, S.ops[o]);
    const int64_t stride = G.stride;
    uint64_t cnt = 0, dsum = 0, dxor = 0;
    CellAcc ca;
    // Work queue per XCD: workgroups are dispatched to the 8 XCDs round-robin, so
    // blockIdx % 8 names the XCD; each XCD sweeps its own contiguous eighth of the
    // chunks in order, which keeps the few HyperCube cells it works on at a time
    // (and their slices of the CoCo arrays) resident in its L2.  Every wave leaves
    // once its XCD's queue is exhausted.
    // LDS-resident operand lists (per operand region): array, begin, end
    const uint32_t* wc_ptr[NOPS];
    int32_t wc_beg[NOPS], wc_end[NOPS];
#pragma unroll
    for (int o = 0; o < NOPS; ++o) {
        wc_ptr[o] = nullptr;
        wc_beg[o] = wc_end[o] = 0;
    }
    const int xcd = (int)(blockIdx.x % kXcd);
    const uint64_t c_lo = n_chunks * (uint64_t)xcd / kXcd, c_hi = n_chunks * (uint64_t)(xcd + 1) / kXcd;
    // A wave whose rank among its XCD's waves reaches the XCD's chunk count would find
    // the queue empty: it leaves without claiming (a device-sized launch always runs
    // the full grid, and idle waves contending on the queue counters cost more than
    // the small launch's work).  The waves that stay claim until the queue is empty.
    if ((uint64_t)(blockIdx.x / kXcd) * kWaves + (threadIdx.x >> 6) >= c_hi - c_lo) return;
    for (;;) {
        unsigned long long t = 0;
        int stop = 0;
        if (lane == 0) {
            t = atomicAdd(&queue[xcd], 1ull);
            // The cancel word is host memory: the wave that takes every 64th chunk of an
            // XCD's queue reads it (a small launch reads it a few times, not once per
            // wave).  A wave that finds it raised pushes every queue 2^40 chunks on, so
            // that all waves leave at their next claim.
            if ((t & 63) == 0 && __atomic_load_n(D.cancel, __ATOMIC_RELAXED)) {
                stop = 1;
                for (int x = 0; x < kXcd; ++x) atomicAdd(&queue[x], 1ull << 40);
            }
        }
        if (uni(stop)) break;
        const uint64_t c = c_lo + uni64(t);
        if (c >= c_hi) break;
        const uint64_t r_begin = c * chunk_sz;
        // Positions inside the chunk are 32-bit offsets from its first item (uniform
        // 64-bit compares would cost vector instructions); so are the bounds of the
        // current entry, [lo_rel, hi_rel), the upper one clamped far beyond the chunk.
        const uint64_t base = item_begin + r_begin;
        const uint32_t n_c = (uint32_t)(r_begin + chunk_sz < n_items ? chunk_sz : n_items - r_begin);
        // current entry and its wave-uniform description
        int64_t e = sload(chunk_entry + c);
        int32_t lo_rel;
        uint32_t hi_rel;
        int it;
        int32_t beg[NOPS], end[NOPS], cur[NOPS];
        auto canon = [&]() {
            if constexpr (kCanon) {
                const bool sw = it == 1;
                arr[0] = sw ? arr0[1] : arr0[0];
                arr[1] = sw ? arr0[0] : arr0[1];
                if (sw) {
                    const int32_t tb = beg[0], te = end[0];
                    beg[0] = beg[NOPS - 1];
                    end[0] = end[NOPS - 1];
                    beg[NOPS - 1] = tb;
                    end[NOPS - 1] = te;
                    cur[0] = beg[0];
                    cur[NOPS - 1] = beg[NOPS - 1];
                }
                it = 0;
            }
        };
        auto load_entry = [&](int64_t ee) {
            lo_rel = (int32_t)(int64_t)(sload(prefix + ee) - base);   // > -2^31: one entry's length
            const uint64_t d1 = sload(prefix + ee + 1) - base;
            const uint32_t big = (uint32_t)(d1 >> 32) != 0u ? 0xFFFFFFFFu : 0u;   // 32-bit ops only
            hi_rel = min((uint32_t)d1 | big, 0x7FFFFFFFu);
            it = sload(G.iter + ee);
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                beg[o] = sload(G.seg + (2 * o) * stride + ee);
                end[o] = sload(G.seg + (2 * o + 1) * stride + ee);
                cur[o] = beg[o];
            }
            canon();
        };
        load_entry(e);
        uint32_t rc = 0;
        while (rc < n_c) {
            const uint64_t g = base + rc;
            if (hi_rel <= rc) {   // move to the entry holding g: usually the next one
                int64_t ne = e + 1;   // ne < e_end, since g < prefix[e_end]
                if (sload(prefix + ne + 1) <= g) ne = (int64_t)advance_entry(prefix, ne + 1, e_end, g);
                e = ne;
                load_entry(e);
            }
            const uint32_t left_wave = n_c - rc;
            const uint32_t left_entry = hi_rel - rc;
            const uint32_t chunk = left_wave < 64 ? left_wave : 64;
            // Modes that write match words keep every step on 64-element boundaries;
            // counting modes let a step end where its entry ends, so only runs of tiny
            // entries take the per-lane path.
            constexpr bool kAligned = !(MODE == M_COUNT || MODE == M_DIGEST || MODE == M_CELLS);
            bool uniform_step;
            uint32_t n_sc;
            if (kAligned) {
                uniform_step = left_entry >= chunk;
                n_sc = left_entry >= left_wave ? left_wave : (left_entry & ~63u);
            } else {
                uniform_step = left_entry >= (uint32_t)kTiny || left_entry >= left_wave;
                n_sc = left_entry < left_wave ? left_entry : left_wave;
            }
            if (uniform_step) {
                // ---- uniform step: up to kSub*64 elements of entry e
                if (n_sc > 64u * kSub) n_sc = 64u * kSub;
                const int nsc = (int)n_sc;
                const int itc = kCanon ? 0 : it;   // the iterated operand
                const int32_t off0 = (int32_t)rc - lo_rel;
                // the step's elements: one uniform base and lane offsets, clamped to the
                // step's last element (lanes past it reload that one: no branches)
                const uint32_t* ab = arr[itc] + (beg[itc] + off0);
                const int last = nsc - 1;
                const uint32_t last4 = (uint32_t)last * 4u;
                uint32_t a[kSub];
                bool v[kSub];
                // match masks, one bit per lane and block: each test below ANDs in the
                // ballot of one compare (a ballot of a plain compare costs nothing more)
                uint64_t fm[kSub];
                int32_t pos[NOPS][kSub];   // absolute positions (materialising modes)
#pragma unroll
                for (int k = 0; k < kSub; ++k) {
                    const int j = k * 64 + lane;
                    v[k] = j < nsc;
                    fm[k] = __ballot(v[k]);   // one vector compare, no scalar mask arithmetic
                    const uint32_t o4 = lane4 + 256u * k;
                    a[k] = *(const uint32_t*)((const char*)ab + (o4 < last4 ? o4 : last4));
#pragma unroll
                    for (int o = 0; o < NOPS; ++o) pos[o][k] = beg[o] + off0 + j;
                }
                const uint64_t r0 = r_begin + rc;   // the step's first element, relative to the launch
                if (kMat && out.pos != nullptr) {
                    // the bitmap pass left every element's match bit and its positions in
                    // the probed operands: write the matches without searching
#pragma unroll
                    for (int k = 0; k < kSub; ++k) {
                        if (64 * k >= nsc) break;
                        const uint64_t bal = sload(words + (r0 >> 6) + k);
                        if ((bal >> lane) & 1ull) {
                            int64_t pp[NOPS];
#pragma unroll
                            for (int o = 0; o < NOPS; ++o)
                                pp[o] = o == itc ? pos[o][k] : out.pos[(size_t)o * n_items + r0 + 64 * k + lane];
                            const int64_t rank =
                                (int64_t)(wprefix[(r0 >> 6) + k] + (uint64_t)__popcll(bal & lanemask_lt()));
                            write_item(MODE, D, S, F + e * S.W_in, a[k], pp, rank, out);
                        }
                    }
                    rc += n_sc;
                    continue;
                }
#pragma unroll
                for (int o = 0; o < NOPS; ++o) {
                    if (o == itc) continue;
                    const uint32_t* B = arr[o];
                    const int32_t full = end[o] - beg[o];
                    // ---- short operand: its whole list sits in this operand's LDS region,
                    // kept across steps and entries while the list stays the same (the
                    // deepest level's entries come in key order, so an operand bound at a
                    // shallower level repeats over long runs of entries)
                    constexpr int kReg = NOPS <= 2 ? kWin : kWin / 4;
                    uint32_t* rw = win + (NOPS <= 2 ? 0 : o * kReg);
                    if (search != SEARCH_WINDOW) {
                        // ---- one search per element (Section 5's methods) from the cursor
                        int32_t q[kSub];
#pragma unroll
                        for (int k = 0; k < kSub; ++k) {
                            q[k] = v[k] ? lane_search(search, B, cur[o], end[o], a[k]) : cur[o];
                            const int32_t qc = q[k] < end[o] ? q[k] : end[o] - 1;   // end > cur here
                            fm[k] &= __ballot(q[k] < end[o]) & __ballot(B[qc] == a[k]);
                            if (kPos) pos[o][k] = q[k];
                        }
                        int32_t ql = cur[o];
#pragma unroll
                        for (int k = 0; k < kSub; ++k) {
                            const int32_t t = __shfl(q[k], last & 63, 64);
                            if (k == (last >> 6)) ql = t;
                        }
                        cur[o] = uni(ql);   // lower bound of the step's last element
                        continue;
                    }
                    if (full <= kReg - 4) {
                        const int32_t base = beg[o] & ~3;
                        const int32_t sh = beg[o] - base;
                        const int32_t len_al = full + sh;
                        const int32_t p2 = pow2_at_least(len_al, 4);
                        if (!(wc_ptr[o] == B && wc_beg[o] == beg[o] && wc_end[o] == end[o])) {
                            wave_sync();   // earlier searches of this region are done
                            stage_window(rw, B, base, sh, len_al, p2, lane);
                            wave_sync();
                            if (NOPS <= 2) {   // one region shared by both operands
#pragma unroll
                                for (int u = 0; u < NOPS; ++u) wc_ptr[u] = nullptr;
                            }
                            wc_ptr[o] = B;
                            wc_beg[o] = beg[o];
                            wc_end[o] = end[o];
                        }
                        int32_t p[kSub];
                        uint32_t x[kSub];
                        const uint32_t w_sh = rw[sh];   // the list's first key (off the search's path)
                        lds_search<kSub>(rw, p2, a, p, x);
#pragma unroll
                        for (int k = 0; k < kSub; ++k) {
                            // slots below sh hold zeros: a lower bound there moves up to sh, whose
                            // key is the list's first; elsewhere the search read the bound's key
                            const int32_t pc = min(max(p[k], sh), p2 - 1);
                            const uint32_t xk = p[k] < sh ? w_sh : x[k];
                            fm[k] &= __ballot(pc < len_al) & __ballot(xk == a[k]);
                            if (kPos) pos[o][k] = base + pc;
                        }
                        continue;
                    }
                    // ---- long operand: the lower bounds of the step's values a_first .. a_last
                    // lie in [cursor, lower bound of a_last].  Keys are hashed, so they spread
                    // over about est = nsc * (rest of B) / (rest of the iterated list) elements
                    // from the cursor: that many, with a margin, are staged in LDS from the
                    // cursor without searching for the range's end, and the step searches
                    // there.  When the estimate exceeds the region, every s-th element of the
                    // estimated cover is staged instead (fences, s = cover / region), the step
                    // searches the fences and each value finishes with a search of its
                    // s-element bucket in place.  When the staged window or fences end below
                    // a_last (an overshoot), the range is found by two wave searches from the
                    // cursor (the second starting with strides sized by est) and staged when
                    // it fits, else fenced.
#pragma unroll
                    for (int u = 0; u < NOPS; ++u) wc_ptr[u] = nullptr;   // the window overwrites every region
                    const uint32_t a_first = sload(ab), a_last = sload(ab + last);
                    const uint32_t est = est_cover((uint32_t)nsc, (uint32_t)(end[o] - cur[o]), hi_rel - rc);
                    {
                        // the window starts at the cursor itself (unaligned 16-byte loads): every
                        // value's lower bound is at or past it, so no slot precedes the first key
                        const int32_t ws = cur[o];
                        const uint32_t want = est + (est >> 2) + 32u;
                        if (want <= (uint32_t)kWin) {
                            const int32_t P = pow2_at_least((int32_t)want, 64);
                            const bool to_end = ws + P >= end[o];
                            const int32_t len_al = to_end ? end[o] - ws : P;
                            if (!to_end)
                                stage_full(win, B, ws, 0, P, lane);
                            else
                                stage_window(win, B, ws, 0, len_al, P, lane);
                            wave_sync();
                            // (the LDS word is the same for every lane: read it as a uniform value, so
                            // that the branch and the cursor stay scalar)
                            if (to_end || (uint32_t)uni((int32_t)win[P - 1]) >= a_last) {
                                int32_t p[kSub];
                                uint32_t x[kSub];   // the key at each bound (padding past the list's end)
                                lds_search<kSub>(win, P, a, p, x);
                                int32_t pl = 0;
#pragma unroll
                                for (int k = 0; k < kSub; ++k) {
                                    fm[k] &= __ballot(p[k] < len_al) & __ballot(x[k] == a[k]);
                                    if (kPos) pos[o][k] = ws + min(p[k], P - 1);
                                    if (k == (last >> 6)) pl = __builtin_amdgcn_readlane(p[k], last & 63);
                                }
                                wave_sync();
                                cur[o] = ws + pl;   // lower bound of the step's last value
                                continue;
                            }
                            wave_sync();
                        }
                    }
                    if (est + (est >> 2) + 32u > (uint32_t)kWin) {
                        // estimated fences: nf fences s apart from the cursor over the
                        // estimated cover (capped at the list's end, where the last bucket
                        // then reaches the end)
                        const uint32_t left_b = (uint32_t)(end[o] - cur[o]);
                        const uint32_t want = min(est + (est >> 2) + 32u, left_b);
                        const bool capped = want == left_b;
                        const int32_t sp = uni((int32_t)((want + (uint32_t)kWin - 1u) / (uint32_t)kWin));
                        const int32_t nf = uni((int32_t)((want + (uint32_t)sp - 1u) / (uint32_t)sp));   // <= kWin
                        const int32_t p2 = pow2_at_least(nf, 4);
                        const int32_t c0 = cur[o], e_o = end[o];
                        {   // fence loads first, then the LDS stores; (nf - 1) * sp < want <= end - cursor
                            uint32_t fv[16];
#pragma unroll
                            for (int i = 0; i < 16; ++i) {
                                const int q = lane + 64 * i;
                                fv[i] = q < nf ? B[c0 + q * sp] : 0xFFFFFFFFu;
                            }
#pragma unroll
                            for (int i = 0; i < 16; ++i)
                                if (lane + 64 * i < p2) win[lane + 64 * i] = fv[i];
                        }
                        wave_sync();
                        if (capped || (uint32_t)uni((int32_t)win[nf - 1]) >= a_last) {
                            int32_t p[kSub];
                            uint32_t xf[kSub];   // the key of fence p[k] when p[k] < nf
                            lds_search<kSub>(win, p2, a, p, xf);   // p[k]: fences below the value (<= nf)
                            bool hit[kSub];
                            if (NOPS <= 3 && sp <= 5) {   // (4-operand levels keep their registers)
                                // buckets of at most 4 keys: one 16-byte load of the 4 keys from
                                // max(r - 4, 0), r the bucket's end (est <= the keys left in the
                                // list, so more than 790 keys precede the list's end and the 4 lie
                                // in the array; only keys in the bucket [l, r) are counted), the
                                // lower bound is l plus the bucket keys below the value, and a bound
                                // at r, fence p, has that fence's key
#pragma unroll
                                for (int k = 0; k < kSub; ++k) {
                                    int32_t q = c0;
                                    bool h = p[k] == 0 && xf[k] == a[k];   // the cursor's key is fence 0
                                    if (p[k] > 0) {
                                        const int32_t l = c0 + (p[k] - 1) * sp + 1;
                                        const int32_t r = c0 + p[k] * sp < e_o ? c0 + p[k] * sp : e_o;
                                        const int32_t s4 = r >= 4 ? r - 4 : 0;
                                        uint4 qd;
                                        __builtin_memcpy(&qd, B + s4, 16);
                                        const uint32_t kv[4] = {qd.x, qd.y, qd.z, qd.w};
                                        int32_t nb = 0;
#pragma unroll
                                        for (int t = 0; t < 4; ++t)
                                            nb += (s4 + t >= l && s4 + t < r && kv[t] < a[k]) ? 1 : 0;
                                        q = l + nb;
                                        uint32_t kq = kv[3];
#pragma unroll
                                        for (int t = 0; t < 3; ++t)
                                            if (s4 + t == q) kq = kv[t];
                                        h = q < r ? kq == a[k] : (r < e_o && xf[k] == a[k]);
                                    }
                                    p[k] = q;
                                    hit[k] = h;
                                }
                            } else {
#pragma unroll
                                for (int k = 0; k < kSub; ++k) {
                                    int32_t q = c0;   // every value's lower bound is at or past the cursor
                                    bool have = false;   // the bound's key is known
                                    uint32_t kq = 0;
                                    if (v[k] && p[k] > 0) {
                                        // between fence p - 1 (key below the value) and fence p
                                        // (key xf, at least the value) when that one exists
                                        const int32_t l = c0 + (p[k] - 1) * sp + 1;
                                        if (NOPS <= 3 && SM == 0 && p[k] < nf) {
                                            q = interp_lb_between(B, l - 1, win[p[k] - 1], c0 + p[k] * sp, xf[k], a[k],
                                                                  kq);
                                            have = true;
                                        } else {
                                            q = lower_bound32(B, l, c0 + p[k] * sp < e_o ? c0 + p[k] * sp : e_o, a[k]);
                                        }
                                    }
                                    if (have) {
                                        hit[k] = kq == a[k];
                                    } else {
                                        const int32_t qc = q < e_o ? q : e_o - 1;
                                        hit[k] = q < e_o && B[qc] == a[k];
                                    }
                                    p[k] = q;
                                }
                            }
                            int32_t ql = c0;
#pragma unroll
                            for (int k = 0; k < kSub; ++k) {
                                fm[k] &= __ballot(hit[k]);
                                if (kPos) pos[o][k] = p[k];
                                if (k == (last >> 6)) ql = __builtin_amdgcn_readlane(p[k], last & 63);
                            }
                            wave_sync();
                            cur[o] = ql;   // lower bound of the step's last value
                            continue;
                        }
                        wave_sync();
                    }
                    const int32_t lo = uni(wave_search(B, cur[o], end[o], a_first, lane));
                    const int32_t hi = uni(wave_search_hint(B, lo, end[o], a_last, lane, est));
                    const int32_t cover = (hi < end[o] ? hi + 1 : end[o]) - lo;
                    if (cover <= kWin - 4) {
                        // The window starts at the 16-byte boundary below lo (16-byte
                        // loads); its first sh slots hold zero so that it stays sorted and
                        // positions below sh are never reported.  It is padded to a power
                        // of two with the largest key, never below a searched value.
                        const int32_t lo_al = lo & ~3;
                        const int32_t sh = lo - lo_al;
                        const int32_t len_al = cover + sh;
                        const int32_t p2 = pow2_at_least(len_al, 4);
                        if (lo_al + p2 <= end[o])
                            stage_window_inlist(win, B, lo_al, sh, len_al, p2, lane);
                        else
                            stage_window(win, B, lo_al, sh, len_al, p2, lane);
                        wave_sync();
                        int32_t p[kSub];
                        uint32_t x[kSub];
                        const uint32_t w_sh = win[sh];   // the key at lo
                        lds_search<kSub>(win, p2, a, p, x);   // all kSub searches advance together
#pragma unroll
                        for (int k = 0; k < kSub; ++k) {
                            const int32_t pc = min(max(p[k], sh), p2 - 1);
                            const uint32_t xk = p[k] < sh ? w_sh : x[k];
                            fm[k] &= __ballot(pc < len_al) & __ballot(xk == a[k]);
                            if (kPos) pos[o][k] = lo_al + pc;
                        }
                    } else {
                        const int32_t sp = (cover + (kWin - 4) - 1) / (kWin - 4);   // fence spacing
                        const int32_t nf = (cover + sp - 1) / sp;
                        const int32_t p2 = pow2_at_least(nf, 4);
                        {   // fence loads first, then the LDS stores (p2 <= 1024 = 16 x 64 lanes)
                            uint32_t fv[16];
#pragma unroll
                            for (int i = 0; i < 16; ++i) {
                                const int q = lane + 64 * i;
                                fv[i] = q < nf ? B[lo + q * sp] : 0xFFFFFFFFu;
                            }
#pragma unroll
                            for (int i = 0; i < 16; ++i)
                                if (lane + 64 * i < p2) win[lane + 64 * i] = fv[i];
                        }
                        wave_sync();
                        int32_t p[kSub];
                        uint32_t xf[kSub];
                        lds_search<kSub>(win, p2, a, p, xf);   // p[k]: fences below the value
#pragma unroll
                        for (int k = 0; k < kSub; ++k) {
                            int32_t q = lo;
                            if (v[k] && p[k] > 0) {
                                const int32_t l = lo + (p[k] - 1) * sp + 1;
                                const int32_t r = lo + p[k] * sp < end[o] ? lo + p[k] * sp : end[o];
                                q = lower_bound32(B, l, r, a[k]);
                            }
                            const int32_t qc = q < end[o] ? q : end[o] - 1;
                            fm[k] &= __ballot(q < end[o]) & __ballot(B[qc] == a[k]);
                            if (kPos) pos[o][k] = q;
                        }
                    }
                    wave_sync();
                    cur[o] = hi;   // lower bound of the step's last value
                }
                if (MODE == M_BITMAP && out.pos != nullptr) {
#pragma unroll
                    for (int k = 0; k < kSub; ++k)
                        if (v[k]) {
#pragma unroll
                            for (int o = 0; o < NOPS; ++o)
                                if (o != itc) out.pos[(size_t)o * n_items + r0 + 64 * k + lane] = (int32_t)pos[o][k];
                        }
                }
#pragma unroll
                for (int k = 0; k < kSub; ++k) {
                    if (S.has_pred) fm[k] &= __ballot(pred_ok(S, F + e * S.W_in, a[k], D.mix));
                    const uint64_t bal = fm[k];
                    const bool hit = (bal >> lane) & 1ull;
                    if (kMat) {
                        if (hit) {
                            int64_t pp[NOPS];
#pragma unroll
                            for (int o = 0; o < NOPS; ++o) pp[o] = pos[o][k];
                            const int64_t rank =
                                (int64_t)(wprefix[((r_begin + rc) >> 6) + k] + (uint64_t)__popcll(bal & lanemask_lt()));
                            write_item(MODE, D, S, F + e * S.W_in, a[k], pp, rank, out);
                        }
                    } else if (MODE == M_BITMAP) {
                        if (lane == 0 && k * 64 < nsc) words[((r_begin + rc) >> 6) + k] = bal;
                    } else {
                        cnt += (uint64_t)__popcll(bal);
                        if (MODE == M_DIGEST && hit) digest_add<MODE>(D, S, F + e * S.W_in, a[k], dsum, dxor);
                        if (MODE == M_CELLS)
                            cell_add(out.cells, ca, (uint32_t)uni(F[e * S.W_in]) >> D.cell_group,
                                     (uint64_t)__popcll(bal), lane);
                    }
                }
                rc += n_sc;
            } else {
                // ---- mixed chunk: 64 elements spanning several entries, one search per lane
                const int nv = (int)chunk;
                const bool valid = lane < nv;
                const uint64_t g_last = g + chunk - 1;
                // The starts of entries e .. e+63, one per lane (one coalesced load), go to
                // LDS; every lane finds its entry there.  The 64 elements span at most 64
                // non-empty entries, but empty ones in between can push the span further:
                // then the entries are found by searches in the prefix array.
                uint64_t* ps = ps_all[threadIdx.x >> 6];
                {
                    const int64_t ej = e + lane;
                    ps[lane] = ej <= e_end ? prefix[ej] : ~0ull;
                }
                wave_sync();
                const bool in_lds = uni64(ps[63]) > g_last;
                int64_t e_hi;
                bool found = false;
                uint32_t av = 0;
                int64_t my_e = e;
                int64_t pp[NOPS];
                uint64_t my_start = 0;
                if (in_lds) {
                    const uint64_t gl = g + (lane < nv ? lane : nv - 1);
                    int32_t pe = 0;   // ps[0] <= g <= gl
#pragma unroll
                    for (int32_t st = 32; st > 0; st >>= 1)
                        if (ps[pe + st] <= gl) pe += st;
                    my_e = e + pe;
                    my_start = ps[pe];
                    e_hi = (int64_t)uni64((uint64_t)__shfl((long long)my_e, nv - 1, 64));
                } else {
                    e_hi = (int64_t)uni64((uint64_t)advance_entry(prefix, e, e_end, g_last));
                    if (valid) {
                        my_e = find_entry(prefix, e, e_hi + 1, g + lane);
                        my_start = prefix[my_e];
                    }
                }
                wave_sync();
                if (valid) {
                    const uint64_t gl = g + lane;
                    const int il = G.iter[my_e];
                    int32_t bl[NOPS], el[NOPS];
#pragma unroll
                    for (int o = 0; o < NOPS; ++o) {
                        bl[o] = G.seg[(2 * o) * stride + my_e];
                        el[o] = G.seg[(2 * o + 1) * stride + my_e];
                    }
                    const int32_t offl = (int32_t)(gl - my_start);
#pragma unroll
                    for (int o = 0; o < NOPS; ++o)
                        if (o == il) {
                            pp[o] = bl[o] + offl;
                            av = arr0[o][bl[o] + offl];
                        }
                    found = true;
                    const uint64_t r0 = r_begin + rc;
                    if (kMat && out.pos != nullptr) {
                        // match bit and positions from the bitmap pass
#pragma unroll
                        for (int o = 0; o < NOPS; ++o)
                            if (o != il) pp[o] = out.pos[(size_t)o * n_items + r0 + lane];
                        found = (sload(words + (r0 >> 6)) >> lane) & 1ull;
                    } else {
#pragma unroll
                        for (int o = 0; o < NOPS; ++o) {
                            if (o == il || !found) continue;
                            // (the default method searches by interpolation: the keys are hashed)
                            int32_t q;
                            if (SM == 0) {
                                uint32_t kq = 0;
                                q = interp_lb(arr0[o], bl[o], el[o], av, kq);
                                found = q < el[o] && kq == av;
                            } else {
                                q = lane_search(search, arr0[o], bl[o], el[o], av);
                                found = q < el[o] && arr0[o][q] == av;
                            }
                            pp[o] = q;
                        }
                        if (found && S.has_pred) found = pred_ok(S, F + my_e * S.W_in, av, D.mix);
                        if (MODE == M_BITMAP && out.pos != nullptr) {
#pragma unroll
                            for (int o = 0; o < NOPS; ++o)
                                if (o != il) out.pos[(size_t)o * n_items + r0 + lane] = (int32_t)pp[o];
                        }
                    }
                }
                const uint64_t bal = __ballot(found);
                if (kMat) {
                    if (found) {
                        const int64_t rank = (int64_t)(wprefix[(r_begin + rc) >> 6] + (uint64_t)__popcll(bal & lanemask_lt()));
                        write_item(MODE, D, S, F + my_e * S.W_in, av, pp, rank, out);
                    }
                } else if (MODE == M_BITMAP) {
                    if (lane == 0) words[(r_begin + rc) >> 6] = bal;
                } else {
                    cnt += (uint64_t)__popcll(bal);
                    if (MODE == M_DIGEST && found) digest_add<MODE>(D, S, F + my_e * S.W_in, av, dsum, dxor);
                    if (MODE == M_CELLS)
                        cell_add_lanes(out.cells, ca, found, found ? (uint32_t)F[my_e * S.W_in] >> D.cell_group : 0u,
                                       lane);
                }
                // continue inside the last entry touched (its cursors restart)
                e = e_hi;
                load_entry(e);
                rc += chunk;
            }
        }
    }
    if (MODE == M_CELLS) cell_flush(out.cells, ca, lane);
    if (MODE == M_COUNT || MODE == M_DIGEST || MODE == M_CELLS) {
        if (MODE == M_DIGEST) {
            dsum = wave_sum(dsum);
            dxor = wave_xor(dxor);
        }
        if (lane == 0) {
            if (cnt) atomicAdd(&acc[0], (unsigned long long)cnt);
            if (MODE == M_DIGEST) {
                atomicAdd(&acc[1], (unsigned long long)dsum);
                atomicXor(&acc[2], (unsigned long long)dxor);
            }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_materialize(KData D, KStep S, const int32_t* __restrict__ F, Seg G,
                                                        const uint64_t* __restrict__ prefix, int64_t e_begin,
                                                        int64_t e_end, uint64_t item_begin, uint64_t n_items,
                                                        const uint64_t* __restrict__ words,
                                                        const uint64_t* __restrict__ wprefix, MatOut out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n_words = (int64_t)((n_items + 63) / 64);
    for (int64_t w = wave; w < n_words; w += nwaves) {
        const uint64_t bal = words[w];
        if (bal == 0) continue;
        const uint64_t rel = (uint64_t)w * 64 + lane;
        const uint64_t g_first = item_begin + (uint64_t)w * 64;
        const uint64_t last_rel = ((uint64_t)w * 64 + 63 < n_items) ? (uint64_t)w * 64 + 63 : n_items - 1;
        const int64_t e_lo = find_entry(prefix, e_begin, e_end, g_first);
        const int64_t e_hi = find_entry(prefix, e_lo, e_end, item_begin + last_rel);
        if (!((bal >> lane) & 1ull)) continue;
        const uint64_t g = item_begin + rel;
        Probe P;
        probe_item(D, S, F, G, prefix, find_entry(prefix, e_lo, e_hi + 1, g), g, P);
        const int64_t rank = (int64_t)(wprefix[w] + (uint64_t)__popcll(bal & lanemask_lt()));
        write_item(MODE, D, S, F + P.e * S.W_in, P.a, P.pos, rank, out);
    }
}

// Request batches (F_0 = one entry per request, each with its first-variable id
// range lo..hi, inclusive, in words pred_word and pred_word + 1).  The mixer is a
// bijection, so the keys a request can bind at the first level are the mixed ids of
// its block: slot g of request t (slot_prefix[t] <= g < slot_prefix[t+1]) mixes id
// lo + (g - slot_prefix[t]) and binary-searches it in every top-level operand.  A
// block of w ids then costs w searches instead of a pass over the top level.
__global__ void k_first_ids(KData D, KStep S, const int32_t* __restrict__ F, const uint64_t* __restrict__ slot_prefix,
                            int64_t n_req, uint64_t n_slots, uint32_t* __restrict__ found, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ pos) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_slots;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t t = find_entry(slot_prefix, 0, n_req, g);
        const int32_t* ent = F + t * S.W_in;
        const uint32_t raw = (uint32_t)ent[S.pred_word] + (uint32_t)(g - slot_prefix[t]);
        const uint32_t key = mix_key(raw, D.mix);
        bool ok = pred_ok(S, ent, key, D.mix);
        for (int o = 0; o < S.n_ops; ++o) {
            int64_t beg, end;
            v0_bounds(D, S.ops[o], ent, (uint32_t)ent[0], beg, end);
            const uint32_t* arr = D.atoms[S.ops[o].atom].V[0];
            const int64_t p = lower_bound_u32(arr, beg, end, key);
            ok = ok && p < end && arr[p] == key;
            pos[(uint64_t)o * n_slots + g] = (int32_t)p;
        }
        found[g] = ok ? 1u : 0u;
        keys[g] = key;
    }
}

__global__ void k_first_write(KData D, KStep S, const int32_t* __restrict__ F, const uint64_t* __restrict__ slot_prefix,
                              int64_t n_req, uint64_t n_slots, const uint32_t* __restrict__ keys,
                              const int32_t* __restrict__ pos, const uint64_t* __restrict__ rank, MatOut out) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_slots;
         g += (uint64_t)gridDim.x * blockDim.x) {
        if (rank[g + 1] == rank[g]) continue;
        const int64_t t = find_entry(slot_prefix, 0, n_req, g);
        int64_t pp[kMaxOps];
        for (int o = 0; o < S.n_ops; ++o) pp[o] = pos[(uint64_t)o * n_slots + g];
        write_item(M_EXPAND, D, S, F + t * S.W_in, keys[g], pp, (int64_t)rank[g], out);
    }
}

__global__ void k_chunk_entries(const uint64_t* __restrict__ prefix, int64_t e_begin, int64_t e_end,
                                uint64_t item_begin, uint64_t n_chunks, uint64_t chunk_sz, int64_t* __restrict__ out) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_chunks;
         t += (uint64_t)gridDim.x * blockDim.x)
        out[t] = find_entry(prefix, e_begin, e_end, item_begin + t * chunk_sz);
}

template <int MODE>
static void launch_probe(const Alloc& A, const KData& D, const KStep& S, const int32_t* F, const Seg& G,
                         const uint64_t* prefix, int64_t e_begin, int64_t e_end, uint64_t item_begin,
                         uint64_t n_items, uint64_t* words, unsigned long long* acc, hipStream_t s,
                         const uint64_t* wprefix = nullptr, MatOut out = MatOut{}) {
    HC_REQUIRE(!mat_mode(MODE) || wprefix != nullptr, HC_ERR_DEVICE, "materialising probe without match ranks");
    HC_REQUIRE(MODE != M_CELLS || out.cells != nullptr, HC_ERR_DEVICE, "per-cell probe without a cell buffer");
    HC_REQUIRE(MODE != M_BITMAP || words != nullptr, HC_ERR_DEVICE, "bitmap probe without match words");
    HC_REQUIRE(MODE == M_BITMAP || mat_mode(MODE) || acc != nullptr, HC_ERR_DEVICE, "counting probe without accumulator");
    if (S.n_ops > 4) {
        if (mat_mode(MODE)) {
            const int64_t nw = (int64_t)((n_items + 63) / 64);
            int64_t g2 = (nw + kWaves - 1) / kWaves;
            if (g2 < 1) g2 = 1;
            if (g2 > 16384) g2 = 16384;
            k_materialize<MODE><<<(unsigned)g2, kBlock, 0, s>>>(D, S, F, G, prefix, e_begin, e_end, item_begin,
                                                                n_items, words, wprefix, out);
            HC_HIP(hipGetLastError());
            return;
        }
        const int64_t nw = (int64_t)((n_items + 63) / 64);
        int64_t g2 = (nw + kWaves - 1) / kWaves;
        if (g2 < 1) g2 = 1;
        if (g2 > 16384) g2 = 16384;
        k_probe<mat_mode(MODE) ? M_BITMAP : MODE><<<(unsigned)g2, kBlock, 0, s>>>(
            D, S, F, G, prefix, e_begin, e_end, item_begin, n_items, words, acc, out.cells);
        HC_HIP(hipGetLastError());
        return;
    }
    // Chunks of kChunk elements; a launch with fewer elements than the persistent grid
    // has waves takes smaller chunks (down to kMinChunk; chunk starts stay on
    // match-word boundaries), so that its waves all get work instead of a few walking
    // long chunks one after another.
    // the persistent grid: 8 workgroups per CU, or the context's limit (a multiple of
    // the 8 XCDs, so that every XCD queue has consumers)
    const uint64_t max_blocks = D.grid_limit > 0 ? std::max<uint64_t>(kXcd, (uint64_t)D.grid_limit / kXcd * kXcd)
                                                 : kPersistBlocks;
    uint64_t chunk_sz = kChunk;
    while (chunk_sz > kMinChunk && n_items / chunk_sz < max_blocks * kWaves) chunk_sz >>= 1;
    const uint64_t n_chunks = (n_items + chunk_sz - 1) / chunk_sz;
    DevBuf<int64_t> ce(A, (size_t)n_chunks + 1);
    DevBuf<unsigned long long> q(A, kXcd);
    HC_HIP(hipMemsetAsync(q.p, 0, sizeof(unsigned long long) * kXcd, s));
    {
        int64_t g = (int64_t)((n_chunks + kBlock - 1) / kBlock);
        if (g < 1) g = 1;
        if (g > 16384) g = 16384;
        k_chunk_entries<<<(unsigned)g, kBlock, 0, s>>>(prefix, e_begin, e_end, item_begin, n_chunks, chunk_sz, ce.p);
        HC_HIP(hipGetLastError());
    }
    // persistent grid: a multiple of 8 workgroups (every XCD queue has consumers)
    uint64_t blocks = (n_chunks + kWaves - 1) / kWaves;
    if (blocks > max_blocks) blocks = max_blocks;
    blocks = ((blocks + kXcd - 1) / kXcd) * kXcd;
#define HC_PROBE2(N)                                                                                          \
    if (S.search == SEARCH_WINDOW)                                                                            \
        k_probe2<MODE, N, 0><<<(unsigned)blocks, kBlock, 0, s>>>(D, S, F, G, prefix, e_begin, e_end,         \
                                                                 item_begin, n_items, ce.p, q.p, n_chunks,    \
                                                                 (uint32_t)chunk_sz,                          \
                                                                 words, acc, wprefix, out);                   \
    else                                                                                                      \
        k_probe2<MODE, N, 1><<<(unsigned)blocks, kBlock, 0, s>>>(D, S, F, G, prefix, e_begin, e_end,         \
                                                                 item_begin, n_items, ce.p, q.p, n_chunks,    \
                                                                 (uint32_t)chunk_sz,                          \
                                                                 words, acc, wprefix, out)
    switch (S.n_ops) {
        case 1: HC_PROBE2(1); break;
        case 2: HC_PROBE2(2); break;
        case 3: HC_PROBE2(3); break;
        default: HC_PROBE2(4); break;
    }
#undef HC_PROBE2
    HC_HIP(hipGetLastError());
}

// (offset, length) of every entry's temporary result, from the match words.
// (n_dev, when set, holds the entry count: entries [0, *n_dev), device-sized sequences)
__global__ void k_tmp_refs(int32_t* F, int W, int word, const uint64_t* __restrict__ prefix, int64_t e_begin,
                           int64_t e_end, uint64_t item_begin, const uint64_t* __restrict__ words,
                           const uint64_t* __restrict__ wprefix, int64_t pool_base,
                           const uint64_t* __restrict__ n_dev = nullptr) {
    if (n_dev) e_end = e_begin + (int64_t)*n_dev;
    auto rank = [&](uint64_t g) -> uint64_t {
        const uint64_t rel = g - item_begin;
        const uint64_t w = rel >> 6, bit = rel & 63;
        uint64_t r = wprefix[w];
        if (bit) r += (uint64_t)__popcll(words[w] & ((1ull << bit) - 1ull));
        return r;
    };
    for (int64_t e = e_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e_end;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t r0 = rank(prefix[e]), r1 = rank(prefix[e + 1]);
        F[e * W + word] = (int32_t)(pool_base + (int64_t)r0);
        F[e * W + word + 1] = (int32_t)(r1 - r0);
    }
}

// Largest e in [lo, hi] with prefix[e] - prefix[lo] <= budget (at least lo+1 when possible).
__global__ void k_split(const uint64_t* prefix, int64_t lo, int64_t hi, uint64_t budget, int64_t* out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const uint64_t base = prefix[lo];
    int64_t a = lo, z = hi;   // invariant: prefix[a] - base <= budget
    while (a < z) {
        const int64_t mid = (a + z + 1) >> 1;
        if (prefix[mid] - base <= budget) a = mid; else z = mid - 1;
    }
    if (a == lo && lo < hi) a = lo + 1;   // a single entry always makes progress
    *out = a;
}

// ---------------------------------------------------------------- host driver
static unsigned grid_for(int64_t n, int64_t cap = 16384) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}
static unsigned grid_waves(int64_t n_words, int64_t cap = 8192) {
    int64_t g = (n_words + kWaves - 1) / kWaves;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

struct Layout {
    int W;
    int node_word[kMaxAtoms][3];   // per atom and CoCo level of the node
    int tmp_word[kMaxGroups];
};

// Words of a frontier F_i entry: the cell id, the i bound keys, the CoCo level-0
// position of every atom whose first variable is bound and whose second is not
// yet, and an (offset, length) pair per live lifted intersection.
static Layout make_layout(const Plan& P, int i) {
    Layout L;
    int w = 1 + i;
    for (int j = 0; j < kMaxAtoms; ++j)
        for (int r = 0; r < 3; ++r) L.node_word[j][r] = -1;
    for (int g = 0; g < kMaxGroups; ++g) L.tmp_word[g] = -1;
    for (int j = 0; j < P.n_atoms; ++j)
        for (int r = 0; r + 1 < P.atom_arity[j]; ++r) {
            const int pr = P.pos[P.atom_lvl_var[j][r]], pn = P.pos[P.atom_lvl_var[j][r + 1]];
            if (pr < i && i <= pn) L.node_word[j][r] = w++;
        }
    for (int g = 0; g < P.n_groups; ++g)
        if (P.groups[g].lift <= i && i <= P.groups[g].consumer) {
            L.tmp_word[g] = w;
            w += 2;
        }
    L.W = w;
    return L;
}

struct Runner {
    hc_ctx* ctx;
    const Alloc& A;
    hipStream_t s;
    Plan P;
    KData D;
    Layout lay[kMaxVars + 1];
    KStep level_step[kMaxVars];
    KStep group_step[kMaxGroups];
    int shares[kMaxVars];
    int cell_shift[kMaxVars];
    int K;
    bool emit, digest;
    int seg_bits = 0;                        // key bits above the mixed bits (batched queries)
    int range_word = -1;                     // F_0 word of a query batch's id ranges
    std::vector<uint64_t> id_slots;          // query batch: exclusive prefix of the id-block widths
    int search_mode = SEARCH_WINDOW;
    unsigned long long* cell_out = nullptr;  // per-cell counts (device), or null
    int64_t cap_entries;
    DevBuf<unsigned long long> acc;
    DevBuf<int64_t> split;
    std::vector<DevBuf<int2>> ranges;
    std::vector<DevBuf<int32_t>> child_tab;
    std::vector<uint64_t> child_key;
    DevBuf<uint32_t> tmp_val[kMaxGroups];
    DevBuf<int32_t> tmp_src[kMaxGroups][kMaxOps];
    int64_t tmp_cap[kMaxGroups] = {};        // elements per lifted-intersection pool (grown on demand)
    int64_t tmp_max = 0;                     // pool size the chunking aims for
    // emit
    void* out_rows = nullptr;
    int64_t out_cap = 0, out_count = 0;
    // profiling
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double leaf_ms = 0;
    int64_t leaf_launches = 0;
    uint64_t leaf_items = 0;

    Runner(hc_ctx* c, const Alloc& a) : ctx(c), A(a), s(c->stream) {}
    ~Runner() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    uint64_t read_u64(const uint64_t* p) {
        uint64_t v = 0;
        HC_HIP(hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, s));
        HC_HIP(hipStreamSynchronize(s));
        check_cancel();
        return v;
    }
    // every level and chunk reads sizes back, so a cancel request stops the call there
    void check_cancel() const { HC_REQUIRE(!ctx->cancel.load(), HC_ERR_CANCELLED, "cancelled"); }

    void setup_layouts() {
        for (int i = 0; i <= P.n_vars; ++i) {
            lay[i] = make_layout(P, i);
            HC_REQUIRE(lay[i].W <= kMaxW, HC_ERR_UNSUPPORTED, "frontier entry too wide");
        }
    }

    KOp make_op(const PlanOp& po, const Layout& L, int var, int fi) {
        KOp o{};
        o.kind = po.kind;
        o.atom = po.atom;
        o.group = po.group;
        o.word = -1;
        o.v0_range = nullptr;
        o.lvl = po.lvl;
        if (po.kind == OP_CHILD) o.word = L.node_word[po.atom][po.lvl - 1];
        if (po.kind == OP_TMP) o.word = L.tmp_word[po.group];
        o.child_range = nullptr;
        o.child_stride = 0;
        o.rng_shift = 0;
        o.rng_k = 0;
        o.rng_word = -1;
        int vk = 0, vshift = 0, vword = -1;
        if (po.kind == OP_V0 && shares[var] > 0) {
            vk = shares[var];
            vshift = cell_shift[var];
        } else if (po.kind == OP_V0 && seg_bits > 0) {
            // segmented keys: every variable stays inside the segment (the key bits
            // above the mixed bits) of the first variable's value; below F_1 that value
            // is not bound yet, and the segment comes from the query's id range (a batch
            // of queries) or from the first variable's cell coordinate
            vk = seg_bits;
            if (fi >= 1) {
                vshift = D.mix.b;
                vword = 1;
            } else if (range_word >= 0) {
                vshift = D.mix.b;
                vword = range_word;
            } else {
                const int v0 = P.order[0];
                vshift = cell_shift[v0] + shares[v0] - seg_bits;
            }
        }
        if (vk > 0) {
            ranges.emplace_back(A, (size_t)1 << vk);
            const DAtom& a = D.atoms[po.atom];
            k_v0_ranges<<<grid_for((int64_t)1 << vk), kBlock, 0, s>>>(a.V[0], a.len[0], D.b, vk, ranges.back().p);
            HC_HIP(hipGetLastError());
            o.v0_range = ranges.back().p;
            o.rng_k = vk;
            o.rng_shift = vshift;
            o.rng_word = vword;
        }
        if (po.kind == OP_CHILD && shares[var] > 0) {
            // sub-range boundaries of every child list for every coordinate, when the
            // table stays small; otherwise the cell's range is found by binary search
            const int k = shares[var];
            const DAtom& a = D.atoms[po.atom];
            const int64_t stride = ((int64_t)1 << k) + 1;
            const int64_t nodes = a.len[po.lvl - 1];
            if (nodes * stride <= cap_entries) {
                const uint64_t key = ((uint64_t)po.atom << 16) | ((uint64_t)po.lvl << 8) | (uint64_t)k;
                int found = -1;
                for (size_t t = 0; t < child_key.size(); ++t)
                    if (child_key[t] == key) found = (int)t;
                if (found < 0) {
                    child_tab.emplace_back(A, (size_t)(nodes * stride + 1));
                    child_key.push_back(key);
                    found = (int)child_tab.size() - 1;
                    k_child_ranges<<<grid_for(nodes * stride), kBlock, 0, s>>>(a.O[po.lvl - 1], a.V[po.lvl],
                                                                                nodes, D.b, k, child_tab.back().p);
                    HC_HIP(hipGetLastError());
                }
                o.child_range = child_tab[found].p;
                o.child_stride = (int32_t)stride;
            }
        }
        return o;
    }

    // Operands of a lifted intersection whose positions the pool keeps: those with a
    // further CoCo level below (their position becomes a node of a later level).
    bool is_source(const PlanOp& o) const { return o.lvl + 1 < P.atom_arity[o.atom]; }

    void setup_steps(const hc_query* q) {
        const int n = P.n_vars;
        for (int i = 0; i < n; ++i) {
            const PlanLevel& PL = P.levels[i];
            KStep& S = level_step[i];
            S = KStep{};
            const Layout& Li = lay[i];
            const Layout& Lo = lay[i + 1];
            S.n_ops = PL.n_ops;
            for (int t = 0; t < PL.n_ops; ++t) S.ops[t] = make_op(PL.ops[t], Li, PL.var, i);
            S.W_in = Li.W;
            S.k_share = shares[PL.var];
            S.cell_shift = cell_shift[PL.var];
            S.search = search_mode;
            S.has_pred = q->var_lo != nullptr;
            S.pred_lo = 0;
            S.pred_hi = INT64_MAX;
            S.pred_word = -1;
            if (S.has_pred) {
                S.pred_lo = q->var_lo[PL.var];
                S.pred_hi = q->var_hi[PL.var];
            }
            S.W_out = Lo.W;
            S.n_copy = 0;
            auto copy = [&](int from, int to) {
                S.copy_from[S.n_copy] = (int8_t)from;
                S.copy_to[S.n_copy] = (int8_t)to;
                ++S.n_copy;
            };
            for (int w = 0; w <= i; ++w) copy(w, w);   // cell and bound values
            S.val_word = i + 1;
            S.n_new = 0;
            S.n_zero = 0;
            for (int j = 0; j < P.n_atoms; ++j)
                for (int r = 0; r + 1 < P.atom_arity[j]; ++r) {
                    if (Lo.node_word[j][r] < 0) continue;
                    if (Li.node_word[j][r] >= 0) {
                        copy(Li.node_word[j][r], Lo.node_word[j][r]);
                        continue;
                    }
                    // new node: the atom's level-r variable is bound at this level; its
                    // position comes from the level's operand on that CoCo level, or
                    // from the lifted intersection that holds it
                    int op = -1, src = -1;
                    for (int t = 0; t < PL.n_ops; ++t)
                        if (PL.ops[t].kind != OP_TMP && PL.ops[t].atom == j && PL.ops[t].lvl == r) op = t;
                    if (op < 0) {
                        for (int t = 0; t < PL.n_ops; ++t)
                            if (PL.ops[t].kind == OP_TMP) {
                                const PlanGroup& g = P.groups[PL.ops[t].group];
                                int sidx = 0;
                                for (int u = 0; u < g.n_ops; ++u) {
                                    if (!is_source(g.ops[u])) continue;
                                    if (g.ops[u].atom == j && g.ops[u].lvl == r) {
                                        op = t;
                                        src = sidx;
                                    }
                                    ++sidx;
                                }
                            }
                    }
                    HC_REQUIRE(op >= 0, HC_ERR_DEVICE, "plan: no source for a node");
                    S.new_word[S.n_new] = (int8_t)Lo.node_word[j][r];
                    S.new_op[S.n_new] = (int8_t)op;
                    S.new_src[S.n_new] = (int8_t)(src < 0 ? 0 : src);
                    ++S.n_new;
                }
            for (int g = 0; g < P.n_groups; ++g) {
                if (Lo.tmp_word[g] < 0) continue;
                if (Li.tmp_word[g] >= 0) {
                    copy(Li.tmp_word[g], Lo.tmp_word[g]);
                    copy(Li.tmp_word[g] + 1, Lo.tmp_word[g] + 1);
                } else {
                    S.zero_word[S.n_zero++] = (int8_t)Lo.tmp_word[g];
                    S.zero_word[S.n_zero++] = (int8_t)(Lo.tmp_word[g] + 1);
                }
            }
            S.n_vars = n;
            for (int v = 0; v < n; ++v) S.head_word[v] = (int8_t)(P.pos[v] < i ? 1 + P.pos[v] : -1);
        }
        for (int g = 0; g < P.n_groups; ++g) {
            const PlanGroup& PG = P.groups[g];
            KStep& S = group_step[g];
            S = KStep{};
            const Layout& L = lay[PG.lift];
            S.n_ops = PG.n_ops;
            for (int t = 0; t < PG.n_ops; ++t) S.ops[t] = make_op(PG.ops[t], L, PG.var, PG.lift);
            S.W_in = L.W;
            S.k_share = shares[PG.var];
            S.cell_shift = cell_shift[PG.var];
            S.has_pred = 0;   // the predicate is applied where the variable is bound
            S.pred_word = -1;
            S.search = search_mode;
            S.group = g;
            S.n_src = 0;
            for (int t = 0; t < PG.n_ops; ++t)
                if (is_source(PG.ops[t])) S.src_op[S.n_src++] = (int8_t)t;
        }
    }

    struct StepBufs {
        DevBuf<int32_t> seg;
        DevBuf<int32_t> iter;
        DevBuf<uint32_t> m;
        DevBuf<uint64_t> prefix;
        Seg G;
    };

    void prep(const KStep& S, const int32_t* F, int64_t e0, int64_t n, StepBufs& B) {
        B.seg = DevBuf<int32_t>(A, (size_t)(2 * S.n_ops) * (size_t)n);
        B.iter = DevBuf<int32_t>(A, (size_t)n);
        B.m = DevBuf<uint32_t>(A, (size_t)n);
        B.prefix = DevBuf<uint64_t>(A, (size_t)n + 1);
        // index arrays by absolute entry e: shift the base pointers by -e0
        B.G.stride = n;
        B.G.seg = B.seg.p - e0;
        B.G.iter = B.iter.p - e0;
        B.G.m = B.m.p - e0;
        k_prep<<<grid_for(n), kBlock, 0, s>>>(D, S, F, e0, n, B.G, nullptr);
        HC_HIP(hipGetLastError());
        scan_exclusive(A, LoadU32{B.m.p}, B.prefix.p, n, s);
    }

    // Items [prefix[ea], prefix[eb]) of a prepared step into match words + their scan.
    // The bitmap pass over items [ib, ib + ni): match words, their scan (returns the
    // matches) and, for the cursor kernel, the positions found in the probed operands,
    // which the materialising pass then reads instead of searching again.
    uint64_t match_words(const KStep& S, const int32_t* F, StepBufs& B, const uint64_t* prefix_abs, int64_t ea,
                         int64_t eb, uint64_t ib, uint64_t ni, DevBuf<uint64_t>& words, DevBuf<uint64_t>& wpre,
                         DevBuf<int32_t>& posb) {
        const int64_t nw = (int64_t)((ni + 63) / 64);
        words = DevBuf<uint64_t>(A, (size_t)nw + 1);
        wpre = DevBuf<uint64_t>(A, (size_t)nw + 1);
        MatOut mo{};
        if (nw > 0 && S.n_ops <= 4) {
            posb = DevBuf<int32_t>(A, (size_t)S.n_ops * (size_t)ni);
            mo.pos = posb.p;
        }
        if (nw > 0) launch_probe<M_BITMAP>(A, D, S, F, B.G, prefix_abs, ea, eb, ib, ni, words.p, nullptr, s, nullptr, mo);
        scan_popc(A, words.p, wpre.p, nw, s);
        return read_u64(wpre.p + nw);
    }

    // (Re)allocate the pool of group g; its previous contents are discarded.
    void grow_tmp(int g, int64_t elems) {
        tmp_val[g] = DevBuf<uint32_t>(A, (size_t)elems);
        for (int u = 0; u < group_step[g].n_src; ++u) tmp_src[g][u] = DevBuf<int32_t>(A, (size_t)elems);
        tmp_cap[g] = elems;
        refresh_tmp_ptrs();
    }

    void refresh_tmp_ptrs() {
        for (int g = 0; g < kMaxGroups; ++g) {
            D.tmp_val[g] = tmp_val[g].p;
            for (int u = 0; u < kMaxOps; ++u) D.tmp_src[g][u] = tmp_src[g][u].p;
        }
    }

    void run_level(int i, const int32_t* F, int32_t* Fmut, int64_t n);
    void first_ids(const int32_t* F, int64_t n);
};

// F_0 -> F_1 of a request batch by searching each request's mixed ids (k_first_ids).
void Runner::first_ids(const int32_t* F, int64_t n) {
    const KStep& S = level_step[0];
    const uint64_t n_slots = id_slots[(size_t)n];
    DevBuf<uint64_t> sp(A, (size_t)n + 1);
    HC_HIP(hipMemcpyAsync(sp.p, id_slots.data(), sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    DevBuf<uint32_t> found(A, (size_t)n_slots), keys(A, (size_t)n_slots);
    DevBuf<int32_t> pos(A, (size_t)S.n_ops * (size_t)n_slots);
    DevBuf<uint64_t> rank(A, (size_t)n_slots + 1);
    k_first_ids<<<grid_for((int64_t)n_slots), kBlock, 0, s>>>(D, S, F, sp.p, n, n_slots, found.p, keys.p, pos.p);
    HC_HIP(hipGetLastError());
    scan_exclusive(A, LoadU32{found.p}, rank.p, (int64_t)n_slots, s);
    const uint64_t got = read_u64(rank.p + n_slots);
    if (got == 0) return;
    DevBuf<int32_t> Fn(A, (size_t)got * (size_t)lay[1].W);
    MatOut mo{};
    mo.F = Fn.p;
    k_first_write<<<grid_for((int64_t)n_slots), kBlock, 0, s>>>(D, S, F, sp.p, n, n_slots, keys.p, pos.p, rank.p, mo);
    HC_HIP(hipGetLastError());
    found.reset();
    keys.reset();
    pos.reset();
    rank.reset();
    run_level(1, Fn.p, Fn.p, (int64_t)got);
}

void Runner::run_level(int i, const int32_t* F, int32_t* Fmut, int64_t n) {
    if (n <= 0) return;
    const int nv = P.n_vars;
    if (i == 0 && !id_slots.empty()) {
        first_ids(F, n);
        return;
    }
    // 1. lifted intersections whose lift level is i, chunked by the tmp pool
    std::vector<int> groups;
    for (int g = 0; g < P.n_groups; ++g)
        if (P.groups[g].lift == i) groups.push_back(g);
    std::vector<StepBufs> gb(groups.size());
    std::vector<uint64_t> gtot(groups.size());
    bool one_chunk = true;   // every group's elements fit its pool: no chunking, no split round trips
    for (size_t t = 0; t < groups.size(); ++t) {
        const int g = groups[t];
        prep(group_step[g], F, 0, n, gb[t]);
        // The pool of a group lifted at this level is dead between calls of this
        // level and between its chunks, so it is sized here: all of this call's
        // elements, up to tmp_max (the chunking below splits the rest).
        gtot[t] = read_u64(gb[t].prefix.p + n);
        const uint64_t need = std::max<uint64_t>(1, std::min<uint64_t>(gtot[t], (uint64_t)tmp_max));
        if (need > (uint64_t)tmp_cap[g]) grow_tmp(g, (int64_t)need);
        one_chunk = one_chunk && gtot[t] <= (uint64_t)tmp_cap[g];
    }
    int64_t ea = 0;
    while (ea < n) {
        int64_t eb = n;
        for (size_t t = 0; t < groups.size() && !one_chunk; ++t) {
            k_split<<<1, 1, 0, s>>>(gb[t].prefix.p, ea, eb, (uint64_t)tmp_cap[groups[t]], split.p);
            HC_HIP(hipGetLastError());
            int64_t e2 = 0;
            HC_HIP(hipMemcpyAsync(&e2, split.p, sizeof(e2), hipMemcpyDeviceToHost, s));
            HC_HIP(hipStreamSynchronize(s));
            eb = std::min(eb, e2);
        }
        for (size_t t = 0; t < groups.size(); ++t) {
            const int g = groups[t];
            const KStep& S = group_step[g];
            uint64_t pr[2] = {0, gtot[t]};
            if (!one_chunk) {
                HC_HIP(hipMemcpyAsync(&pr[0], gb[t].prefix.p + ea, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
                HC_HIP(hipMemcpyAsync(&pr[1], gb[t].prefix.p + eb, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
                HC_HIP(hipStreamSynchronize(s));
            }
            const uint64_t ni = pr[1] - pr[0];
            HC_REQUIRE(ni <= (uint64_t)tmp_cap[g] || eb == ea + 1, HC_ERR_DEVICE, "tmp chunking failed");
            if (ni > (uint64_t)tmp_cap[g]) grow_tmp(g, (int64_t)ni);   // one entry larger than the pool
            DevBuf<uint64_t> words, wpre;
            DevBuf<int32_t> posb;
            match_words(S, F, gb[t], gb[t].prefix.p, ea, eb, pr[0], ni, words, wpre, posb);
            const int64_t nw = (int64_t)((ni + 63) / 64);
            if (nw > 0) {
                MatOut mo{};
                mo.pos = posb.p;
                mo.tval = tmp_val[g].p;
                for (int u = 0; u < S.n_src; ++u) mo.tsrc[u] = tmp_src[g][u].p;
                launch_probe<M_TMPW>(A, D, S, F, gb[t].G, gb[t].prefix.p, ea, eb, pr[0], ni, words.p, nullptr, s,
                                     wpre.p, mo);
            }
            k_tmp_refs<<<grid_for(eb - ea), kBlock, 0, s>>>(Fmut, lay[i].W, lay[i].tmp_word[g], gb[t].prefix.p, ea,
                                                            eb, pr[0], words.p, wpre.p, 0);
            HC_HIP(hipGetLastError());
        }
        // 2. the level's own intersection over entries [ea, eb)
        const KStep& S = level_step[i];
        StepBufs B;
        prep(S, F, ea, eb - ea, B);
        const uint64_t total = read_u64(B.prefix.p + (eb - ea));
        // B.prefix is indexed relative to ea: present it as absolute
        const uint64_t* prefix_abs = B.prefix.p - ea;
        if (i == nv - 1) {
            if (!emit) {
                if (total > 0) {
                    if (ctx->profiling) HC_HIP(hipEventRecord(ev0, s));
                    if (digest)
                        launch_probe<M_DIGEST>(A, D, S, F, B.G, prefix_abs, ea, eb, 0, total, nullptr, acc.p, s);
                    else if (cell_out) {
                        MatOut mo{};
                        mo.cells = cell_out;
                        launch_probe<M_CELLS>(A, D, S, F, B.G, prefix_abs, ea, eb, 0, total, nullptr, acc.p, s,
                                              nullptr, mo);
                    } else
                        launch_probe<M_COUNT>(A, D, S, F, B.G, prefix_abs, ea, eb, 0, total, nullptr, acc.p, s);
                    if (ctx->profiling) {
                        HC_HIP(hipEventRecord(ev1, s));
                        HC_HIP(hipEventSynchronize(ev1));
                        float ms = 0;
                        HC_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                        leaf_ms += ms;
                        ++leaf_launches;
                    }
                    leaf_items += total;
                }
            } else {
                // emit in chunks of at most cap_entries elements
                uint64_t ib = 0;
                while (ib < total) {
                    const uint64_t ni = std::min<uint64_t>(total - ib, (uint64_t)cap_entries);
                    DevBuf<uint64_t> words, wpre;
                    DevBuf<int32_t> posb;
                    const uint64_t got = match_words(S, F, B, prefix_abs, ea, eb, ib, ni, words, wpre, posb);
                    if (got > 0 && out_count < out_cap) {
                        MatOut mo{};
                        mo.pos = posb.p;
                        mo.rows = out_rows;
                        mo.row_base = out_count;
                        mo.row_cap = out_cap;
                        launch_probe<M_EMIT>(A, D, S, F, B.G, prefix_abs, ea, eb, ib, ni, words.p, nullptr, s,
                                             wpre.p, mo);
                    }
                    out_count += (int64_t)got;
                    ib += ni;
                }
            }
        } else {
            // expand in chunks of entries whose elements fit the next frontier
            int64_t ca = ea;
            while (ca < eb) {
                int64_t cb = eb;
                uint64_t pr[2] = {0, total};   // prefix_abs[ea] = 0, prefix_abs[eb] = total
                if (ca != ea || total > (uint64_t)cap_entries) {
                    k_split<<<1, 1, 0, s>>>(prefix_abs, ca, eb, (uint64_t)cap_entries, split.p);
                    HC_HIP(hipGetLastError());
                    HC_HIP(hipMemcpyAsync(&cb, split.p, sizeof(cb), hipMemcpyDeviceToHost, s));
                    HC_HIP(hipStreamSynchronize(s));
                    HC_HIP(hipMemcpyAsync(&pr[0], prefix_abs + ca, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
                    HC_HIP(hipMemcpyAsync(&pr[1], prefix_abs + cb, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
                    HC_HIP(hipStreamSynchronize(s));
                }
                const uint64_t ni = pr[1] - pr[0];
                DevBuf<uint64_t> words, wpre;
                DevBuf<int32_t> posb;
                const uint64_t got = match_words(S, F, B, prefix_abs, ca, cb, pr[0], ni, words, wpre, posb);
                if (got > 0) {
                    DevBuf<int32_t> Fn(A, (size_t)got * (size_t)lay[i + 1].W);
                    MatOut mo{};
                    mo.F = Fn.p;
                    mo.pos = posb.p;
                    launch_probe<M_EXPAND>(A, D, S, F, B.G, prefix_abs, ca, cb, pr[0], ni, words.p, nullptr, s,
                                           wpre.p, mo);
                    words.reset();
                    wpre.reset();
                    posb.reset();
                    run_level(i + 1, Fn.p, Fn.p, (int64_t)got);
                }
                ca = cb;
            }
        }
        ea = eb;
    }
}

// Validates a join call and sets R up: plan, CoCo descriptors, shares and cell
// layout, frontier layouts, steps and the operands' range tables.
static void setup_runner(Runner& R, hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                         const int32_t* shares, uint32_t flags, bool emit, bool digest, void* out, int64_t capacity,
                         int64_t n_multi, const int64_t* multi_ranges, int64_t cap_entries, bool cell_counts) {
    // A batch of queries has one F_0 entry per query: an intersection of whole top
    // levels lifted to F_0 would be recomputed for every query, so it is not lifted.
    R.P = compile_plan(q, order, !(flags & HC_NO_REWRITE), n_multi > 0 ? 1 : 0);
    const Plan& P = R.P;
    // CoCos: same key width and mixer, columns ordered by the variable order
    int b = -1, mb = -1;
    uint64_t seed = 0;
    int dtype64 = 0;
    for (int j = 0; j < P.n_atoms; ++j) {
        const hc_coco* c = atoms[j];
        HC_REQUIRE(c != nullptr, HC_ERR_INVALID, "atom CoCo handle is NULL");
        HC_REQUIRE(c->arity == P.atom_arity[j], HC_ERR_INVALID, "CoCo arity does not match its atom");
        if (b < 0) {
            b = c->key_bits;
            seed = c->mix_seed;
            mb = c->mix_bits;
            dtype64 = c->dtype == HC_I64;
        }
        HC_REQUIRE(c->key_bits == b && c->mix_seed == seed && c->mix_bits == mb, HC_ERR_INVALID,
                   "all CoCos of a join must share key_bits and mix_seed");
        if (c->arity >= 2 && !(c->symmetric && c->arity == 2)) {
            // level r of the CoCo must hold the atom's column of its r-th variable in order
            int off = 0;
            for (int t = 0; t < j; ++t) off += q->atom_arity[t];
            for (int r = 0; r < c->arity; ++r) {
                int col = -1;
                for (int cc = 0; cc < c->arity; ++cc)
                    if (q->atom_vars[off + cc] == P.atom_lvl_var[j][r]) col = cc;
                HC_REQUIRE(c->col_order[r] == col, HC_ERR_INVALID,
                           "CoCo column order does not follow the variable order for atom " + std::to_string(j));
            }
        }
    }
    int K = 0;
    for (int v = 0; v < P.n_vars; ++v) {
        R.shares[v] = shares ? shares[v] : 0;
        HC_REQUIRE(R.shares[v] >= 0 && R.shares[v] <= b, HC_ERR_INVALID, "log2 share out of range [0, key_bits]");
        K += R.shares[v];
    }
    HC_REQUIRE(K <= 24, HC_ERR_INVALID, "more than 2^24 cells");
    R.seg_bits = b - mb;
    if (R.seg_bits > 0 && n_multi <= 0) {
        // segmented keys (batched queries): the first variable's coordinate must name
        // the segment, and no other variable may be split
        HC_REQUIRE(R.shares[P.order[0]] >= R.seg_bits, HC_ERR_INVALID,
                   "segmented CoCos: the first variable's share must cover the segment bits");
        for (int v = 0; v < P.n_vars; ++v)
            HC_REQUIRE(v == P.order[0] || R.shares[v] == 0, HC_ERR_INVALID,
                       "segmented CoCos: only the first variable of the order may have a share");
    }
    if (n_multi > 0) {
        // many queries in one pass: F_0 holds one entry per query (its index and its id
        // range on the first variable); the per-cell counts are then per-query counts
        HC_REQUIRE(K == 0, HC_ERR_INVALID, "query batches take no shares");
        if (R.seg_bits > 0) {
            // with segmented CoCos every query stays inside one segment
            for (int64_t t = 0; t < n_multi; ++t) {
                const int64_t lo = std::max<int64_t>(multi_ranges[2 * t], 0);
                const int64_t hi = std::min<int64_t>(multi_ranges[2 * t + 1], (int64_t)1 << b);
                HC_REQUIRE(lo >= hi || (lo >> mb) == ((hi - 1) >> mb), HC_ERR_INVALID,
                           "a query's id range spans two segments (query " + std::to_string(t) + ")");
            }
        }
        HC_REQUIRE(!emit && cell_counts && multi_ranges != nullptr, HC_ERR_INVALID,
                   "query batches are a per-query counting mode");
        HC_REQUIRE(n_multi <= ((int64_t)1 << 24), HC_ERR_INVALID, "more than 2^24 queries in one batch");
    }
    R.K = K;
    {
        // cell id: the first variable of the order in the low bits, the deepest in the
        // high bits, so consecutive cells share the deepest level's key range (and
        // the slices of the child lists the deepest intersections read)
        int acc_shift = 0;
        for (int i = 0; i < P.n_vars; ++i) {
            R.cell_shift[P.order[i]] = acc_shift;
            acc_shift += R.shares[P.order[i]];
        }
    }
    R.D = KData{};
    for (int j = 0; j < P.n_atoms; ++j) {
        const hc_coco* c = atoms[j];
        for (int r = 0; r < 4; ++r) {
            R.D.atoms[j].V[r] = r < c->arity ? c->V[r] : nullptr;
            R.D.atoms[j].len[r] = r < c->arity ? c->level_len[r] : 0;
        }
        for (int r = 0; r < 3; ++r) R.D.atoms[j].O[r] = r + 1 < c->arity ? c->O[r] : nullptr;
    }
    HC_REQUIRE(!ctx->cancel.load(), HC_ERR_CANCELLED, "cancelled");
    R.D.mix = make_mixer(mb, seed, b);
    R.D.b = b;
    R.D.cancel = ctx->d_cancel;
    R.D.grid_limit = ctx->grid_limit;
    R.D.dtype64 = dtype64;
    R.emit = emit;
    R.digest = digest;
    R.out_rows = out;
    R.out_cap = capacity;
    R.cap_entries = cap_entries > 0 ? cap_entries : kDefaultCap;
    R.tmp_max = R.cap_entries;
    R.acc = DevBuf<unsigned long long>(R.A, 4);
    R.split = DevBuf<int64_t>(R.A, 2);
    HC_HIP(hipMemsetAsync(R.acc.p, 0, sizeof(unsigned long long) * 4, R.s));
    R.search_mode = (int)((flags & HC_SEARCH_MASK) >> HC_SEARCH_SHIFT);
    HC_REQUIRE(R.search_mode <= SEARCH_BY_SIZE, HC_ERR_INVALID, "unknown search method in flags");
    // the forced methods of Section 5: the merge is the cursor's linear scan,
    // galloping the exponential search
    if (flags & (HC_FORCE_MERGE | HC_FORCE_GALLOP)) {
        HC_REQUIRE((flags & (HC_FORCE_MERGE | HC_FORCE_GALLOP)) != (HC_FORCE_MERGE | HC_FORCE_GALLOP),
                   HC_ERR_INVALID, "HC_FORCE_MERGE and HC_FORCE_GALLOP exclude each other");
        const int forced = (flags & HC_FORCE_MERGE) ? SEARCH_LINEAR : SEARCH_EXPONENTIAL;
        HC_REQUIRE(R.search_mode == SEARCH_WINDOW || R.search_mode == forced, HC_ERR_INVALID,
                   "a forced intersection method contradicts the HC_SEARCH_* method");
        R.search_mode = forced;
    }
    R.setup_layouts();
    // query batches: F_0 entries end with the query's id range (lo, hi inclusive) on
    // the first variable; word 0 (the cell) is the query index
    const int range_word = R.lay[0].W;
    if (n_multi > 0) {
        R.range_word = range_word;
        R.lay[0].W += 2;
        HC_REQUIRE(R.lay[0].W <= kMaxW, HC_ERR_UNSUPPORTED, "frontier entry too wide");
    }
    R.setup_steps(q);
    if (n_multi > 0) {
        R.level_step[0].has_pred = 1;
        R.level_step[0].pred_word = range_word;
    }
    R.refresh_tmp_ptrs();
}

void join_run(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order, const int32_t* shares,
              uint32_t flags, bool emit, uint64_t* count, uint64_t* digest, void* out, int64_t capacity,
              int64_t* n_out, uint64_t* cell_counts, int64_t n_multi, const int64_t* multi_ranges,
              const Alloc* alloc, int64_t cap_entries, int cell_group) {
    Runner R(ctx, alloc ? *alloc : ctx->alloc);
    setup_runner(R, ctx, q, atoms, order, shares, flags, emit, digest != nullptr, out, capacity, n_multi, multi_ranges,
                 cap_entries, cell_counts != nullptr);
    const Plan& P = R.P;
    const int K = R.K, b = R.D.b;
    const int range_word = R.range_word;
    if (ctx->profiling) {
        HC_HIP(hipEventCreate(&R.ev0));
        HC_HIP(hipEventCreate(&R.ev1));
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->profiling) {
        HC_HIP(hipEventCreate(&t0));
        HC_HIP(hipEventCreate(&t1));
        HC_HIP(hipEventRecord(t0, R.s));
    }
    // F_0: one entry per cell (per query of a batch)
    const int64_t ncell = n_multi > 0 ? n_multi : (int64_t)1 << K;
    // per-cell counters, one per group of 2^cell_group consecutive cells
    HC_REQUIRE(cell_group >= 0 && (n_multi > 0 ? cell_group == 0 : cell_group <= K), HC_ERR_INVALID,
               "cell groups larger than the cells");
    R.D.cell_group = cell_group;
    const int64_t ngroup = ncell >> cell_group;
    DevBuf<unsigned long long> cells;
    if (cell_counts) {
        HC_REQUIRE(!emit, HC_ERR_INVALID, "per-cell counts are a counting mode");
        cells = DevBuf<unsigned long long>(R.A, (size_t)ngroup);
        HC_HIP(hipMemsetAsync(cells.p, 0, sizeof(unsigned long long) * ngroup, R.s));
        R.cell_out = cells.p;
    }
    DevBuf<int32_t> F0(R.A, (size_t)ncell * (size_t)R.lay[0].W);
    std::vector<int32_t> f0_host;
    if (n_multi > 0) {
        const int W0 = R.lay[0].W;
        f0_host.assign((size_t)ncell * W0, 0);   // lifted-intersection references start empty
        for (int64_t t = 0; t < ncell; ++t) {
            const int64_t lo = std::max<int64_t>(multi_ranges[2 * t], 0);
            const int64_t hi = std::min<int64_t>(multi_ranges[2 * t + 1], (int64_t)1 << 32);
            int32_t* e = f0_host.data() + (size_t)t * W0;
            e[0] = (int32_t)t;
            e[range_word] = (int32_t)(uint32_t)(lo < hi ? lo : 1);       // empty range: lo 1 > hi 0
            e[range_word + 1] = (int32_t)(uint32_t)(lo < hi ? hi - 1 : 0);
        }
        HC_HIP(hipMemcpyAsync(F0.p, f0_host.data(), sizeof(int32_t) * f0_host.size(), hipMemcpyHostToDevice, R.s));
    } else {
        k_init_cells<<<grid_for(ncell), kBlock, 0, R.s>>>(F0.p, ncell, R.lay[0].W);
        HC_HIP(hipGetLastError());
    }
    if (n_multi > 0 && P.n_vars > 1) {
        // small id blocks: search the blocks' mixed ids in the top levels instead of
        // walking them (taken when the blocks hold fewer ids than a quarter of the
        // smallest top-level operand)
        bool all_v0 = true;
        int64_t len0 = INT64_MAX;
        for (int t = 0; t < P.levels[0].n_ops; ++t) {
            const PlanOp& o = P.levels[0].ops[t];
            all_v0 = all_v0 && o.kind == OP_V0;
            if (o.kind == OP_V0) len0 = std::min<int64_t>(len0, atoms[o.atom]->level_len[0]);
        }
        std::vector<uint64_t> slots((size_t)ncell + 1, 0);
        for (int64_t t = 0; t < ncell; ++t) {
            const int64_t lo = std::max<int64_t>(multi_ranges[2 * t], 0);
            const int64_t hi = std::min<int64_t>(multi_ranges[2 * t + 1], (int64_t)1 << b);
            slots[(size_t)t + 1] = slots[(size_t)t] + (uint64_t)(hi > lo ? hi - lo : 0);
        }
        const uint64_t total = slots[(size_t)ncell];
        if (all_v0 && total <= ((uint64_t)1 << 27) && (int64_t)total * 4 <= len0) R.id_slots = std::move(slots);
    }
    R.run_level(0, F0.p, F0.p, ncell);
    unsigned long long a[3] = {0, 0, 0};
    HC_HIP(hipMemcpyAsync(a, R.acc.p, sizeof(a), hipMemcpyDeviceToHost, R.s));
    if (cell_counts)
        HC_HIP(hipMemcpyAsync(cell_counts, cells.p, sizeof(unsigned long long) * ngroup, hipMemcpyDeviceToHost, R.s));
    HC_HIP(hipStreamSynchronize(R.s));
    R.check_cancel();   // a kernel may have left early
    if (emit) {
        *count = (uint64_t)R.out_count;
        if (n_out) *n_out = R.out_count;
    } else {
        *count = a[0];
        if (digest) {
            digest[0] = a[1];
            digest[1] = a[2];
        }
    }
    if (ctx->profiling) {
        HC_HIP(hipEventRecord(t1, R.s));
        HC_HIP(hipEventSynchronize(t1));
        float ms = 0;
        HC_HIP(hipEventElapsedTime(&ms, t0, t1));
        ctx->timing.total_ms = ms;
        ctx->timing.leaf_ms = R.leaf_ms;
        ctx->timing.leaf_launches = R.leaf_launches;
        ctx->timing.leaf_items = R.leaf_items;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    } else {
        ctx->timing = hc_timing{};
        ctx->timing.leaf_items = R.leaf_items;
    }
}

double small_join_count_bytes(const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                              const int32_t* shares, uint32_t flags);

// Upper bound of the device memory one join call allocates (frontiers, per-level
// step buffers, match words, lifted-intersection pools, work-queue tables), from
// host-side CoCo statistics only.  Entries of F_{i+1} are bounded by those of F_i
// times the longest list of level i's shortest operand (a predicate bounds it by
// its id range); below F_0 every frontier chunk, pool and match-word array holds at
// most max(cap, one entry's elements) items, cap being the chunking cap of the call.
uint64_t join_workspace_bound(const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                              const int32_t* shares, uint32_t flags, int64_t n_queries, int64_t first_width,
                              int64_t cap_entries, bool with_small_path) {
    const Plan P = compile_plan(q, order, !(flags & HC_NO_REWRITE), n_queries > 0 ? 1 : 0);
    const double kCap = (double)cap_entries;   // frontier entries / pool elements per chunk
    int K = 0;
    for (int v = 0; v < P.n_vars; ++v) K += (shares && n_queries == 0) ? shares[v] : 0;
    auto op_max = [&](const PlanOp& o) -> double {
        const hc_coco* c = atoms[o.atom];
        return o.kind == OP_CHILD ? (double)c->max_children[o.lvl - 1] : (double)c->level_len[0];
    };
    double gmax[kMaxGroups];
    for (int g = 0; g < P.n_groups; ++g) {
        double m = 1e30;
        for (int t = 0; t < P.groups[g].n_ops; ++t) m = std::min(m, op_max(P.groups[g].ops[t]));
        gmax[g] = m;
    }
    double E = n_queries > 0 ? (double)n_queries : std::ldexp(1.0, K);
    double bytes = (double)(1 << 20);   // allocation granularity of the many small buffers
    bytes += 8.0 * E + (n_queries > 0 ? 12.0 * E : 0.0);   // per-cell (per-query) counts, query ranges
    // Tables the operands take at set-up (Runner::make_op): the key range of a top
    // level per coordinate (8 bytes per coordinate of a share, or of the segment
    // bits) and, per (atom, CoCo level, share), the child sub-range table of
    // nodes * (2^k + 1) + 1 int32 when it has at most cap entries.
    {
        const int seg_bits = atoms[0]->key_bits - atoms[0]->mix_bits;
        std::vector<uint64_t> tab_keys;
        auto op_tables = [&](const PlanOp& o, int var) {
            const int k = (shares && n_queries == 0) ? shares[var] : 0;
            if (o.kind == OP_V0) {
                const int vk = k > 0 ? k : seg_bits;
                if (vk > 0) bytes += 8.0 * std::ldexp(1.0, vk);
            } else if (o.kind == OP_CHILD && k > 0) {
                const double nodes = (double)atoms[o.atom]->level_len[o.lvl - 1];
                const double entries = nodes * (std::ldexp(1.0, k) + 1.0);
                const uint64_t key = ((uint64_t)o.atom << 16) | ((uint64_t)o.lvl << 8) | (uint64_t)k;
                if (entries <= kCap && std::find(tab_keys.begin(), tab_keys.end(), key) == tab_keys.end()) {
                    tab_keys.push_back(key);
                    bytes += 4.0 * (entries + 1.0);
                }
            }
        };
        for (int i = 0; i < P.n_vars; ++i)
            for (int t = 0; t < P.levels[i].n_ops; ++t) op_tables(P.levels[i].ops[t], P.levels[i].var);
        for (int g = 0; g < P.n_groups; ++g)
            for (int t = 0; t < P.groups[g].n_ops; ++t) op_tables(P.groups[g].ops[t], P.groups[g].var);
    }
    const double setup_bytes = bytes;   // slack, per-cell counts and set-up tables, common to both paths
    double chunk = 1e30;   // entries of one frontier chunk: F_0 is never split
    for (int i = 0; i < P.n_vars; ++i) {
        const PlanLevel& L = P.levels[i];
        double m = 1e30;
        for (int t = 0; t < L.n_ops; ++t)
            m = std::min(m, L.ops[t].kind == OP_TMP ? gmax[L.ops[t].group] : op_max(L.ops[t]));
        if (q->var_lo && q->var_hi && q->var_hi[L.var] > q->var_lo[L.var])
            m = std::min(m, (double)q->var_hi[L.var] - (double)q->var_lo[L.var]);
        if (i == 0 && n_queries > 0 && first_width > 0) m = std::min(m, (double)first_width);
        const double n = std::min(E, chunk);
        const Layout Li = make_layout(P, i);
        bytes += n * 4.0 * (Li.W + (i == 0 && n_queries > 0 ? 2 : 0));   // F_i
        bytes += n * (8.0 * L.n_ops + 16.0) + 8.0;             // ranges, iterated operand, length, prefix
        for (int g = 0; g < P.n_groups; ++g) {
            if (P.groups[g].lift != i) continue;
            // a pool holds at most the cap, or one entry's elements when that is larger
            const double pool = std::min(n * gmax[g], std::max(kCap, gmax[g]));
            bytes += n * (8.0 * P.groups[g].n_ops + 16.0) + 8.0;
            bytes += pool * 4.0 * (1 + P.groups[g].n_ops) + (pool / 64 + 1) * 16.0;
            bytes += pool * 4.0 * P.groups[g].n_ops;                       // positions of the bitmap pass
        }
        const double items = std::min(n * m, 1e18);
        const double citems = std::min(items, std::max(kCap, m));   // elements of one expand / emit chunk
        if (i == 0 && n_queries > 0)   // id-block search of a request batch: found flag, key, rank
            bytes += std::min(items, kCap) * 24.0 + 8.0 * (n + 1);
        if (i + 1 < P.n_vars) {
            bytes += (citems / 64 + 1) * 16.0;   // match words of a chunk
            bytes += citems * 4.0 * L.n_ops;     // positions of the bitmap pass
        }
        // work-queue chunk table: chunks of 4096 elements, or fewer than 16384 smaller ones
        bytes += (std::max(items / 2048.0, 16384.0) + 1) * 8.0 + 64.0;
        E = std::min(E * m, 1e18);
        chunk = std::max(kCap, m);
    }
    // a small count runs the device-sized sequence instead (fixed capacities)
    if (n_queries == 0 && with_small_path)
        bytes = std::max(bytes, setup_bytes + small_join_count_bytes(q, atoms, order, shares, flags));
    return (uint64_t)std::min(bytes, 1.8e19);
}

// ---------------------------------------------------------------- device-sized joins (captured graphs)
// The same levels as Runner::run_level, with every count read by the kernel that
// needs it from a DevSizes block the kernel before it wrote: no host read-back
// between launches, so the whole sequence is captured once in a HIP graph and
// replayed.  Frontiers and match-word arrays have fixed capacities; a level that
// exceeds one raises the overflow word, the levels after it see no entries, and
// the caller's result then comes from the eager path.

// Zero the control words (per-level sizes, overflow word, accumulators) and set
// F_0's size.
__global__ void k_graph_start(uint64_t* __restrict__ ctl, int64_t n_ctl, uint64_t n0) {
    for (int64_t i = threadIdx.x; i < n_ctl; i += blockDim.x) ctl[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) ctl[0] = n0;   // DevSizes::n of level 0
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_copy_u64(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = *src;
}

// Empties a level once the overflow word is raised: after a lifted intersection that
// overflowed, the level's entries would reference pool ranges this replay never
// wrote.
__global__ void k_drop_on_overflow(uint64_t* __restrict__ n, const unsigned long long* __restrict__ overflow) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && *overflow) *n = 0;
}

// After the entry scan: the level's elements (checked against item_cap when it is
// nonzero; beyond it the overflow word is raised and the level emptied), the
// chunking of its passes (chosen as launch_probe chooses it, with
// chunks grown until they fit the chunk table of chunk_cap entries) and the table
// itself.  Every thread derives the chunking from the scanned total; the first
// records it and resets the queues.
__global__ void k_size_chunks(DevSizes* __restrict__ d, const uint64_t* __restrict__ prefix, uint64_t item_cap,
                              uint64_t chunk_cap, uint64_t min_chunks, unsigned long long* __restrict__ overflow,
                              int64_t* __restrict__ ce) {
    const int64_t n = (int64_t)d->n;
    uint64_t total = prefix[n];
    const bool over = item_cap && total > item_cap;
    if (over) total = 0;
    uint64_t cs = kChunk;
    while (cs > kMinChunk && total / cs < min_chunks) cs >>= 1;
    while ((total + cs - 1) / cs > chunk_cap) cs <<= 1;
    const uint64_t nc = (total + cs - 1) / cs;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (over) {
            // the level's entries are dropped too, so no later kernel of the sequence
            // reads their element ranks (other threads then read n = 0 or an n whose
            // total overflows: either way no chunk)
            *overflow = 1ull;
            d->n = 0;
        }
        d->total = total;
        d->chunk_sz = cs;
        d->n_chunks = nc;
        d->nw = (total + 63) >> 6;
        d->got = 0;
        for (int x = 0; x < kXcd; ++x) d->queue[x] = 0;
    }
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nc; t += (uint64_t)gridDim.x * blockDim.x)
        ce[t] = find_entry(prefix, 0, n, t * cs);
}

// After the match-word scan: the matches, the next frontier's size (checked
// against its capacity) and a fresh queue for the materialising pass, which does
// nothing when there is no match or the next frontier would overflow.
__global__ void k_size_matches(DevSizes* __restrict__ d, DevSizes* __restrict__ next,
                               const uint64_t* __restrict__ wpre, uint64_t next_cap,
                               unsigned long long* __restrict__ overflow) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint64_t got = wpre[d->nw];
    d->got = got;
    if (next) {
        if (got > next_cap) {
            *overflow = 1ull;
            got = 0;
        }
        next->n = got;
    }
    if (got == 0) d->n_chunks = 0;
    for (int x = 0; x < kXcd; ++x) d->queue[x] = 0;
}

static uint64_t persistent_blocks(const KData& D) {
    return D.grid_limit > 0 ? std::max<uint64_t>(kXcd, (uint64_t)D.grid_limit / kXcd * kXcd) : kPersistBlocks;
}

// One pass of a level over its elements, every count from d (the grid is the full
// persistent grid; waves leave when their XCD's queue is empty).
template <int MODE>
static void launch_probe_dev(const KData& D, const KStep& S, const int32_t* F, const Seg& G, const uint64_t* prefix,
                             const int64_t* ce, DevSizes* d, uint64_t* words, unsigned long long* acc,
                             const uint64_t* wprefix, MatOut out, hipStream_t s) {
    const unsigned blocks = (unsigned)persistent_blocks(D);
#define HC_PROBE2D(N)                                                                                     \
    k_probe2<MODE, N, 0, true><<<blocks, kBlock, 0, s>>>(D, S, F, G, prefix, 0, 0, 0, 0, ce, d->queue, 0, 0, \
                                                         words, acc, wprefix, out, d)
    switch (S.n_ops) {
        case 1: HC_PROBE2D(1); break;
        case 2: HC_PROBE2D(2); break;
        case 3: HC_PROBE2D(3); break;
        default: HC_PROBE2D(4); break;
    }
#undef HC_PROBE2D
    HC_HIP(hipGetLastError());
}

}  // namespace hc

// Device buffers of one level of a captured join.
struct GraphLevel {
    hc::DevBuf<int32_t> F;          // F_i (ecap entries)
    hc::DevBuf<int32_t> seg, iter;  // prepared ranges and iterated operand
    hc::DevBuf<uint32_t> m;
    hc::DevBuf<uint64_t> prefix, scan_ws;
    hc::DevBuf<int64_t> ce;         // work-queue chunk table
    hc::DevBuf<uint64_t> words, wpre, wscan_ws;
    hc::DevBuf<int32_t> pos;        // positions found by the bitmap pass
    hc::Seg G{};
    int64_t ecap = 0, ce_cap = 0;
};

struct hc_join_graph {
    hc_ctx* ctx = nullptr;
    std::unique_ptr<hc::Runner> R;
    // the call, kept for the eager path
    std::vector<int32_t> arity, vars, order, shares;
    std::vector<int64_t> lo, hi;
    hc_query q{};
    std::vector<const hc_coco*> atoms;
    uint32_t flags = 0;
    int32_t cell_group = -1;   // >= 0: per-cell counts in groups of 2^cell_group cells
    void* out = nullptr;       // emit: device rows
    int64_t capacity = 0;
    // capacities and buffers
    int64_t ncell = 0, ngroup = 0, fcap = 0, icap = 0;
    std::vector<GraphLevel> lv;
    std::vector<GraphLevel> grp;   // per lifted intersection: its step's buffers (F unused)
    hc::DevBuf<uint64_t> ctl;   // DevSizes per level and per lifted intersection, then the
                                // overflow word and 4 accumulators
    hc::DevBuf<unsigned long long> cells;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int launched = 0;
    ~hc_join_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

namespace hc {

constexpr int kCtlPerLevel = (int)(sizeof(DevSizes) / sizeof(uint64_t));

static void graph_record(hc_join_graph* g, hipStream_t s) {
    Runner& R = *g->R;
    const int nv = R.P.n_vars, ng = R.P.n_groups;
    uint64_t* ctl = g->ctl.p;
    auto dsz = [&](int i) { return (DevSizes*)(ctl + (size_t)kCtlPerLevel * i); };   // groups at nv + g
    unsigned long long* ovf = (unsigned long long*)(ctl + (size_t)kCtlPerLevel * (nv + ng));
    unsigned long long* acc = ovf + 1;
    const bool emit = g->out != nullptr;
    const uint64_t min_chunks = persistent_blocks(R.D) * kWaves;
    k_graph_start<<<1, kBlock, 0, s>>>(ctl, (int64_t)kCtlPerLevel * (nv + ng) + 8, (uint64_t)g->ncell);
    HC_HIP(hipGetLastError());
    if (g->cell_group >= 0) {
        k_zero_u64<<<grid_for(g->ngroup), kBlock, 0, s>>>(g->cells.p, g->ngroup);
        HC_HIP(hipGetLastError());
    }
    k_init_cells<<<grid_for(g->ncell), kBlock, 0, s>>>(g->lv[0].F.p, g->ncell, R.lay[0].W);
    HC_HIP(hipGetLastError());
    for (int i = 0; i < nv; ++i) {
        GraphLevel& L = g->lv[i];
        const KStep& S = R.level_step[i];
        DevSizes* d = dsz(i);
        const bool leaf = i == nv - 1;
        const bool bitmap = !leaf || emit;
        // lifted intersections computed on this frontier (Section 6.1): the same
        // passes as a level over the group's operands, their matches written to the
        // group's pool, and every entry's (offset, length) into its words
        for (int gi = 0; gi < ng; ++gi) {
            if (R.P.groups[gi].lift != i) continue;
            GraphLevel& GG = g->grp[gi];
            const KStep& GS = R.group_step[gi];
            DevSizes* dg = dsz(nv + gi);
            k_copy_u64<<<1, 64, 0, s>>>(&dg->n, &d->n);
            HC_HIP(hipGetLastError());
            k_prep<<<grid_for(L.ecap, 512), kBlock, 0, s>>>(R.D, GS, L.F.p, 0, L.ecap, GG.G, &dg->n);
            HC_HIP(hipGetLastError());
            scan_exclusive_dn(LoadU32{GG.m.p}, GG.prefix.p, &dg->n, L.ecap, GG.scan_ws.p, s);
            k_size_chunks<<<grid_for(GG.ce_cap, 512), kBlock, 0, s>>>(dg, GG.prefix.p, (uint64_t)g->icap,
                                                                     (uint64_t)GG.ce_cap, min_chunks, ovf, GG.ce.p);
            HC_HIP(hipGetLastError());
            MatOut gb{};
            gb.pos = GG.pos.p;
            launch_probe_dev<M_BITMAP>(R.D, GS, L.F.p, GG.G, GG.prefix.p, GG.ce.p, dg, GG.words.p, nullptr, nullptr, gb,
                                       s);
            scan_exclusive_dn(LoadPopc{GG.words.p}, GG.wpre.p, &dg->nw, g->icap / 64 + 1, GG.wscan_ws.p, s);
            k_size_matches<<<1, 64, 0, s>>>(dg, nullptr, GG.wpre.p, 0, ovf);
            HC_HIP(hipGetLastError());
            MatOut gt{};
            gt.pos = GG.pos.p;
            gt.tval = R.tmp_val[gi].p;
            for (int u = 0; u < GS.n_src; ++u) gt.tsrc[u] = R.tmp_src[gi][u].p;
            launch_probe_dev<M_TMPW>(R.D, GS, L.F.p, GG.G, GG.prefix.p, GG.ce.p, dg, GG.words.p, nullptr, GG.wpre.p,
                                     gt, s);
            k_tmp_refs<<<grid_for(L.ecap, 512), kBlock, 0, s>>>(L.F.p, R.lay[i].W, R.lay[i].tmp_word[gi], GG.prefix.p,
                                                                0, 0, 0, GG.words.p, GG.wpre.p, 0, &dg->n);
            HC_HIP(hipGetLastError());
            k_drop_on_overflow<<<1, 64, 0, s>>>(&d->n, ovf);
            HC_HIP(hipGetLastError());
        }
        k_prep<<<grid_for(L.ecap, 512), kBlock, 0, s>>>(R.D, S, L.F.p, 0, L.ecap, L.G, &d->n);
        HC_HIP(hipGetLastError());
        scan_exclusive_dn(LoadU32{L.m.p}, L.prefix.p, &d->n, L.ecap, L.scan_ws.p, s);
        k_size_chunks<<<grid_for(L.ce_cap, 512), kBlock, 0, s>>>(d, L.prefix.p, bitmap ? (uint64_t)g->icap : 0,
                                                                (uint64_t)L.ce_cap, min_chunks, ovf, L.ce.p);
        HC_HIP(hipGetLastError());
        if (!bitmap) {
            if (g->cell_group >= 0) {
                MatOut mo{};
                mo.cells = g->cells.p;
                launch_probe_dev<M_CELLS>(R.D, S, L.F.p, L.G, L.prefix.p, L.ce.p, d, nullptr, acc, nullptr, mo, s);
            } else {
                launch_probe_dev<M_COUNT>(R.D, S, L.F.p, L.G, L.prefix.p, L.ce.p, d, nullptr, acc, nullptr, MatOut{},
                                          s);
            }
            continue;
        }
        MatOut mb{};
        mb.pos = L.pos.p;
        launch_probe_dev<M_BITMAP>(R.D, S, L.F.p, L.G, L.prefix.p, L.ce.p, d, L.words.p, nullptr, nullptr, mb, s);
        scan_exclusive_dn(LoadPopc{L.words.p}, L.wpre.p, &d->nw, g->icap / 64 + 1, L.wscan_ws.p, s);
        k_size_matches<<<1, 64, 0, s>>>(d, leaf ? nullptr : dsz(i + 1), L.wpre.p,
                                        leaf ? 0 : (uint64_t)g->lv[i + 1].ecap, ovf);
        HC_HIP(hipGetLastError());
        MatOut mo{};
        mo.pos = L.pos.p;
        if (leaf) {
            mo.rows = g->out;
            mo.row_base = 0;
            mo.row_cap = g->capacity;
            launch_probe_dev<M_EMIT>(R.D, S, L.F.p, L.G, L.prefix.p, L.ce.p, d, L.words.p, nullptr, L.wpre.p, mo, s);
        } else {
            mo.F = g->lv[i + 1].F.p;
            launch_probe_dev<M_EXPAND>(R.D, S, L.F.p, L.G, L.prefix.p, L.ce.p, d, L.words.p, nullptr, L.wpre.p, mo,
                                       s);
        }
    }
}

// capture = false: the buffers and set-up only (the sequence is then launched
// directly on the context's stream, see join_small_device_sized).
static hc_join_graph* graph_create(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                                   const int32_t* shares, uint32_t flags, int32_t cell_group, void* out,
                                   int64_t capacity, int64_t frontier_cap, int64_t item_cap, bool capture,
                                   int64_t leaf_items = 0) {
    std::unique_ptr<hc_join_graph> g(new hc_join_graph());
    g->ctx = ctx;
    // own copies of the call
    int n_terms = 0;
    for (int j = 0; j < q->n_atoms; ++j) n_terms += q->atom_arity[j];
    g->arity.assign(q->atom_arity, q->atom_arity + q->n_atoms);
    g->vars.assign(q->atom_vars, q->atom_vars + n_terms);
    g->q = *q;
    g->q.atom_arity = g->arity.data();
    g->q.atom_vars = g->vars.data();
    if (q->var_lo) {
        g->lo.assign(q->var_lo, q->var_lo + q->n_vars);
        g->hi.assign(q->var_hi, q->var_hi + q->n_vars);
        g->q.var_lo = g->lo.data();
        g->q.var_hi = g->hi.data();
    }
    g->atoms.assign(atoms, atoms + q->n_atoms);
    g->order.assign(order, order + q->n_vars);
    g->shares.assign((size_t)q->n_vars, 0);
    if (shares) g->shares.assign(shares, shares + q->n_vars);
    g->flags = flags;
    g->cell_group = cell_group;
    g->out = out;
    g->capacity = capacity;
    g->fcap = frontier_cap > 0 ? frontier_cap : (int64_t)1 << 20;
    g->icap = item_cap > 0 ? item_cap : (int64_t)1 << 22;
    HC_REQUIRE(g->fcap <= ((int64_t)1 << 28) && g->icap <= ((int64_t)1 << 30), HC_ERR_INVALID,
               "graph capacities above 2^28 entries or 2^30 elements");
    HC_REQUIRE(!(out && cell_group >= 0), HC_ERR_INVALID, "a graph either emits rows or counts per cell");
    g->R.reset(new Runner(ctx, ctx->alloc));
    Runner& R = *g->R;
    setup_runner(R, ctx, &g->q, g->atoms.data(), g->order.data(), g->shares.data(), flags, out != nullptr, false,
                 out, capacity, 0, nullptr, 0, cell_group >= 0);
    const Plan& P = R.P;
    for (int i = 0; i < P.n_vars; ++i)
        HC_REQUIRE(P.levels[i].n_ops <= 4, HC_ERR_UNSUPPORTED, "captured joins take at most 4 operands per level");
    for (int gi = 0; gi < P.n_groups; ++gi)
        HC_REQUIRE(P.groups[gi].n_ops <= 4, HC_ERR_UNSUPPORTED,
                   "captured joins take at most 4 operands per lifted intersection");
    HC_REQUIRE(R.search_mode == SEARCH_WINDOW, HC_ERR_UNSUPPORTED, "captured joins use the default search");
    g->ncell = (int64_t)1 << R.K;
    HC_REQUIRE(cell_group <= R.K, HC_ERR_INVALID, "cell groups larger than the cells");
    R.D.cell_group = cell_group > 0 ? cell_group : 0;
    g->ngroup = cell_group >= 0 ? g->ncell >> cell_group : 0;
    if (cell_group >= 0) g->cells = DevBuf<unsigned long long>(R.A, (size_t)g->ngroup);
    const int nv = P.n_vars;
    g->ctl = DevBuf<uint64_t>(R.A, (size_t)kCtlPerLevel * (nv + P.n_groups) + 8);
    g->lv.resize((size_t)nv);
    for (int i = 0; i < nv; ++i) {
        GraphLevel& L = g->lv[i];
        const KStep& S = R.level_step[i];
        const bool leaf = i == nv - 1;
        const bool bitmap = !leaf || out != nullptr;
        L.ecap = i == 0 ? g->ncell : g->fcap;
        L.F = DevBuf<int32_t>(R.A, (size_t)L.ecap * (size_t)R.lay[i].W);
        L.seg = DevBuf<int32_t>(R.A, (size_t)(2 * S.n_ops) * (size_t)L.ecap);
        L.iter = DevBuf<int32_t>(R.A, (size_t)L.ecap);
        L.m = DevBuf<uint32_t>(R.A, (size_t)L.ecap);
        L.prefix = DevBuf<uint64_t>(R.A, (size_t)L.ecap + 1);
        L.scan_ws = DevBuf<uint64_t>(R.A, (size_t)scan_dn_ws_size(L.ecap));
        L.G.stride = L.ecap;
        L.G.seg = L.seg.p;
        L.G.iter = L.iter.p;
        L.G.m = L.m.p;
        // chunk table: chunks of at least kMinChunk elements over the item capacity,
        // or (a counting leaf) 2^20 chunks, larger ones beyond 2^32 elements (fewer
        // when a bound on the leaf's elements is known; chunks grow to fit)
        L.ce_cap = bitmap ? g->icap / (int64_t)kMinChunk + 1
                          : (leaf_items > 0 ? std::min<int64_t>((int64_t)1 << 20, leaf_items / (int64_t)kMinChunk + 1)
                                            : (int64_t)1 << 20);
        L.ce = DevBuf<int64_t>(R.A, (size_t)L.ce_cap + 1);
        if (bitmap) {
            const int64_t nw = g->icap / 64 + 1;
            L.words = DevBuf<uint64_t>(R.A, (size_t)nw + 1);
            L.wpre = DevBuf<uint64_t>(R.A, (size_t)nw + 1);
            L.wscan_ws = DevBuf<uint64_t>(R.A, (size_t)scan_dn_ws_size(nw));
            L.pos = DevBuf<int32_t>(R.A, (size_t)S.n_ops * (size_t)g->icap);
        }
    }
    // lifted intersections: step buffers over the frontier they are lifted to, and a
    // pool of item_cap elements (with the positions of its sources)
    g->grp.resize((size_t)P.n_groups);
    for (int gi = 0; gi < P.n_groups; ++gi) {
        GraphLevel& GG = g->grp[gi];
        const KStep& GS = R.group_step[gi];
        const int64_t ecap = g->lv[(size_t)P.groups[gi].lift].ecap;
        GG.ecap = ecap;
        GG.seg = DevBuf<int32_t>(R.A, (size_t)(2 * GS.n_ops) * (size_t)ecap);
        GG.iter = DevBuf<int32_t>(R.A, (size_t)ecap);
        GG.m = DevBuf<uint32_t>(R.A, (size_t)ecap);
        GG.prefix = DevBuf<uint64_t>(R.A, (size_t)ecap + 1);
        GG.scan_ws = DevBuf<uint64_t>(R.A, (size_t)scan_dn_ws_size(ecap));
        GG.G.stride = ecap;
        GG.G.seg = GG.seg.p;
        GG.G.iter = GG.iter.p;
        GG.G.m = GG.m.p;
        GG.ce_cap = g->icap / (int64_t)kMinChunk + 1;
        GG.ce = DevBuf<int64_t>(R.A, (size_t)GG.ce_cap + 1);
        const int64_t nw = g->icap / 64 + 1;
        GG.words = DevBuf<uint64_t>(R.A, (size_t)nw + 1);
        GG.wpre = DevBuf<uint64_t>(R.A, (size_t)nw + 1);
        GG.wscan_ws = DevBuf<uint64_t>(R.A, (size_t)scan_dn_ws_size(nw));
        GG.pos = DevBuf<int32_t>(R.A, (size_t)GS.n_ops * (size_t)g->icap);
        R.grow_tmp(gi, g->icap);   // the pool (also sets the kernels' pool pointers)
    }
    if (!capture) return g.release();
    HC_HIP(hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking));
    HC_HIP(hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal));
    try {
        graph_record(g.get(), g->cs);
    } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(g->cs, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    HC_HIP(hipStreamEndCapture(g->cs, &g->graph));
    HC_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    // the set-up tables were computed on the context's stream, where the replays run
    return g.release();
}

hc_join_graph* join_graph_create(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                                 const int32_t* shares, uint32_t flags, int32_t cell_group, void* out,
                                 int64_t capacity, int64_t frontier_cap, int64_t item_cap) {
    return graph_create(ctx, q, atoms, order, shares, flags, cell_group, out, capacity, frontier_cap, item_cap, true);
}

// Frontier and element bounds of a join from the CoCo statistics alone: F_0 has
// 2^K entries; a level's elements are at most its entries times the longest list of
// its shortest operand (a predicate's width bounds it too), and the next frontier at
// most those elements; a lifted intersection's elements at most its frontier's
// entries times its shortest operand's longest list.  False when a level's operand
// is beyond the captured sequence's reach (more than 4 operands).
static bool small_join_bounds(const hc_query* q, const hc_coco* const* atoms, const Plan& P, const int32_t* shares,
                              bool emit, double* fmax, double* imax, double* leaf) {
    auto op_max = [&](const PlanOp& o) -> double {
        const hc_coco* c = atoms[o.atom];
        return o.kind == OP_CHILD ? (double)c->max_children[o.lvl - 1] : (double)c->level_len[0];
    };
    double gmax[kMaxGroups];
    for (int g = 0; g < P.n_groups; ++g) {
        if (P.groups[g].n_ops > 4) return false;
        double m = 1e300;
        for (int t = 0; t < P.groups[g].n_ops; ++t) m = std::min(m, op_max(P.groups[g].ops[t]));
        gmax[g] = m;
    }
    int K = 0;
    for (int v = 0; v < P.n_vars; ++v) K += shares ? shares[v] : 0;
    double E = std::ldexp(1.0, K);
    *fmax = 0;
    *imax = 0;
    for (int i = 0; i < P.n_vars; ++i) {
        const PlanLevel& L = P.levels[i];
        if (L.n_ops > 4) return false;
        for (int g = 0; g < P.n_groups; ++g)
            if (P.groups[g].lift == i) *imax = std::max(*imax, E * gmax[g]);
        double m = 1e300;
        for (int t = 0; t < L.n_ops; ++t)
            m = std::min(m, L.ops[t].kind == OP_TMP ? gmax[L.ops[t].group] : op_max(L.ops[t]));
        if (q->var_lo && q->var_hi[L.var] > q->var_lo[L.var])
            m = std::min(m, (double)q->var_hi[L.var] - (double)q->var_lo[L.var]);
        const double items = E * m;
        if (i + 1 < P.n_vars || emit) *imax = std::max(*imax, items);
        if (i + 1 < P.n_vars) *fmax = std::max(*fmax, items);
        *leaf = items;
        E = items;
    }
    return true;
}

// Bytes the buffers of a device-sized sequence take (graph_create) beyond the set-up
// tables the eager call allocates as well: each rounded up to 512 bytes, and a
// buffer over 1 MiB given 1 MiB more (a caching allocator may hand it a larger free
// block without splitting it).
static double dev_sequence_bytes(const Plan& P, int64_t ncell, int64_t fcap, int64_t icap, int64_t leaf_ce,
                                 bool emit, bool cells) {
    double b = 0;
    auto buf = [&](double bytes) {
        b += std::ceil(std::max(bytes, 1.0) / 512.0) * 512.0 + (bytes > 1048576.0 ? 1048576.0 : 0.0);
    };
    auto step = [&](int n_ops, int64_t ecap, bool bitmap, int64_t ce_cap) {
        buf(2.0 * n_ops * ecap * 4);
        buf(ecap * 4.0);
        buf(ecap * 4.0);
        buf((ecap + 1) * 8.0);
        buf(scan_dn_ws_size(ecap) * 8.0);
        buf((ce_cap + 1) * 8.0);
        if (bitmap) {
            const int64_t nw = icap / 64 + 1;
            buf((nw + 1) * 8.0);
            buf((nw + 1) * 8.0);
            buf(scan_dn_ws_size(nw) * 8.0);
            buf((double)n_ops * icap * 4);
        }
    };
    if (cells) buf(ncell * 8.0);
    buf((kCtlPerLevel * (P.n_vars + P.n_groups) + 8) * 8.0);
    for (int i = 0; i < P.n_vars; ++i) {
        const int64_t ecap = i == 0 ? ncell : fcap;
        const bool bitmap = i + 1 < P.n_vars || emit;
        buf(ecap * 4.0 * make_layout(P, i).W);
        step(P.levels[i].n_ops, ecap, bitmap, bitmap ? icap / (int64_t)kMinChunk + 1 : leaf_ce);
    }
    for (int g = 0; g < P.n_groups; ++g) {
        const int64_t ecap = P.groups[g].lift == 0 ? ncell : fcap;
        step(P.groups[g].n_ops, ecap, true, icap / (int64_t)kMinChunk + 1);
        for (int u = 0; u <= P.groups[g].n_ops; ++u) buf(icap * 4.0);   // the pool and its sources
    }
    return b;
}

// Whether a call takes the device-sized path, and its capacities: joins whose bounds
// stay within 2^20 frontier entries and 2^23 elements per level, with the default
// search (the plan is compiled here; invalid calls are left to the eager path's
// checks).
struct SmallJoin {
    Plan P;
    int64_t ncell = 0, fcap = 0, icap = 0, leaf_items = 0, leaf_ce = 0;
};
static bool small_join_plan(const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                            const int32_t* shares, uint32_t flags, bool emit, SmallJoin* sj) {
    constexpr double kFrontierMax = (double)(1 << 20), kItemsMax = (double)(1 << 23);
    if (flags & ~HC_NO_REWRITE) return false;   // the default search only
    for (int j = 0; j < q->n_atoms; ++j)
        if (!atoms[j]) return false;
    int K = 0;
    for (int v = 0; v < q->n_vars; ++v) K += shares ? shares[v] : 0;
    if (K < 0 || K > 24) return false;
    sj->P = compile_plan(q, order, !(flags & HC_NO_REWRITE));
    double fmax = 0, imax = 0, leaf = 0;
    if (!small_join_bounds(q, atoms, sj->P, shares, emit, &fmax, &imax, &leaf)) return false;
    if (fmax > kFrontierMax || imax > kItemsMax) return false;
    sj->ncell = (int64_t)1 << K;
    sj->fcap = std::max<int64_t>(1024, (int64_t)fmax);
    sj->icap = std::max<int64_t>(4096, (int64_t)imax);
    sj->leaf_items = (int64_t)std::min(leaf, 1e15);
    sj->leaf_ce = std::min<int64_t>((int64_t)1 << 20, sj->leaf_items / (int64_t)kMinChunk + 1);
    return true;
}

// Device memory of a count or per-cell count call on the device-sized path (0 when
// the call takes the eager one); hc_join_workspace_bound includes it.
double small_join_count_bytes(const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                              const int32_t* shares, uint32_t flags) {
    SmallJoin sj;
    if (!small_join_plan(q, atoms, order, shares, flags, false, &sj)) return 0.0;
    return dev_sequence_bytes(sj.P, sj.ncell, sj.fcap, sj.icap, sj.leaf_ce, false, true);
}

bool join_small_device_sized(hc_ctx* ctx, const hc_query* q, const hc_coco* const* atoms, const int32_t* order,
                             const int32_t* shares, uint32_t flags, int32_t cell_group, void* out, int64_t capacity,
                             uint64_t* count, uint64_t* cell_counts, int64_t* n_out) {
    SmallJoin sj;
    if (!small_join_plan(q, atoms, order, shares, flags, out != nullptr, &sj)) return false;
    std::unique_ptr<hc_join_graph> g(graph_create(ctx, q, atoms, order, shares, flags, cell_group, out, capacity,
                                                  sj.fcap, sj.icap, false, sj.leaf_items));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->profiling) {
        HC_HIP(hipEventCreate(&t0));
        HC_HIP(hipEventCreate(&t1));
        HC_HIP(hipEventRecord(t0, ctx->stream));
    }
    graph_record(g.get(), ctx->stream);
    g->launched = 1;
    int64_t no = 0;
    try {
        join_graph_result(g.get(), count, cell_counts, &no, nullptr);
    } catch (...) {
        if (n_out) *n_out = no;
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        throw;
    }
    if (n_out) *n_out = no;
    ctx->timing = hc_timing{};
    if (ctx->profiling) {
        HC_HIP(hipEventRecord(t1, ctx->stream));
        HC_HIP(hipEventSynchronize(t1));
        float ms = 0;
        HC_HIP(hipEventElapsedTime(&ms, t0, t1));
        ctx->timing.total_ms = ms;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    return true;
}

void join_graph_launch(hc_join_graph* g) {
    HC_REQUIRE(!g->ctx->cancel.load(), HC_ERR_CANCELLED, "cancelled");
    HC_HIP(hipGraphLaunch(g->exec, g->ctx->stream));
    g->launched = 1;
}

void join_graph_result(hc_join_graph* g, uint64_t* count, uint64_t* cell_counts, int64_t* n_out, int32_t* replayed) {
    HC_REQUIRE(g->launched, HC_ERR_INVALID, "hc_join_graph_result before hc_join_graph_launch");
    hc_ctx* ctx = g->ctx;
    const int nv = g->R->P.n_vars, nc = nv + g->R->P.n_groups;
    std::vector<uint64_t> h((size_t)kCtlPerLevel * nc + 8);
    HC_HIP(hipMemcpyAsync(h.data(), g->ctl.p, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    if (cell_counts && g->cell_group >= 0)
        HC_HIP(hipMemcpyAsync(cell_counts, g->cells.p, sizeof(uint64_t) * (size_t)g->ngroup, hipMemcpyDeviceToHost,
                              ctx->stream));
    HC_HIP(hipStreamSynchronize(ctx->stream));
    g->launched = 0;
    HC_REQUIRE(!ctx->cancel.load(), HC_ERR_CANCELLED, "cancelled");   // a kernel may have left early
    const bool ovf = h[(size_t)kCtlPerLevel * nc] != 0;
    if (!ovf) {
        const uint64_t got = g->out ? h[(size_t)kCtlPerLevel * (nv - 1) + offsetof(DevSizes, got) / 8]
                                    : h[(size_t)kCtlPerLevel * nc + 1];
        *count = got;
        *n_out = (int64_t)got;
        if (replayed) *replayed = 1;
    } else {
        // a frontier or a level's elements exceeded the capacities: the eager path
        if (replayed) *replayed = 0;
        int64_t no = 0;
        join_run(ctx, &g->q, g->atoms.data(), g->order.data(), g->shares.data(), g->flags, g->out != nullptr, count,
                 nullptr, g->out, g->capacity, &no, g->cell_group >= 0 ? cell_counts : nullptr, 0, nullptr, nullptr,
                 0, g->cell_group > 0 ? g->cell_group : 0);
        if (g->out) *count = (uint64_t)no;
        *n_out = g->out ? no : (int64_t)*count;
    }
    if (g->out && *n_out > g->capacity)
        fail(HC_ERR_OVERFLOW, "hc_join_graph_result: " + std::to_string(*n_out) + " rows exceed capacity " +
                                  std::to_string(g->capacity));
}

hc_ctx* join_graph_ctx(const hc_join_graph* g) { return g->ctx; }

void join_graph_destroy(hc_join_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);   // no replay may still use the buffers
    delete g;
}

}  // namespace hc
