/*
 * CPU oracle for the Generic Join hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package's smoke check and the bench's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the GPU
 * library: it works on plain int64 tuple arrays, sorted with qsort, probed with
 * binary search, and never touches a trie index.
 *
 * What it computes (Section 2, Eq. (1), full conjunctive query under set
 * semantics): Q(D) = { t : for every atom j, the projection of t on the
 * variables of atom j is a tuple of R_j }.  Generic Join (Section 2, "Generic
 * Join Algorithm") reaches exactly this set for any variable order: one nested
 * loop per variable X_sigma(i); each loop intersects the columns R_j.X_sigma(i)
 * of the atoms that contain the variable, each relation already restricted by
 * the values bound in the enclosing loops, binds the variable to every value of
 * the intersection and recurses.  The intersection iterates the operand with
 * the fewest candidates and probes the others (Section 2, "in time
 * proportional to the smallest of the sets") -- here by plain binary search
 * on sorted tuple arrays.
 *
 * Optional pieces:
 *  - range predicates lo <= X_v < hi on raw ids (predicate push-down into
 *    the atoms, Section 2), used for chunked output;
 *  - an order-independent digest of the output set (count, sum and xor of a
 *    per-tuple SplitMix64-finaliser chain);
 *  - the galloping work counter of the cost model (Section 6.2, per-level
 *    cost |S| * min N * log2(1 + max N / min N)), expressed as elements
 *    touched: m + sum over the other operands of min(|op|, m*ceil(log2(1+|op|/m)))
 *    where m is the smallest operand (binary atoms only).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OQ_MAX_VARS 8
#define OQ_MAX_ATOMS 16
#define OQ_MAX_ARITY 4

typedef struct {
    int64_t* t;      /* rows x k, columns permuted into variable-order position order */
    int64_t rows;
    int k;
    int var_of_col[OQ_MAX_ARITY];
    int64_t distinct0;  /* number of distinct first-column values */
    int perm[OQ_MAX_ARITY];  /* input column of each sorted column */
    int shared;         /* t is another atom's sorted copy (same input, same column permutation) */
} oq_rel;

typedef struct {
    int n_vars, n_atoms;
    const int* order;              /* order[i] = var id bound at level i */
    int pos[OQ_MAX_VARS];          /* pos[var] = level */
    oq_rel rel[OQ_MAX_ATOMS];
    int n_ops[OQ_MAX_VARS];        /* atoms containing the level's variable */
    int ops[OQ_MAX_VARS][OQ_MAX_ATOMS];
    const int64_t* lo;             /* nullable range predicates */
    const int64_t* hi;
    int64_t* out;
    int64_t out_cap;
    int want_digest;
    int want_work;
} oq_state;

typedef struct {
    int64_t lo[OQ_MAX_ATOMS], hi[OQ_MAX_ATOMS];
    int depth[OQ_MAX_ATOMS];
    int64_t val[OQ_MAX_VARS];
    uint64_t count, dsum, dxor;
    uint64_t work[OQ_MAX_VARS];
    int64_t* out_pos;              /* shared cursor */
} oq_frame;

static int g_k;  /* qsort comparator width (set before each qsort, single-threaded) */
static int cmp_rows(const void* a, const void* b) {
    const int64_t* x = (const int64_t*)a;
    const int64_t* y = (const int64_t*)b;
    for (int c = 0; c < g_k; ++c) {
        if (x[c] < y[c]) return -1;
        if (x[c] > y[c]) return 1;
    }
    return 0;
}

/* SplitMix64 finaliser (Steele, Lea, Flood 2014). */
static uint64_t fmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Digest of one head-order tuple: h <- F(h ^ (t_k + (k+1)*GAMMA)). */
static uint64_t tuple_hash(const int64_t* t, int n) {
    uint64_t h = 0x6A09E667F3BCC909ULL;
    for (int k = 0; k < n; ++k)
        h = fmix64(h ^ ((uint64_t)t[k] + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ULL));
    return h;
}

/* first row in [lo,hi) whose column c is >= v (rows sorted on column c in range) */
static int64_t lower_row(const oq_rel* r, int c, int64_t lo, int64_t hi, int64_t v) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (r->t[mid * r->k + c] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
static int64_t upper_row(const oq_rel* r, int c, int64_t lo, int64_t hi, int64_t v) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (r->t[mid * r->k + c] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Number of distinct values of column c in rows [lo,hi) of r, for the work counter.
 * For binary atoms the operand is either the whole first column (distinct0) or a
 * child list, whose rows are all distinct. */
static int64_t operand_size(const oq_state* s, int a, const oq_frame* f) {
    const oq_rel* r = &s->rel[a];
    if (f->depth[a] == 0) return r->distinct0;
    return f->hi[a] - f->lo[a];
}

static uint64_t ceil_log2_ratio(int64_t big, int64_t m) {
    /* ceil(log2(1 + big/m)) in exact integer arithmetic: smallest e with 2^e >= 1 + big/m,
       i.e. m * 2^e >= m + big. */
    uint64_t e = 0;
    while ((uint64_t)m << e < (uint64_t)(m + big)) ++e;
    return e;
}

static void gj_level(const oq_state* s, oq_frame* f, int i);

static void bind_and_recurse(const oq_state* s, oq_frame* f, int i, int64_t v,
                             const int64_t* nlo, const int64_t* nhi) {
    int var = s->order[i];
    int na = s->n_ops[i];
    int64_t slo[OQ_MAX_ATOMS], shi[OQ_MAX_ATOMS];
    for (int q = 0; q < na; ++q) {
        int a = s->ops[i][q];
        slo[q] = f->lo[a]; shi[q] = f->hi[a];
        f->lo[a] = nlo[q]; f->hi[a] = nhi[q]; f->depth[a] += 1;
    }
    f->val[var] = v;
    gj_level(s, f, i + 1);
    for (int q = 0; q < na; ++q) {
        int a = s->ops[i][q];
        f->lo[a] = slo[q]; f->hi[a] = shi[q]; f->depth[a] -= 1;
    }
}

static void emit(const oq_state* s, oq_frame* f) {
    f->count += 1;
    if (s->want_digest) {
        uint64_t h = tuple_hash(f->val, s->n_vars);
        f->dsum += h; f->dxor ^= h;
    }
    if (s->out) {
        int64_t p;
#pragma omp atomic capture
        p = (*f->out_pos)++;
        if (p < s->out_cap) memcpy(s->out + p * s->n_vars, f->val, sizeof(int64_t) * s->n_vars);
    }
}

/* Level i: intersect the candidate columns of the atoms containing order[i]. */
static void gj_level(const oq_state* s, oq_frame* f, int i) {
    if (i == s->n_vars) { emit(s, f); return; }
    int var = s->order[i];
    int na = s->n_ops[i];
    /* pick the operand with the fewest candidate rows */
    int best = 0;
    for (int q = 1; q < na; ++q) {
        int a = s->ops[i][q], b = s->ops[i][best];
        if (f->hi[a] - f->lo[a] < f->hi[b] - f->lo[b]) best = q;
    }
    if (s->want_work) {
        int64_t m = -1;
        for (int q = 0; q < na; ++q) {
            int64_t z = operand_size(s, s->ops[i][q], f);
            if (m < 0 || z < m) m = z;
        }
        uint64_t w = (uint64_t)m;
        int skipped = 0;
        for (int q = 0; q < na; ++q) {
            int64_t z = operand_size(s, s->ops[i][q], f);
            if (z == m && !skipped) { skipped = 1; continue; }
            if (m == 0) continue;
            uint64_t g = (uint64_t)m * ceil_log2_ratio(z, m);
            w += (uint64_t)z < g ? (uint64_t)z : g;
        }
        f->work[i] += w;
    }
    int ab = s->ops[i][best];
    const oq_rel* rb = &s->rel[ab];
    int cb = f->depth[ab];
    int64_t nlo[OQ_MAX_ATOMS], nhi[OQ_MAX_ATOMS];
    int64_t r = f->lo[ab];
    while (r < f->hi[ab]) {
        int64_t v = rb->t[r * rb->k + cb];
        int64_t r1 = upper_row(rb, cb, r, f->hi[ab], v);
        int ok = 1;
        if (s->lo && (v < s->lo[var] || v >= s->hi[var])) ok = 0;
        for (int q = 0; q < na && ok; ++q) {
            int a = s->ops[i][q];
            if (q == best) { nlo[q] = r; nhi[q] = r1; continue; }
            const oq_rel* ra = &s->rel[a];
            int ca = f->depth[a];
            int64_t e0 = lower_row(ra, ca, f->lo[a], f->hi[a], v);
            int64_t e1 = upper_row(ra, ca, e0, f->hi[a], v);
            if (e0 == e1) ok = 0;
            nlo[q] = e0; nhi[q] = e1;
        }
        if (ok) bind_and_recurse(s, f, i, v, nlo, nhi);
        r = r1;
    }
}

/*
 * Run Generic Join.
 *   n_vars, n_atoms, arity[n_atoms], atom_vars[sum arity]: the query (var ids are head order)
 *   rel[j]: row-major int64 tuples of atom j (rows[j] rows), duplicates allowed
 *   order[n_vars]: variable order (a permutation of 0..n_vars-1)
 *   var_lo/var_hi: nullable, per-variable range predicate lo <= x < hi
 *   out/out_cap: nullable output buffer, head-order rows, arbitrary row order
 *   digest: nullable uint64[2] (sum, xor)
 *   work: nullable uint64[n_vars] galloping work counter per level
 * Returns the count, or -1 on an invalid query.
 */
static void free_state(oq_state* s) {
    for (int j = 0; j < OQ_MAX_ATOMS; ++j) {
        if (!s->rel[j].shared) free(s->rel[j].t);
        s->rel[j].t = NULL;
    }
}

/* Sort and deduplicate every atom in variable-order column order; returns 0 or -1. */
static int prepare(oq_state* s, int n_vars, int n_atoms, const int* arity, const int* atom_vars,
                   const int64_t* const* rel, const int64_t* rows, const int* order) {
    if (n_vars < 1 || n_vars > OQ_MAX_VARS || n_atoms < 1 || n_atoms > OQ_MAX_ATOMS) return -1;
    memset(s, 0, sizeof(*s));
    s->n_vars = n_vars; s->n_atoms = n_atoms; s->order = order;
    int seen[OQ_MAX_VARS] = {0};
    for (int i = 0; i < n_vars; ++i) {
        if (order[i] < 0 || order[i] >= n_vars || seen[order[i]]) return -1;
        seen[order[i]] = 1; s->pos[order[i]] = i;
    }
    int covered[OQ_MAX_VARS] = {0};
    const int* av = atom_vars;
    for (int j = 0; j < n_atoms; ++j) {
        int k = arity[j];
        if (k < 1 || k > OQ_MAX_ARITY) { free_state(s); return -1; }
        oq_rel* r = &s->rel[j];
        r->k = k;
        /* columns sorted by the level of their variable */
        int perm[OQ_MAX_ARITY];
        for (int c = 0; c < k; ++c) {
            if (av[c] < 0 || av[c] >= n_vars) { free_state(s); return -1; }
            for (int c2 = 0; c2 < c; ++c2) if (av[c2] == av[c]) { free_state(s); return -1; }
            perm[c] = c; covered[av[c]] = 1;
        }
        for (int x = 1; x < k; ++x)
            for (int y = x; y > 0 && s->pos[av[perm[y]]] < s->pos[av[perm[y - 1]]]; --y) {
                int tmp = perm[y]; perm[y] = perm[y - 1]; perm[y - 1] = tmp;
            }
        for (int c = 0; c < k; ++c) r->var_of_col[c] = av[perm[c]];
        /* an atom over the same input array with the same column permutation as an
           earlier atom reuses that atom's sorted, deduplicated copy */
        int same = -1;
        for (int j2 = 0; j2 < j && same < 0; ++j2) {
            if (rel[j2] != rel[j] || rows[j2] != rows[j] || s->rel[j2].k != k) continue;
            int eq = 1;
            for (int c = 0; c < k; ++c) eq = eq && s->rel[j2].perm[c] == perm[c];
            if (eq) same = j2;
        }
        for (int c = 0; c < k; ++c) r->perm[c] = perm[c];
        if (same >= 0) {
            r->t = s->rel[same].t;
            r->rows = s->rel[same].rows;
            r->distinct0 = s->rel[same].distinct0;
            r->shared = 1;
            av += k;
            continue;
        }
        r->t = (int64_t*)malloc(sizeof(int64_t) * (size_t)(rows[j] > 0 ? rows[j] : 1) * k);
        for (int64_t row = 0; row < rows[j]; ++row)
            for (int c = 0; c < k; ++c) r->t[row * k + c] = rel[j][row * k + perm[c]];
        g_k = k;
        qsort(r->t, (size_t)rows[j], sizeof(int64_t) * k, cmp_rows);
        /* set semantics: drop duplicate rows */
        int64_t w = 0;
        for (int64_t row = 0; row < rows[j]; ++row)
            if (w == 0 || cmp_rows(r->t + row * k, r->t + (w - 1) * k) != 0) {
                if (w != row) memcpy(r->t + w * k, r->t + row * k, sizeof(int64_t) * k);
                ++w;
            }
        r->rows = w;
        r->distinct0 = 0;
        for (int64_t row = 0; row < w; ++row)
            if (row == 0 || r->t[row * k] != r->t[(row - 1) * k]) r->distinct0++;
        av += k;
    }
    for (int v = 0; v < n_vars; ++v) if (!covered[v]) { free_state(s); return -1; }
    for (int i = 0; i < n_vars; ++i) {
        s->n_ops[i] = 0;
        for (int j = 0; j < n_atoms; ++j)
            for (int c = 0; c < s->rel[j].k; ++c)
                if (s->rel[j].var_of_col[c] == order[i]) s->ops[i][s->n_ops[i]++] = j;
    }
    return 0;
}

typedef struct {
    int best;                /* operand of level 0 whose runs are split across threads */
    int64_t nruns;
    int64_t* starts;         /* run start rows, nruns + 1 entries */
} oq_level0;

static void level0_runs(const oq_state* s, oq_level0* L) {
    int na = s->n_ops[0];
    L->best = 0;
    for (int q = 1; q < na; ++q)
        if (s->rel[s->ops[0][q]].rows < s->rel[s->ops[0][L->best]].rows) L->best = q;
    const oq_rel* rb = &s->rel[s->ops[0][L->best]];
    L->nruns = rb->distinct0;
    L->starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L->nruns + 1));
    int64_t q0 = 0;
    for (int64_t row = 0; row < rb->rows; ++row)
        if (row == 0 || rb->t[row * rb->k] != rb->t[(row - 1) * rb->k]) L->starts[q0++] = row;
    L->starts[L->nruns] = rb->rows;
}

/* Generic Join over the level-0 runs [run_lo, run_hi), OpenMP over runs; adds into acc. */
static void run_runs(const oq_state* s, const oq_level0* L, int64_t run_lo, int64_t run_hi,
                     uint64_t* tc, uint64_t* ts, uint64_t* tx, uint64_t* tw, int64_t* out_pos) {
    oq_frame base;
    memset(&base, 0, sizeof(base));
    for (int j = 0; j < s->n_atoms; ++j) { base.lo[j] = 0; base.hi[j] = s->rel[j].rows; base.depth[j] = 0; }
    const int na = s->n_ops[0];
    const int best = L->best;
    const oq_rel* rb = &s->rel[s->ops[0][best]];
#pragma omp parallel
    {
        oq_frame f = base;
        f.out_pos = out_pos;
#pragma omp for schedule(dynamic, 16)
        for (int64_t run = run_lo; run < run_hi; ++run) {
            int64_t r = L->starts[run], r1 = L->starts[run + 1];
            int64_t v = rb->t[r * rb->k];
            int var = s->order[0];
            if (s->lo && (v < s->lo[var] || v >= s->hi[var])) continue;
            int64_t nlo[OQ_MAX_ATOMS], nhi[OQ_MAX_ATOMS];
            int ok = 1;
            for (int q = 0; q < na && ok; ++q) {
                int a = s->ops[0][q];
                if (q == best) { nlo[q] = r; nhi[q] = r1; continue; }
                const oq_rel* ra = &s->rel[a];
                int64_t e0 = lower_row(ra, 0, 0, ra->rows, v);
                int64_t e1 = upper_row(ra, 0, e0, ra->rows, v);
                if (e0 == e1) ok = 0;
                nlo[q] = e0; nhi[q] = e1;
            }
            if (ok) bind_and_recurse(s, &f, 0, v, nlo, nhi);
        }
#pragma omp critical
        {
            *tc += f.count; *ts += f.dsum; *tx ^= f.dxor;
            for (int q = 0; q < OQ_MAX_VARS; ++q) tw[q] += f.work[q];
        }
    }
}

/*
 * Run Generic Join.
 *   n_vars, n_atoms, arity[n_atoms], atom_vars[sum arity]: the query (var ids are head order)
 *   rel[j]: row-major int64 tuples of atom j (rows[j] rows), duplicates allowed
 *   order[n_vars]: variable order (a permutation of 0..n_vars-1)
 *   var_lo/var_hi: nullable, per-variable range predicate lo <= x < hi
 *   out/out_cap: nullable output buffer, head-order rows, arbitrary row order
 *   digest: nullable uint64[2] (sum, xor)
 *   work: nullable uint64[n_vars] galloping work counter per level
 * Returns the count, or -1 on an invalid query.
 */
int64_t oracle_gj(int n_vars, int n_atoms, const int* arity, const int* atom_vars,
                  const int64_t* const* rel, const int64_t* rows, const int* order,
                  const int64_t* var_lo, const int64_t* var_hi,
                  int64_t* out, int64_t out_cap, uint64_t* digest, uint64_t* work,
                  int nthreads) {
    oq_state s;
    if (prepare(&s, n_vars, n_atoms, arity, atom_vars, rel, rows, order) != 0) return -1;
    s.lo = var_lo; s.hi = var_hi;
    s.out = out; s.out_cap = out_cap;
    s.want_digest = digest != NULL;
    s.want_work = work != NULL;
    oq_level0 L;
    level0_runs(&s, &L);
    uint64_t tc = 0, ts = 0, tx = 0, tw[OQ_MAX_VARS] = {0};
    if (s.want_work) {
        /* level-0 intersection work, counted once */
        oq_frame wf;
        memset(&wf, 0, sizeof(wf));
        for (int j = 0; j < n_atoms; ++j) { wf.lo[j] = 0; wf.hi[j] = s.rel[j].rows; }
        int na = s.n_ops[0];
        int64_t m = -1;
        for (int q = 0; q < na; ++q) {
            int64_t z = operand_size(&s, s.ops[0][q], &wf);
            if (m < 0 || z < m) m = z;
        }
        uint64_t w0 = (uint64_t)m;
        int skipped = 0;
        for (int q = 0; q < na; ++q) {
            int64_t z = operand_size(&s, s.ops[0][q], &wf);
            if (z == m && !skipped) { skipped = 1; continue; }
            if (m == 0) continue;
            uint64_t g = (uint64_t)m * ceil_log2_ratio(z, m);
            w0 += (uint64_t)z < g ? (uint64_t)z : g;
        }
        tw[0] += w0;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t out_pos = 0;
    run_runs(&s, &L, 0, L.nruns, &tc, &ts, &tx, tw, &out_pos);
    free(L.starts);
    free_state(&s);
    if (digest) { digest[0] = ts; digest[1] = tx; }
    if (work) for (int q = 0; q < n_vars; ++q) work[q] = tw[q];
    return (int64_t)tc;
}

#ifdef _OPENMP
static double now_s(void) { return omp_get_wtime(); }
#else
#include <time.h>
static double now_s(void) {
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return t.tv_sec + 1e-9 * t.tv_nsec;
}
#endif

/*
 * Timed sample for the CPU baseline: sort once, then run Generic Join on the level-0
 * runs in a seeded random order (a Fisher-Yates shuffle driven by splitmix64, so any
 * prefix is a uniform sample of the first variable's values; an order by value would
 * follow the generator's id structure, e.g. R-MAT's heavy low-bit-zero ids) as ONE
 * parallel loop, like the whole job, in which a thread takes no new run once budget_s
 * seconds of join time have passed.  Heavy runs thus overlap with the others as they
 * do in the whole job, and only the runs in flight at the deadline finish alone.
 * Writes the count of the runs done, the loop's wall time, the busy thread-seconds
 * (the sum over threads of the time from the loop's start to the end of their last
 * run) and the number of runs done; returns the number of level-0 runs (or -1).
 * *sort_s receives the sort + dedup time.
 */
int64_t oracle_gj_timed(int n_vars, int n_atoms, const int* arity, const int* atom_vars,
                        const int64_t* const* rel, const int64_t* rows, const int* order,
                        uint64_t seed, double budget_s, uint64_t* count, double* wall, double* busy,
                        int64_t* runs_done, double* sort_s, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double t0 = now_s();
    oq_state s;
    if (prepare(&s, n_vars, n_atoms, arity, atom_vars, rel, rows, order) != 0) return -1;
    oq_level0 L;
    level0_runs(&s, &L);
    *sort_s = now_s() - t0;
    const int64_t nruns = L.nruns;
    /* position j of the loop runs level-0 run perm[j] */
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nruns + 1));
    for (int64_t j = 0; j < nruns; ++j) perm[j] = j;
    uint64_t st = seed;
    for (int64_t j = nruns - 1; j > 0; --j) {
        st += 0x9E3779B97F4A7C15ull;                 /* splitmix64 step */
        uint64_t k = (uint64_t)(((unsigned __int128)fmix64(st) * (uint64_t)(j + 1)) >> 64);
        int64_t tmp = perm[j]; perm[j] = perm[k]; perm[k] = tmp;
    }
    uint64_t tc = 0;
    double bsum = 0;
    int64_t done = 0;
    volatile int stop = 0;
    double t1 = now_s();
    const double deadline = t1 + budget_s;
#pragma omp parallel
    {
        oq_frame f;
        memset(&f, 0, sizeof(f));
        for (int j = 0; j < s.n_atoms; ++j) { f.lo[j] = 0; f.hi[j] = s.rel[j].rows; f.depth[j] = 0; }
        int64_t out_pos = 0;
        f.out_pos = &out_pos;
        const int na = s.n_ops[0];
        const oq_rel* rb = &s.rel[s.ops[0][L.best]];
        double t_last = t1;
        int64_t my_done = 0;
#pragma omp for schedule(dynamic, 16) nowait
        for (int64_t j = 0; j < nruns; ++j) {
            if (stop) continue;
            int64_t run = perm[j];
            int64_t r = L.starts[run], r1 = L.starts[run + 1];
            int64_t v = rb->t[r * rb->k];
            int64_t nlo[OQ_MAX_ATOMS], nhi[OQ_MAX_ATOMS];
            int ok = 1;
            for (int q = 0; q < na && ok; ++q) {
                int a = s.ops[0][q];
                if (q == L.best) { nlo[q] = r; nhi[q] = r1; continue; }
                const oq_rel* ra = &s.rel[a];
                int64_t e0 = lower_row(ra, 0, 0, ra->rows, v);
                int64_t e1 = upper_row(ra, 0, e0, ra->rows, v);
                if (e0 == e1) ok = 0;
                nlo[q] = e0; nhi[q] = e1;
            }
            if (ok) bind_and_recurse(&s, &f, 0, v, nlo, nhi);
            ++my_done;
            t_last = now_s();
            if (t_last >= deadline) stop = 1;
        }
#pragma omp critical
        { tc += f.count; bsum += t_last - t1; done += my_done; }
    }
    *wall = now_s() - t1;
    *count = tc;
    *busy = bsum;
    *runs_done = done;
    free(perm);
    free(L.starts);
    free_state(&s);
    return nruns;
}

/* Digest of an explicit list of head-order tuples (so tests can digest brute-force
 * or chunked outputs with the same definition). */
void oracle_digest_rows(const int64_t* t, int64_t rows, int n, uint64_t* digest) {
    uint64_t sum = 0, x = 0;
    for (int64_t r = 0; r < rows; ++r) {
        uint64_t h = tuple_hash(t + r * n, n);
        sum += h; x ^= h;
    }
    digest[0] = sum; digest[1] = x;
}
