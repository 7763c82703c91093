/*
 * Textbook subgraph counters used only to pin the oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * These are classical algorithms unrelated to Generic Join, so agreement with
 * the oracle on large graphs is evidence that the oracle has no dropped term or
 * wrong index:
 *  - triangles: the degree-ordered "forward" algorithm (Schank and Wagner 2005;
 *    Latapy 2008): orient every edge from lower to higher (degree, id) rank and
 *    count, for each oriented edge (u, v), the common out-neighbours of u and v;
 *  - 4-cliques: the same orientation (Chiba and Nishizeki 1985 style): for each
 *    oriented edge (u, v), W = out(u) & out(v), then count oriented edges inside W;
 *  - triangles per edge and per vertex (the same forward enumeration, each triangle
 *    credited to its three edges and three vertices), which give the ordered
 *    diamond count sum_e 2 t(e)^2 and the ordered two-triangle count
 *    sum_v (2 t(v))^2 in closed form.
 * Both count unordered subgraphs of a simple undirected graph given as its
 * symmetric edge list (duplicates and self-loops ignored).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    int64_t* off;   /* n+1 */
    int64_t* adj;   /* oriented out-neighbours */
} tb_graph;

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Build the degree-oriented graph from a symmetric edge list. */
static int tb_build(const int64_t* e, int64_t m, tb_graph* g) {
    int64_t n = 0;
    for (int64_t i = 0; i < 2 * m; ++i) {
        if (e[i] < 0) return -1;
        if (e[i] + 1 > n) n = e[i] + 1;
    }
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) if (e[2 * i] != e[2 * i + 1]) off[e[2 * i] + 1]++;
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t* nb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(cur, off, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < m; ++i)
        if (e[2 * i] != e[2 * i + 1]) nb[cur[e[2 * i]]++] = e[2 * i + 1];
    /* dedup neighbour lists to get true degrees */
    for (int64_t v = 0; v < n; ++v) {
        int64_t a = off[v], b = off[v + 1];
        qsort(nb + a, (size_t)(b - a), sizeof(int64_t), cmp_i64);
        int64_t w = 0;
        for (int64_t i = a; i < b; ++i) if (w == 0 || nb[i] != nb[a + w - 1]) nb[a + w++] = nb[i];
        deg[v] = w;
    }
    /* oriented adjacency: keep v->w when rank(v) < rank(w) */
    int64_t* oo = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) {
        int64_t c = 0;
        for (int64_t i = off[v]; i < off[v] + deg[v]; ++i) {
            int64_t w = nb[i];
            if (deg[v] < deg[w] || (deg[v] == deg[w] && v < w)) ++c;
        }
        oo[v + 1] = c;
    }
    for (int64_t v = 0; v < n; ++v) oo[v + 1] += oo[v];
    int64_t* oa = (int64_t*)malloc(sizeof(int64_t) * (size_t)(oo[n] > 0 ? oo[n] : 1));
    for (int64_t v = 0; v < n; ++v) {
        int64_t c = oo[v];
        for (int64_t i = off[v]; i < off[v] + deg[v]; ++i) {
            int64_t w = nb[i];
            if (deg[v] < deg[w] || (deg[v] == deg[w] && v < w)) oa[c++] = w;
        }
    }
    free(deg); free(off); free(nb); free(cur);
    g->n = n; g->off = oo; g->adj = oa;
    return 0;
}

/* e: symmetric edge list, m rows of (u, v). Returns the number of triangles. */
int64_t textbook_triangles(const int64_t* e, int64_t m, int nthreads) {
    tb_graph g;
    if (tb_build(e, m, &g) != 0) return -1;
    uint64_t total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        unsigned char* mark = (unsigned char*)calloc((size_t)g.n + 1, 1);
        uint64_t local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < g.n; ++u) {
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mark[g.adj[i]] = 1;
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) {
                int64_t v = g.adj[i];
                for (int64_t j = g.off[v]; j < g.off[v + 1]; ++j) local += mark[g.adj[j]];
            }
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mark[g.adj[i]] = 0;
        }
#pragma omp atomic
        total += local;
        free(mark);
    }
    free(g.off); free(g.adj);
    return (int64_t)total;
}

/* Returns the number of 4-cliques. */
int64_t textbook_4cliques(const int64_t* e, int64_t m, int nthreads) {
    tb_graph g;
    if (tb_build(e, m, &g) != 0) return -1;
    uint64_t total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        unsigned char* mu = (unsigned char*)calloc((size_t)g.n + 1, 1);
        unsigned char* mw = (unsigned char*)calloc((size_t)g.n + 1, 1);
        int64_t* wl = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g.n + 1));
        uint64_t local = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < g.n; ++u) {
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mu[g.adj[i]] = 1;
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) {
                int64_t v = g.adj[i];
                int64_t nw = 0;
                for (int64_t j = g.off[v]; j < g.off[v + 1]; ++j)
                    if (mu[g.adj[j]]) { wl[nw++] = g.adj[j]; mw[g.adj[j]] = 1; }
                for (int64_t a = 0; a < nw; ++a) {
                    int64_t w = wl[a];
                    for (int64_t j = g.off[w]; j < g.off[w + 1]; ++j) local += mw[g.adj[j]];
                }
                for (int64_t a = 0; a < nw; ++a) mw[wl[a]] = 0;
            }
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mu[g.adj[i]] = 0;
        }
#pragma omp atomic
        total += local;
        free(mu); free(mw); free(wl);
    }
    free(g.off); free(g.adj);
    return (int64_t)total;
}

/* Digest of the ordered output of the 4-clique query on a symmetric relation:
 * every K4 {a,b,c,d} found by the oriented enumeration contributes all 24
 * orderings as head-order tuples.  The per-tuple hash is the digest definition
 * (SplitMix64 finaliser chain over the fields, seeded 0x6A09E667F3BCC909,
 * field k offset by (k+1) * 0x9E3779B97F4A7C15); digest = (sum, xor). */
static uint64_t tb_fmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static uint64_t tb_hash4(int64_t a, int64_t b, int64_t c, int64_t d) {
    const int64_t t[4] = {a, b, c, d};
    uint64_t h = 0x6A09E667F3BCC909ULL;
    for (int k = 0; k < 4; ++k) h = tb_fmix64(h ^ ((uint64_t)t[k] + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ULL));
    return h;
}

int64_t textbook_4clique_digest(const int64_t* e, int64_t m, int nthreads, uint64_t* digest) {
    tb_graph g;
    if (tb_build(e, m, &g) != 0) return -1;
    uint64_t total = 0, dsum = 0, dxor = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        unsigned char* mu = (unsigned char*)calloc((size_t)g.n + 1, 1);
        unsigned char* mw = (unsigned char*)calloc((size_t)g.n + 1, 1);
        int64_t* wl = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g.n + 1));
        uint64_t local = 0, ls = 0, lx = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < g.n; ++u) {
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mu[g.adj[i]] = 1;
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) {
                int64_t v = g.adj[i];
                int64_t nw = 0;
                for (int64_t j = g.off[v]; j < g.off[v + 1]; ++j)
                    if (mu[g.adj[j]]) { wl[nw++] = g.adj[j]; mw[g.adj[j]] = 1; }
                for (int64_t a = 0; a < nw; ++a) {
                    int64_t w = wl[a];
                    for (int64_t j = g.off[w]; j < g.off[w + 1]; ++j) {
                        int64_t x = g.adj[j];
                        if (!mw[x]) continue;
                        const int64_t q[4] = {u, v, w, x};
                        /* all 24 orderings */
                        for (int p0 = 0; p0 < 4; ++p0)
                            for (int p1 = 0; p1 < 4; ++p1) {
                                if (p1 == p0) continue;
                                for (int p2 = 0; p2 < 4; ++p2) {
                                    if (p2 == p0 || p2 == p1) continue;
                                    int p3 = 6 - p0 - p1 - p2;
                                    uint64_t h = tb_hash4(q[p0], q[p1], q[p2], q[p3]);
                                    ls += h; lx ^= h;
                                }
                            }
                        local += 1;
                    }
                }
                for (int64_t a = 0; a < nw; ++a) mw[wl[a]] = 0;
            }
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) mu[g.adj[i]] = 0;
        }
#pragma omp critical
        { total += local; dsum += ls; dxor ^= lx; }
        free(mu); free(mw); free(wl);
    }
    free(g.off); free(g.adj);
    digest[0] = dsum; digest[1] = dxor;
    return (int64_t)total;
}

/* Closed 4-walks (the ordered 4-cycle query under homomorphism semantics):
 * sum over ordered pairs (u, w) of c(u, w)^2, c = number of common neighbours,
 * by wedge counting from every u over the deduplicated, loop-free adjacency. */
int64_t textbook_closed_4walks(const int64_t* e, int64_t m, int nthreads) {
    int64_t n = 0;
    for (int64_t i = 0; i < 2 * m; ++i) {
        if (e[i] < 0) return -1;
        if (e[i] + 1 > n) n = e[i] + 1;
    }
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) if (e[2 * i] != e[2 * i + 1]) off[e[2 * i] + 1]++;
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t* nb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    memcpy(cur, off, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < m; ++i)
        if (e[2 * i] != e[2 * i + 1]) nb[cur[e[2 * i]]++] = e[2 * i + 1];
    for (int64_t v = 0; v < n; ++v) {
        int64_t a = off[v], b = off[v + 1];
        qsort(nb + a, (size_t)(b - a), sizeof(int64_t), cmp_i64);
        int64_t w = 0;
        for (int64_t i = a; i < b; ++i) if (w == 0 || nb[i] != nb[a + w - 1]) nb[a + w++] = nb[i];
        deg[v] = w;
    }
    uint64_t total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        uint64_t* cnt = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
        int64_t* touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        uint64_t local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) {
            int64_t nt = 0;
            for (int64_t i = off[u]; i < off[u] + deg[u]; ++i) {
                int64_t v = nb[i];
                for (int64_t j = off[v]; j < off[v] + deg[v]; ++j) {
                    int64_t w = nb[j];
                    if (cnt[w]++ == 0) touched[nt++] = w;
                }
            }
            for (int64_t t = 0; t < nt; ++t) {
                local += cnt[touched[t]] * cnt[touched[t]];
                cnt[touched[t]] = 0;
            }
        }
#pragma omp atomic
        total += local;
        free(cnt); free(touched);
    }
    free(off); free(nb); free(cur); free(deg);
    return (int64_t)total;
}

/* Closed forms of two homomorphism counts over a symmetric loop-free relation E
 * (ordered tuples, no inequalities between variables):
 *   diamond  R(a,b) R(a,c) R(b,d) R(c,d) R(b,c): for every ordered edge (b,c), a and
 *            d range independently over the common neighbours of b and c, so the
 *            count is sum over unordered edges e of 2 t(e)^2, t(e) = triangles on e;
 *   two triangles sharing a vertex c, R(a,b) R(a,c) R(b,c) R(c,d) R(c,e) R(d,e):
 *            every side is an ordered pair of adjacent neighbours of c, 2 t(c) of
 *            them, t(c) = triangles on c, so the count is sum over c of (2 t(c))^2.
 * t(e) and t(v) come from the forward enumeration, each triangle credited to its
 * three edges and vertices.  out[0] = diamond, out[1] = two-triangle; returns 0
 * (-1 on a negative id). */
int64_t textbook_triangle_stats(const int64_t* e, int64_t m, int nthreads, uint64_t* out) {
    tb_graph g;
    if (tb_build(e, m, &g) != 0) return -1;
    const int64_t ne = g.off[g.n];
    uint64_t* te = (uint64_t*)calloc((size_t)ne + 1, sizeof(uint64_t));
    uint64_t* tv = (uint64_t*)calloc((size_t)g.n + 1, sizeof(uint64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int64_t* slot = (int64_t*)calloc((size_t)g.n + 1, sizeof(int64_t));   /* edge index + 1 of (u, w) */
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < g.n; ++u) {
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) slot[g.adj[i]] = i + 1;
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) {
                const int64_t v = g.adj[i];
                for (int64_t j = g.off[v]; j < g.off[v + 1]; ++j) {
                    const int64_t w = g.adj[j];
                    if (slot[w] == 0) continue;
                    /* triangle u, v, w: edges (u,v) = i, (v,w) = j, (u,w) = slot[w] - 1 */
#pragma omp atomic
                    te[i]++;
#pragma omp atomic
                    te[j]++;
#pragma omp atomic
                    te[slot[w] - 1]++;
#pragma omp atomic
                    tv[u]++;
#pragma omp atomic
                    tv[v]++;
#pragma omp atomic
                    tv[w]++;
                }
            }
            for (int64_t i = g.off[u]; i < g.off[u + 1]; ++i) slot[g.adj[i]] = 0;
        }
        free(slot);
    }
    uint64_t dia = 0, two = 0;
    for (int64_t i = 0; i < ne; ++i) dia += 2 * te[i] * te[i];
    for (int64_t v = 0; v < g.n; ++v) two += 4 * tv[v] * tv[v];
    out[0] = dia;
    out[1] = two;
    free(te); free(tv); free(g.off); free(g.adj);
    return 0;
}
