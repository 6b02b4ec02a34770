/*
 * graphgen.c -- seeded synthetic input generators (R-MAT, perturbed grid
 * lattice, symmetric edge weights, source sampling).
 *
 * This module produces INPUTS only.  It is shared by the CPU oracle and the
 * GPU engine so that both see byte-identical graphs; it contains none of the
 * traversal/ranking arithmetic that either side computes.
 *
 * Every random draw comes from a counter-based generator: a splitmix64
 * finaliser applied to (seed, counter, sub-counter).  Outputs therefore do not
 * depend on thread count or evaluation order.
 *
 * Graph conventions (the paper converts every dataset to an undirected graph,
 * Sec. 6, and evaluates on simple CSR graphs, Sec. 3):
 *   - symmetric: (u,v) present  <=>  (v,u) present
 *   - no self loops, no duplicate edges
 *   - CSR rows sorted by column id
 *   - int32 row offsets (m < 2^31) and int32 column ids
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_EXPORT __attribute__((visibility("default")))

/* ---------------------------------------------------------------- RNG ---- */
static inline uint64_t gg_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* hash of (seed, a, b): three chained finaliser rounds */
static inline uint64_t gg_hash3(uint64_t seed, uint64_t a, uint64_t b)
{
    return gg_mix(gg_mix(gg_mix(seed) ^ a) ^ b);
}

/* uniform double in [0,1) with 53 random bits */
static inline double gg_unit(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

GG_EXPORT uint64_t gg_hash(uint64_t seed, uint64_t a, uint64_t b) { return gg_hash3(seed, a, b); }

/* --------------------------------------------------------- CSR builder ---- */
typedef struct gg_graph {
    int32_t n;
    int64_t m;
    int32_t *row;   /* n+1 */
    int32_t *col;   /* m   */
} gg_graph;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* LSD radix sort of a small int32 array of non-negative keys (used for the
 * long rows of hub vertices; qsort is used for short rows). */
static void sort_row(int32_t *a, int64_t len, int32_t *tmp)
{
    if (len < 64) {
        /* insertion sort */
        for (int64_t i = 1; i < len; ++i) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
        return;
    }
    if (!tmp) { qsort(a, (size_t)len, sizeof(int32_t), cmp_i32); return; }
    int64_t cnt[256];
    int32_t *src = a, *dst = tmp;
    for (int pass = 0; pass < 4; ++pass) {
        int sh = pass * 8;
        memset(cnt, 0, sizeof cnt);
        for (int64_t i = 0; i < len; ++i) cnt[((uint32_t)src[i] >> sh) & 255]++;
        int64_t s = 0;
        for (int k = 0; k < 256; ++k) { int64_t c = cnt[k]; cnt[k] = s; s += c; }
        for (int64_t i = 0; i < len; ++i) dst[cnt[((uint32_t)src[i] >> sh) & 255]++] = src[i];
        int32_t *t = src; src = dst; dst = t;
    }
    /* after 4 passes the data is back in a */
}

/*
 * Build a symmetric simple CSR from an undirected edge list (eu[i], ev[i]).
 * Self loops are dropped, both directions are inserted, rows sorted, duplicates
 * removed.  Takes ownership of nothing; returns a heap graph or NULL on OOM.
 */
static gg_graph *build_csr(int32_t n, int64_t ne, const int32_t *eu, const int32_t *ev)
{
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) return NULL;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        int32_t u = eu[i], v = ev[i];
        if (u == v) continue;
        __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
    }
    int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!off) { free(deg); return NULL; }
    off[0] = 0;
    for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
    int64_t total = off[n];
    int32_t *tmpcol = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    if (!tmpcol) { free(deg); free(off); return NULL; }
    /* deg[] becomes the insertion cursor */
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) deg[i] = off[i];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        int32_t u = eu[i], v = ev[i];
        if (u == v) continue;
        int64_t pu = __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
        tmpcol[pu] = v;
        int64_t pv = __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
        tmpcol[pv] = u;
    }
    /* sort + dedup each row in place; deg[i] := unique count */
    int32_t maxlen = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t l = off[i + 1] - off[i];
        if (l > maxlen) maxlen = (int32_t)l;
    }
    #pragma omp parallel
    {
        int32_t *tmp = (int32_t *)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof(int32_t));
        #pragma omp for schedule(dynamic, 1024)
        for (int32_t i = 0; i < n; ++i) {
            int32_t *a = tmpcol + off[i];
            int64_t len = off[i + 1] - off[i];
            sort_row(a, len, tmp);
            int64_t k = 0;
            for (int64_t j = 0; j < len; ++j)
                if (k == 0 || a[j] != a[k - 1]) a[k++] = a[j];
            deg[i] = k;
        }
        free(tmp);
    }
    gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
    int64_t m = 0;
    for (int32_t i = 0; i < n; ++i) m += deg[i];
    g->n = n;
    g->m = m;
    g->row = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!g->row || !g->col || m > INT32_MAX) {
        free(g->row); free(g->col); free(g); free(deg); free(off); free(tmpcol);
        return NULL;
    }
    g->row[0] = 0;
    for (int32_t i = 0; i < n; ++i) g->row[i + 1] = (int32_t)(g->row[i] + deg[i]);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i)
        memcpy(g->col + g->row[i], tmpcol + off[i], (size_t)deg[i] * sizeof(int32_t));
    free(deg); free(off); free(tmpcol);
    return g;
}

/* ------------------------------------------------------------ R-MAT ---- */
/*
 * R-MAT: edge i (0 <= i < ef * 2^scale) descends `scale` levels of the
 * adjacency quadtree.  At level l it draws r = U(seed, i, l) and picks the
 * quadrant (0,0) with prob a, (0,1) with prob b, (1,0) with prob c, (1,1)
 * otherwise, setting bit (scale-1-l) of u and/or v.  No noise, no vertex
 * permutation: vertex 0 is the densest corner.
 */
/* endpoints of R-MAT edge i: one quadrant draw per level, counter (i, level) */
static void rmat_edge(int32_t scale, double a, double b, double c, uint64_t s0, int64_t i, int32_t *pu,
                      int32_t *pv)
{
    const double ab = a + b, abc = a + b + c;
    uint64_t hi = gg_mix(s0 ^ (uint64_t)i);
    int32_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; ++l) {
        double r = gg_unit(gg_mix(hi ^ ((uint64_t)(l + 1) * 0xD1B54A32D192ED03ull)));
        int32_t bit = (int32_t)1 << (scale - 1 - l);
        if (r < a) {
        } else if (r < ab) {
            v |= bit;
        } else if (r < abc) {
            u |= bit;
        } else {
            u |= bit;
            v |= bit;
        }
    }
    *pu = u;
    *pv = v;
}

GG_EXPORT gg_graph *gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
                            uint64_t seed)
{
    if (scale < 1 || scale > 30 || edge_factor < 1) return NULL;
    int32_t n = (int32_t)1 << scale;
    int64_t ne = (int64_t)edge_factor << scale;
    int32_t *eu = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    int32_t *ev = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return NULL; }
    const uint64_t s0 = gg_mix(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) rmat_edge(scale, a, b, c, s0, i, eu + i, ev + i);
    gg_graph *g = build_csr(n, ne, eu, ev);
    free(eu);
    free(ev);
    return g;
}

/*
 * Bipartite R-MAT: 2^scale vertices on each side; R-MAT edge (u, v) joins
 * left vertex u to right vertex 2^scale + v (a "who follows whom" graph:
 * users on the left, the accounts they follow on the right).  Symmetric
 * simple CSR over n = 2^(scale+1) vertices; duplicates removed.
 */
GG_EXPORT gg_graph *gg_bipartite_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
                                      uint64_t seed)
{
    if (scale < 1 || scale > 29 || edge_factor < 1) return NULL;
    const int32_t half = (int32_t)1 << scale;
    const int64_t ne = (int64_t)edge_factor << scale;
    int32_t *eu = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    int32_t *ev = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return NULL; }
    const uint64_t s0 = gg_mix(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        rmat_edge(scale, a, b, c, s0, i, eu + i, ev + i);
        ev[i] += half;
    }
    gg_graph *g = build_csr(2 * half, ne, eu, ev);
    free(eu);
    free(ev);
    return g;
}

/* ------------------------------------------------------------- grid ---- */
/*
 * side x side 2D lattice, vertex id = r*side + c.  Each of the 2*side*(side-1)
 * lattice edges is kept with probability 1 - p_drop (draw U(seed, edge, 0)).
 * Then n_long extra edges with endpoints uniform over all vertices (u != v;
 * draw k of long edge j uses counters (j, 2k+1) and (j, 2k+2)).
 */
GG_EXPORT gg_graph *gg_grid(int32_t side, double p_drop, int64_t n_long, uint64_t seed)
{
    if (side < 2 || side > 46340) return NULL;
    int32_t n = side * side;
    int64_t nlat = 2LL * side * (side - 1);
    int64_t cap = nlat + (n_long > 0 ? n_long : 0);
    int32_t *eu = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    int32_t *ev = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return NULL; }
    const uint64_t s0 = gg_mix(seed);
    /* lattice edge id k: k < side*(side-1) -> horizontal, else vertical */
    const int64_t nh = (int64_t)side * (side - 1);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nlat; ++k) {
        int32_t u, v;
        if (k < nh) {
            int32_t r = (int32_t)(k / (side - 1)), cc = (int32_t)(k % (side - 1));
            u = r * side + cc;
            v = u + 1;
        } else {
            int64_t kk = k - nh;
            int32_t r = (int32_t)(kk / side), cc = (int32_t)(kk % side);
            u = r * side + cc;
            v = u + side;
        }
        double rd = gg_unit(gg_mix(gg_mix(s0 ^ (uint64_t)k)));
        if (rd < p_drop) { u = v = 0; } /* dropped: encoded as a self loop */
        eu[k] = u;
        ev[k] = v;
    }
    const uint64_t s1 = gg_mix(seed ^ 0xA5A5A5A5A5A5A5A5ull);
    for (int64_t j = 0; j < n_long; ++j) {
        int32_t u = 0, v = 0;
        for (uint64_t t = 0;; ++t) {
            u = (int32_t)(gg_hash3(s1, (uint64_t)j, 2 * t + 1) % (uint64_t)n);
            v = (int32_t)(gg_hash3(s1, (uint64_t)j, 2 * t + 2) % (uint64_t)n);
            if (u != v) break;
        }
        eu[nlat + j] = u;
        ev[nlat + j] = v;
    }
    gg_graph *g = build_csr(n, cap, eu, ev);
    free(eu);
    free(ev);
    return g;
}

/* Build a graph from a caller edge list (tests: paths, stars, random graphs). */
GG_EXPORT gg_graph *gg_from_edges(int32_t n, int64_t ne, const int32_t *eu, const int32_t *ev)
{
    if (n < 1) return NULL;
    for (int64_t i = 0; i < ne; ++i)
        if (eu[i] < 0 || eu[i] >= n || ev[i] < 0 || ev[i] >= n) return NULL;
    return build_csr(n, ne, eu, ev);
}

GG_EXPORT int32_t gg_graph_n(const gg_graph *g) { return g->n; }
GG_EXPORT int64_t gg_graph_m(const gg_graph *g) { return g->m; }
GG_EXPORT void gg_graph_copy(const gg_graph *g, int32_t *row, int32_t *col)
{
    memcpy(row, g->row, ((size_t)g->n + 1) * sizeof(int32_t));
    memcpy(col, g->col, (size_t)g->m * sizeof(int32_t));
}
GG_EXPORT void gg_graph_free(gg_graph *g)
{
    if (!g) return;
    free(g->row);
    free(g->col);
    free(g);
}

/* ---------------------------------------------------------- weights ---- */
/*
 * Symmetric integer weights: w(u,v) = 1 + H(seed, min(u,v), max(u,v)) mod maxw,
 * so both directions of an undirected edge carry the same weight and the
 * weight depends only on the unordered pair.
 */
GG_EXPORT void gg_weights(int32_t n, const int32_t *row, const int32_t *col, uint32_t maxw,
                          uint64_t seed, uint32_t *w)
{
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = row[u]; e < row[u + 1]; ++e) {
            int32_t v = col[e];
            uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
            w[e] = 1u + (uint32_t)(gg_hash3(seed, lo, hi) % (uint64_t)maxw);
        }
    }
}

/* -------------------------------------------------- source sampling ---- */
/*
 * Input selection only: mark the vertices of the largest connected component
 * (ties -> the one holding the smallest vertex id) with an explicit-stack
 * flood fill, then draw k distinct sources uniformly from it by rejection
 * with counter-based draws H(seed, j, 0) mod n.  Returns the component size,
 * or -1 on allocation failure / if fewer than k vertices are eligible.
 */
GG_EXPORT int64_t gg_sample_sources(int32_t n, const int32_t *row, const int32_t *col, int32_t k,
                                    uint64_t seed, int32_t *out)
{
    int32_t *comp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *stack = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!comp || !stack) { free(comp); free(stack); return -1; }
    for (int32_t i = 0; i < n; ++i) comp[i] = -1;
    int32_t best = -1;
    int64_t best_size = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        int64_t size = 0, sp = 0;
        stack[sp++] = s;
        comp[s] = s;
        while (sp > 0) {
            int32_t u = stack[--sp];
            ++size;
            for (int32_t e = row[u]; e < row[u + 1]; ++e) {
                int32_t v = col[e];
                if (comp[v] < 0) { comp[v] = s; stack[sp++] = v; }
            }
        }
        if (size > best_size) { best_size = size; best = s; }
    }
    free(stack);
    if (best_size < k) { free(comp); return -1; }
    int32_t got = 0;
    for (uint64_t j = 0; got < k; ++j) {
        int32_t v = (int32_t)(gg_hash3(seed, j, 0) % (uint64_t)n);
        if (comp[v] != best) continue;
        int dup = 0;
        for (int32_t t = 0; t < got; ++t) if (out[t] == v) { dup = 1; break; }
        if (!dup) out[got++] = v;
    }
    free(comp);
    return best_size;
}
