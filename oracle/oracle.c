/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the graph
 * primitives of the frontier engine.  TEST INFRASTRUCTURE ONLY: it is used by
 * the test-suite, by the smoke check and by the benchmark's CPU-baseline leg,
 * never by the product path.  It shares no code with the GPU engine.
 *
 * Graphs are symmetric simple CSR (row offsets R[n+1], column ids C[m], optional
 * uint32 weights W[m]), the form the paper evaluates on (Sec. 3 for CSR, Sec. 6
 * for the undirected conversion).  Everything is single threaded.
 *
 * Output conventions (fixed here because the paper leaves them open):
 *   BFS   depth int32, source 0, unreached -1.
 *   SSSP  dist uint32, source 0, unreached 0xFFFFFFFF; sums formed in uint64.
 *   pred  source -> itself, unreached -1, else the first neighbour one step closer.
 *   BC    unnormalised sum over ordered pairs (s in S, t in V), no halving.
 *   CC    label = smallest vertex id of the component.
 *   PR    uniform teleport (1-d)/N, dangling mass spread uniformly, L1 stop.
 *   2-hop uint64 walk counts per end vertex.
 *   PPR   teleport and dangling mass uniform over the seeds, x_0 on the seeds.
 *   SALSA / HITS  hubs = [0, nl), authorities = [nl, n), every edge across.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* -------------------------------------------------------------- BFS ---- */
/*
 * Hop distance from the source (Sec. 5.1: each iteration reaches the
 * unvisited neighbours of the current frontier and sets their depth).
 * Written as the textbook FIFO-queue BFS.
 * Returns the number of vertices reached, -1 on bad input / OOM.
 */
OR_EXPORT int64_t or_bfs(int32_t n, const int32_t *R, const int32_t *C, int32_t src, int32_t *depth)
{
    if (n <= 0 || src < 0 || src >= n) return -1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -1;
    for (int32_t v = 0; v < n; ++v) depth[v] = -1;
    int64_t head = 0, tail = 0;
    depth[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = R[u]; e < R[u + 1]; ++e) {
            int32_t v = C[e];
            if (depth[v] < 0) {
                depth[v] = depth[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return tail;
}

/* ------------------------------------------------------------- SSSP ---- */
/*
 * Shortest-path distances with non-negative weights (Sec. 4.1 assumes
 * non-negative weights, which permits Dijkstra).  Binary min-heap keyed on the
 * tentative distance with lazy deletion; sums in uint64.
 * Returns the number of vertices reached; -2 if a distance does not fit below
 * 0xFFFFFFFF; -1 on bad input / OOM.
 */
typedef struct { uint64_t d; int32_t v; } or_item;

static void heap_push(or_item *h, int64_t *len, or_item x)
{
    int64_t i = (*len)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= x.d) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = x;
}

static or_item heap_pop(or_item *h, int64_t *len)
{
    or_item top = h[0];
    or_item x = h[--(*len)];
    int64_t i = 0, L = *len;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        uint64_t ds = x.d;
        if (l < L && h[l].d < ds) { s = l; ds = h[l].d; }
        if (r < L && h[r].d < ds) { s = r; }
        if (s == i) break;
        h[i] = h[s];
        i = s;
    }
    if (L > 0) h[i] = x;
    return top;
}

OR_EXPORT int64_t or_sssp(int32_t n, const int32_t *R, const int32_t *C, const uint32_t *W,
                          int32_t src, uint32_t *dist)
{
    if (n <= 0 || src < 0 || src >= n || !W) return -1;
    uint64_t *d = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
    int64_t cap = (int64_t)R[n] + 1;
    or_item *heap = (or_item *)malloc((size_t)cap * sizeof(or_item));
    if (!d || !done || !heap) { free(d); free(done); free(heap); return -1; }
    const uint64_t INF = UINT64_MAX;
    for (int32_t v = 0; v < n; ++v) d[v] = INF;
    int64_t len = 0, reached = 0;
    d[src] = 0;
    heap_push(heap, &len, (or_item){0, src});
    while (len > 0) {
        or_item it = heap_pop(heap, &len);
        int32_t u = it.v;
        if (done[u] || it.d != d[u]) continue;
        done[u] = 1;
        ++reached;
        for (int32_t e = R[u]; e < R[u + 1]; ++e) {
            int32_t v = C[e];
            uint64_t nd = d[u] + (uint64_t)W[e];
            if (nd < d[v]) {
                d[v] = nd;
                heap_push(heap, &len, (or_item){nd, v});
            }
        }
    }
    int64_t rc = reached;
    for (int32_t v = 0; v < n; ++v) {
        if (d[v] == INF) dist[v] = 0xFFFFFFFFu;
        else if (d[v] >= 0xFFFFFFFFull) { dist[v] = 0xFFFFFFFFu; rc = -2; }
        else dist[v] = (uint32_t)d[v];
    }
    free(d); free(done); free(heap);
    return rc;
}

/* ----------------------------------------------------- predecessors ---- */
/*
 * Predecessors read off the distances (a BFS tree, Sec. 5.1, and a
 * shortest-path tree, Sec. 5.2): pred[src] = src, -1 where unreached, and
 * otherwise the first neighbour u in v's list that lies one step closer:
 * depth[u] = depth[v] - 1 for BFS, dist[u] + w(v,u) = dist[v] for SSSP (the
 * smallest such id when rows are sorted).  The distances come from or_bfs /
 * or_sssp and are returned too.  Same return codes as those.
 */
OR_EXPORT int64_t or_bfs_pred(int32_t n, const int32_t *R, const int32_t *C, int32_t src, int32_t *depth,
                              int32_t *pred)
{
    const int64_t rc = or_bfs(n, R, C, src, depth);
    if (rc < 0) return rc;
    for (int32_t v = 0; v < n; ++v) {
        pred[v] = -1;
        if (depth[v] < 0) continue;
        if (v == src) {
            pred[v] = src;
            continue;
        }
        for (int32_t e = R[v]; e < R[v + 1]; ++e) {
            if (depth[C[e]] == depth[v] - 1) {
                pred[v] = C[e];
                break;
            }
        }
    }
    return rc;
}

OR_EXPORT int64_t or_sssp_pred(int32_t n, const int32_t *R, const int32_t *C, const uint32_t *W, int32_t src,
                               uint32_t *dist, int32_t *pred)
{
    const int64_t rc = or_sssp(n, R, C, W, src, dist);
    if (rc < 0) return rc;
    for (int32_t v = 0; v < n; ++v) {
        pred[v] = -1;
        if (dist[v] == 0xFFFFFFFFu) continue;
        if (v == src) {
            pred[v] = src;
            continue;
        }
        for (int32_t e = R[v]; e < R[v + 1]; ++e) {
            const int32_t u = C[e];
            if (dist[u] != 0xFFFFFFFFu && (uint64_t)dist[u] + W[e] == (uint64_t)dist[v]) {
                pred[v] = u;
                break;
            }
        }
    }
    return rc;
}

/* --------------------------------------------------------------- BC ---- */
/*
 * Betweenness centrality restricted to the given sources (Sec. 5.3: a forward
 * BFS that counts shortest paths sigma, then a backward pass over the BFS
 * levels that accumulates dependencies delta; Brandes' formulation).
 *   sigma_s(s) = 1,  sigma_s(v) = sum of sigma_s(u) over predecessors u of v
 *   delta_s(v) = sum over successors w of sigma_s(v)/sigma_s(w) * (1 + delta_s(w))
 *   bc(v)      = sum over s in S, s != v, of delta_s(v)
 * All in FP64.  Sources must be distinct and in range.  Returns 0, or -1.
 */
OR_EXPORT int32_t or_bc(int32_t n, const int32_t *R, const int32_t *C, const int32_t *sources,
                        int32_t k, double *bc)
{
    if (n <= 0 || k < 0) return -1;
    for (int32_t i = 0; i < k; ++i) {
        if (sources[i] < 0 || sources[i] >= n) return -1;
        for (int32_t j = 0; j < i; ++j) if (sources[j] == sources[i]) return -1;
    }
    int32_t *depth = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    double *sigma = (double *)malloc((size_t)n * sizeof(double));
    double *delta = (double *)malloc((size_t)n * sizeof(double));
    if (!depth || !order || !sigma || !delta) {
        free(depth); free(order); free(sigma); free(delta);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;
    for (int32_t si = 0; si < k; ++si) {
        int32_t s = sources[si];
        for (int32_t v = 0; v < n; ++v) { depth[v] = -1; sigma[v] = 0.0; delta[v] = 0.0; }
        int64_t head = 0, tail = 0;
        depth[s] = 0;
        sigma[s] = 1.0;
        order[tail++] = s;
        /* forward: BFS order; every edge into the next level adds sigma */
        while (head < tail) {
            int32_t u = order[head++];
            for (int32_t e = R[u]; e < R[u + 1]; ++e) {
                int32_t v = C[e];
                if (depth[v] < 0) {
                    depth[v] = depth[u] + 1;
                    order[tail++] = v;
                }
                if (depth[v] == depth[u] + 1) sigma[v] += sigma[u];
            }
        }
        /* backward: reverse BFS order */
        for (int64_t i = tail - 1; i >= 0; --i) {
            int32_t w = order[i];
            for (int32_t e = R[w]; e < R[w + 1]; ++e) {
                int32_t v = C[e];
                if (depth[v] == depth[w] - 1)
                    delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
            }
            if (w != s) bc[w] += delta[w];
        }
    }
    free(depth); free(order); free(sigma); free(delta);
    return 0;
}

/* --------------------------------------------------------------- CC ---- */
/*
 * Connected-component labels (Sec. 5.4 asks for a unique id per component;
 * the id used here is the smallest vertex id in the component).
 * Disjoint-set forest: union makes the larger root point to the smaller one,
 * find uses path halving; so every root is its set's minimum.
 * Returns the number of components, or -1.
 */
static int32_t uf_find(int32_t *p, int32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

OR_EXPORT int32_t or_cc(int32_t n, const int32_t *R, const int32_t *C, int32_t *label)
{
    if (n <= 0) return -1;
    for (int32_t v = 0; v < n; ++v) label[v] = v;
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = R[u]; e < R[u + 1]; ++e) {
            int32_t a = uf_find(label, u), b = uf_find(label, C[e]);
            if (a < b) label[b] = a;
            else if (b < a) label[a] = b;
        }
    }
    int32_t ncomp = 0;
    for (int32_t v = 0; v < n; ++v) {
        label[v] = uf_find(label, v);
        if (label[v] == v) ++ncomp;
    }
    return ncomp;
}

/* --------------------------------------------------------- PageRank ---- */
/* PageRank pieces shared by both PageRank functions (Sec. 5.5): the rank
 * mass on vertices without edges, a vertex's sum of neighbour contributions
 * x(u)/deg(u), and the damped update with uniform teleport and dangling
 * redistribution. */
static double pr_dangling_mass(int32_t n, const int32_t *R, const double *x)
{
    double dangling = 0.0;
    for (int32_t u = 0; u < n; ++u)
        if (R[u + 1] == R[u]) dangling += x[u];
    return dangling;
}

static double pr_neighbour_sum(const int32_t *R, const int32_t *C, const double *x, int32_t v)
{
    double s = 0.0;
    for (int32_t e = R[v]; e < R[v + 1]; ++e) {
        int32_t u = C[e];
        s += x[u] / (double)(R[u + 1] - R[u]);
    }
    return s;
}

static double pr_update(double damping, double N, double s, double dangling)
{
    return (1.0 - damping) / N + damping * (s + dangling / N);
}

/*
 * Power iteration (Sec. 5.5: start every vertex with a value and update from
 * neighbours until convergence), in FP64:
 *   x_0(v)     = 1/N
 *   x_{k+1}(v) = (1-d)/N + d * ( sum_{u in N(v)} x_k(u)/deg(u)  +  D_k/N )
 *   D_k        = sum of x_k(u) over vertices with deg(u) = 0
 * Stops after the first k with ||x_{k+1} - x_k||_1 < tol, or after max_iter
 * iterations; x holds the last iterate.  tol <= 0 runs exactly max_iter
 * iterations.  Writes the iteration count and the last L1 change.
 */
OR_EXPORT int32_t or_pagerank(int32_t n, const int32_t *R, const int32_t *C, double damping,
                              double tol, int32_t max_iter, double *x, int32_t *iters,
                              double *last_l1)
{
    if (n <= 0 || max_iter < 0 || !(damping > 0.0 && damping < 1.0)) return -1;
    double *y = (double *)malloc((size_t)n * sizeof(double));
    if (!y) return -1;
    const double N = (double)n;
    for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / N;
    int32_t k = 0;
    double l1 = 0.0;
    while (k < max_iter) {
        const double dangling = pr_dangling_mass(n, R, x);
        for (int32_t v = 0; v < n; ++v) y[v] = pr_update(damping, N, pr_neighbour_sum(R, C, x, v), dangling);
        l1 = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            l1 += fabs(y[v] - x[v]);
            x[v] = y[v];
        }
        ++k;
        if (tol > 0.0 && l1 < tol) break;
    }
    free(y);
    if (iters) *iters = k;
    if (last_l1) *last_l1 = l1;
    return 0;
}

/*
 * PageRank with per-vertex convergence filtering (Sec. 5.5): the frontier
 * starts with every vertex; each iteration recomputes the rank of the
 * frontier's vertices from the current ranks of all vertices (those outside
 * the frontier keep their last value), then the filter keeps in the frontier
 * only the vertices whose rank changed by at least `vertex_tol`.  Stops when
 * the frontier is empty or after max_iter iterations.  An approximation: a
 * vertex leaves the frontier with a residual change below vertex_tol.
 * `active` (n bytes, may be NULL) receives the final frontier membership;
 * `last_l1` the summed change of the last iteration.
 */
OR_EXPORT int32_t or_pagerank_filtered(int32_t n, const int32_t *R, const int32_t *C, double damping,
                                       double vertex_tol, int32_t max_iter, double *x, int32_t *iters,
                                       double *last_l1, uint8_t *active_out)
{
    if (n <= 0 || max_iter < 0 || vertex_tol < 0.0 || !(damping > 0.0 && damping < 1.0)) return -1;
    double *y = (double *)malloc((size_t)n * sizeof(double));
    uint8_t *active = (uint8_t *)malloc((size_t)n);
    if (!y || !active) {
        free(y);
        free(active);
        return -1;
    }
    const double N = (double)n;
    int32_t in_frontier = n;
    for (int32_t v = 0; v < n; ++v) {
        x[v] = 1.0 / N;
        active[v] = 1;
    }
    int32_t k = 0;
    double l1 = 0.0;
    while (k < max_iter && in_frontier > 0) {
        /* advance: new ranks of the frontier, from the ranks of this iterate */
        const double dangling = pr_dangling_mass(n, R, x);
        for (int32_t v = 0; v < n; ++v)
            if (active[v]) y[v] = pr_update(damping, N, pr_neighbour_sum(R, C, x, v), dangling);
        /* filter: drop the vertices that moved less than vertex_tol */
        l1 = 0.0;
        in_frontier = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (!active[v]) continue;
            double dx = fabs(y[v] - x[v]);
            l1 += dx;
            x[v] = y[v];
            if (dx >= vertex_tol) ++in_frontier;
            else active[v] = 0;
        }
        ++k;
    }
    if (active_out) memcpy(active_out, active, (size_t)n);
    free(y);
    free(active);
    if (iters) *iters = k;
    if (last_l1) *last_l1 = l1;
    return 0;
}

/* ------------------------------------------------- 2-hop and ranking ---- */
static int32_t distinct_in_range(int32_t n, const int32_t *v, int32_t k)
{
    if (k < 1) return 0;
    for (int32_t i = 0; i < k; ++i) {
        if (v[i] < 0 || v[i] >= n) return 0;
        for (int32_t j = 0; j < i; ++j) if (v[j] == v[i]) return 0;
    }
    return 1;
}

/*
 * Walks of length two from a vertex set (Sec. 4.1, the fourth use of advance:
 * from the seeds' edges to their neighbouring edges, returning the far-end
 * vertices): count[v] = number of walks s - u - v with s a seed, u a
 * neighbour of s and v a neighbour of u.  Seeds distinct and in range.
 */
OR_EXPORT int32_t or_two_hop(int32_t n, const int32_t *R, const int32_t *C, const int32_t *seeds, int32_t k,
                             uint64_t *count)
{
    if (n <= 0 || !distinct_in_range(n, seeds, k)) return -1;
    for (int32_t v = 0; v < n; ++v) count[v] = 0;
    for (int32_t i = 0; i < k; ++i) {
        const int32_t s = seeds[i];
        for (int32_t e = R[s]; e < R[s + 1]; ++e) {
            const int32_t u = C[e];
            for (int32_t f = R[u]; f < R[u + 1]; ++f) count[C[f]] += 1;
        }
    }
    return 0;
}

/*
 * Personalized PageRank (one of the bipartite node rankings built on
 * advance, Sec. 5.5's list of further uses): the teleport vector p is uniform
 * over the seeds and also receives the rank of zero-degree vertices,
 *   x_0     = p
 *   x_{k+1}(v) = (1-d) p(v) + d * ( sum_{u in N(v)} x_k(u)/deg(u) + D_k p(v) )
 * with D_k the rank on zero-degree vertices.  Stops like or_pagerank: after
 * the first iteration whose L1 change is below tol, or after max_iter.
 */
OR_EXPORT int32_t or_ppr(int32_t n, const int32_t *R, const int32_t *C, const int32_t *seeds, int32_t k,
                         double damping, double tol, int32_t max_iter, double *x, int32_t *iters,
                         double *last_l1)
{
    if (n <= 0 || max_iter < 0 || !(damping > 0.0 && damping < 1.0) || !distinct_in_range(n, seeds, k))
        return -1;
    double *p = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    if (!p || !y) {
        free(p);
        free(y);
        return -1;
    }
    for (int32_t i = 0; i < k; ++i) p[seeds[i]] = 1.0 / (double)k;
    for (int32_t v = 0; v < n; ++v) x[v] = p[v];
    int32_t it = 0;
    double l1 = 0.0;
    while (it < max_iter) {
        const double dangling = pr_dangling_mass(n, R, x);
        for (int32_t v = 0; v < n; ++v)
            y[v] = (1.0 - damping) * p[v] + damping * (pr_neighbour_sum(R, C, x, v) + dangling * p[v]);
        l1 = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            l1 += fabs(y[v] - x[v]);
            x[v] = y[v];
        }
        ++it;
        if (l1 < tol && tol > 0.0) break;
    }
    free(p);
    free(y);
    if (iters) *iters = it;
    if (last_l1) *last_l1 = l1;
    return 0;
}

/* every edge must join the two sides [0, nl) and [nl, n) */
static int32_t is_bipartite_split(int32_t n, const int32_t *R, const int32_t *C, int32_t nl)
{
    if (nl < 1 || nl >= n) return 0;
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = R[v]; e < R[v + 1]; ++e)
            if ((v < nl) == (C[e] < nl)) return 0;
    return 1;
}

/*
 * SALSA on a bipartite graph (hubs on the left [0, nl), authorities on the
 * right [nl, n)): random-walk scores, starting from h_0 = 1/nl on every hub;
 * each iteration
 *   a(r) = sum_{l in N(r)} h(l) / deg(l)     then
 *   h(l) = sum_{r in N(l)} a(r) / deg(r)     (with the new a).
 * hub[nl] and auth[n - nl] receive the scores after `iters` iterations.
 */
OR_EXPORT int32_t or_salsa(int32_t n, const int32_t *R, const int32_t *C, int32_t nl, int32_t iters,
                           double *hub, double *auth)
{
    if (n <= 1 || iters < 0 || !is_bipartite_split(n, R, C, nl)) return -1;
    const int32_t nr = n - nl;
    for (int32_t l = 0; l < nl; ++l) hub[l] = 1.0 / (double)nl;
    for (int32_t r = 0; r < nr; ++r) auth[r] = 0.0;
    for (int32_t it = 0; it < iters; ++it) {
        for (int32_t r = 0; r < nr; ++r) {
            const int32_t v = nl + r;
            double s = 0.0;
            for (int32_t e = R[v]; e < R[v + 1]; ++e) {
                const int32_t l = C[e];
                s += hub[l] / (double)(R[l + 1] - R[l]);
            }
            auth[r] = s;
        }
        for (int32_t l = 0; l < nl; ++l) {
            double s = 0.0;
            for (int32_t e = R[l]; e < R[l + 1]; ++e) {
                const int32_t v = C[e];
                s += auth[v - nl] / (double)(R[v + 1] - R[v]);
            }
            hub[l] = s;
        }
    }
    return 0;
}

static void scale_to_unit_l2(double *a, int32_t len)
{
    double ss = 0.0;
    for (int32_t i = 0; i < len; ++i) ss += a[i] * a[i];
    if (ss > 0.0) {
        const double inv = 1.0 / sqrt(ss);
        for (int32_t i = 0; i < len; ++i) a[i] *= inv;
    }
}

/*
 * HITS on a bipartite graph (hubs left, authorities right): h_0 = 1/sqrt(nl);
 * each iteration a = B^T h, scaled to unit L2 norm, then h = B a, scaled to
 * unit L2 norm (a zero vector stays zero), B the biadjacency matrix.
 */
OR_EXPORT int32_t or_hits(int32_t n, const int32_t *R, const int32_t *C, int32_t nl, int32_t iters, double *hub,
                          double *auth)
{
    if (n <= 1 || iters < 0 || !is_bipartite_split(n, R, C, nl)) return -1;
    const int32_t nr = n - nl;
    for (int32_t l = 0; l < nl; ++l) hub[l] = 1.0 / sqrt((double)nl);
    for (int32_t r = 0; r < nr; ++r) auth[r] = 0.0;
    for (int32_t it = 0; it < iters; ++it) {
        for (int32_t r = 0; r < nr; ++r) {
            const int32_t v = nl + r;
            double s = 0.0;
            for (int32_t e = R[v]; e < R[v + 1]; ++e) s += hub[C[e]];
            auth[r] = s;
        }
        scale_to_unit_l2(auth, nr);
        for (int32_t l = 0; l < nl; ++l) {
            double s = 0.0;
            for (int32_t e = R[l]; e < R[l + 1]; ++e) s += auth[C[e] - nl];
            hub[l] = s;
        }
        scale_to_unit_l2(hub, nl);
    }
    return 0;
}
