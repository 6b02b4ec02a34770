/*
 * gfr.h -- C ABI of the MI355X frontier graph engine.
 *
 * The engine implements the data-centric frontier model of Gunrock
 * (Wang et al., "Gunrock: A High-Performance Graph Processing Library on the
 * GPU", PPoPP'16): an *advance* operator that expands every frontier vertex's
 * CSR neighbour list under load balancing (Sec. 4.1, Sec. 4.4) and a *filter*
 * operator that culls and deduplicates the result (Sec. 4.1, Sec. 4.5), driving
 * BFS, SSSP, BC, CC and PageRank (Sec. 5), PageRank with per-vertex
 * convergence filtering, 2-hop walk counts and the bipartite rankings of
 * Sec. 5.5 (personalized PageRank, SALSA, HITS).  The two operators are also
 * callable on their own (advance from a vertex or from an edge frontier),
 * with the scan and the near/far split they are built from;
 * batched 64-source BFS / SSSP and a serving runtime
 * sit on top.  All kernels are HIP for gfx950.
 *
 * General conventions
 *   - Every call returns a gfr_status; nothing throws across the ABI.
 *   - A failed call leaves its output buffers unspecified unless stated
 *     otherwise and records a message readable with gfr_last_error().
 *   - Output buffers are caller-owned and may be host memory or device memory
 *     (for example a torch tensor's data_ptr on the context's device); the
 *     library detects which.  Device outputs avoid the PCIe copy.
 *   - Calls are synchronous: results are complete when the call returns and
 *     the library keeps no reference to caller buffers (except the serving
 *     calls, which lend `out` until the ticket completes).
 *   - `stream` is a hipStream_t of the context's device, or NULL for the
 *     context's own stream, a blocking stream: work queued earlier on the
 *     device's null stream (PyTorch's default stream) completes before the
 *     call's first kernel.  Work is enqueued on it and waited for.
 *   - One context may be used from several host threads; calls on one context
 *     are serialised internally.
 */
#ifndef GFR_H
#define GFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gfr_status;
#define GFR_OK            0
#define GFR_E_INVALID    -1 /* bad argument, bad graph, unusable input           */
#define GFR_E_OOM        -2 /* device or host allocation failed                    */
#define GFR_E_DEVICE     -3 /* HIP error or device-side watchdog                   */
#define GFR_E_NOT_FOUND  -4 /* unknown graph handle or ticket                      */
#define GFR_E_NOT_READY  -5 /* ticket not finished                                 */
#define GFR_E_CAPACITY   -6 /* request larger than the admission budget            */

typedef struct gfr_ctx gfr_ctx;   /* opaque, owned by the library                   */
typedef int64_t gfr_graph;        /* handle of a resident graph; 0 is never valid   */
typedef int64_t gfr_ticket;       /* handle of a served query; 0 is never valid     */
typedef void *gfr_stream;         /* hipStream_t or NULL                            */

/* flags of gfr_graph_load_csr / gfr_validate_csr */
#define GFR_VALIDATE      1u  /* also reject asymmetric graphs, self loops, duplicate or unsorted columns */

/* ---------------------------------------------------------------- context */
/*
 * Create a context on HIP device `device`.  `tuning_json` may be NULL or a
 * JSON object (the tuning file) whose members are either
 *   "<option>": number        a context-wide value (keys as for gfr_set_option), or
 *   "<class>": {"<option>": number, ...}
 *                             values used for graphs of that class, where
 *                             <class> is "scalefree" (largest degree at least
 *                             16 times the mean degree) or "mesh" (all others);
 *                             only solver options (bfs.*, sssp.*, advance.*,
 *                             msbfs.*, batch.*, bc.*, twohop.*) may be given
 *                             per class.
 * Per-class values apply during each call on a graph of that class, except for
 * options later set explicitly with gfr_set_option, which win.  Options change
 * how the result is reached, never the result.  The string is only read
 * during the call.
 * On success *out receives the context.  GFR_E_INVALID if the tuning file is
 * malformed or names an unknown option or an out-of-range value (checked
 * before the device is touched); GFR_E_DEVICE if the device is missing or
 * not gfx950.
 */
gfr_status gfr_ctx_create(int32_t device, const char *tuning_json, gfr_ctx **out);

/* Destroy a context and free every graph and buffer it owns. NULL is a no-op. */
gfr_status gfr_ctx_destroy(gfr_ctx *ctx);

/* Message of the last failed call on this context (valid until the next call). */
const char *gfr_last_error(const gfr_ctx *ctx);

/*
 * Set a numeric option of the context.  Keys:
 *   "bfs.direction"   0 auto (per-level push/pull choice, Sec. 4.5), 1 push only, 2 pull only
 *   "bfs.alpha"       push->pull when frontier edges > unvisited edges / alpha
 *   "bfs.beta"        pull->push when frontier vertices < n / beta
 *   "bfs.dedup"       0 atomic claim (each vertex enqueued once), 1 idempotent (Sec. 4.5)
 *   "bfs.frontier"    0 auto, 1 queue levels (advance + compaction), 2 mark-byte levels:
 *                     the frontier is a byte per vertex, one launch per level, push
 *                     only (auto: mark bytes on mesh-class graphs unless pull is forced)
 *   "sssp.pull_alpha" single-source SSSP direction (the pull advance of Sec. 4.5 applied to
 *                     SSSP): an iteration whose near queue carries more than m / alpha edges
 *                     relaxes by a pull sweep over every list (one pre-checked atomicMin per
 *                     vertex instead of per edge); 0 (default) = always push
 *   "sssp.frontier"   0 auto (= 1), 1 queue iterations (advance + compaction), 2 mark-byte
 *                     iterations: the near and far sets are bytes per vertex, one launch
 *                     per iteration
 *   "sssp.delta"      bucket width of the near/far priority queue (Sec. 4.5);
 *                     0 = "sssp.delta_factor" (default 2) times the mean edge weight
 *   "advance.chunk"   edges per work-group chunk of the load-balanced advance (Sec. 4.4),
 *                     one of 256, 512, 1024, 2048, 4096
 *   "advance.mapping" BFS push work mapping (Sec. 4.4): 1 (default) equal edge chunks
 *                     (load-balanced partitioning); 2 per-vertex groups (lists of a work-group's
 *                     size or more by the whole work-group, of 64 or more by a wave, the rest
 *                     by one thread each); 0 the paper's hybrid: per-vertex groups while the
 *                     frontier has fewer than "advance.twc_threshold" vertices (default 4096)
 *   "msbfs.alpha"     batched BFS: pull when the frontier's edges exceed m / alpha
 *   "batch.delta"     batched SSSP bucket width; 0 = "batch.delta_factor" times the
 *                     mean edge weight, where factor 0 (default) = a single bucket
 *   "batch.pull_alpha" batched SSSP: relax by a pull sweep (one owner-side minimum per
 *                     vertex and query) when the frontier's edges exceed m / alpha;
 *                     0 (default) = always push
 *   "batch.narrow"    batched SSSP distance rows: 0 (default) 32 bits; 1 auto (scale-free graphs
 *                     start at the narrowest width no earlier batch on the graph outgrew); 2 try
 *                     16 bits first; 3 try 8 bits first.  A batch whose distances outgrow its rows
 *                     is solved again with rows twice as wide; results do not change
 *   "batch.blocks_per_cu"  batched SSSP relaxation grid: work-groups per CU (default 64, at
 *                     most 64, and never more than one per 1024 edges of the graph), 0 = as
 *                     many as are resident at once
 *   "batch.pair"      batched SSSP with 32-bit rows: 1 relaxes two edges per distance-row
 *                     load (each half-wave one edge), 0 (default) one edge per load
 *   "batch.pending"   batched SSSP: 1 (default) a queued vertex also relaxes the queries improved
 *                     at it earlier in the same relaxation launch (read from its marks, which
 *                     stay); 0 only its queued queries.  Results do not change
 *   "batch.sparse"    batched SSSP with 32-bit rows and one edge per row load (batch.pair 0):
 *                     a group of 64 queued edges each carrying at most this many queries
 *                     (default 8) is relaxed one lane per edge, loading single distances
 *                     instead of whole 64-query rows; 0 never.  Results do not change
 *   "graph.steps"     1: the level loops of BFS, SSSP and the batched solvers replay their
 *                     speculative batches of level launches from hipGraphs captured once per
 *                     distinct set of launch arguments; 0 (default): plain launches
 *   "bc.direction"    BC forward discovery (Sec. 5.3 with the push/pull choice of
 *                     Sec. 4.5): 0 auto, 1 push only, 2 pull only; results do not change
 *   "bc.alpha", "bc.beta"  the same ratios as bfs.alpha / bfs.beta for BC's levels
 *   "twohop.direction" second advance of gfr_two_hop: 0 auto, 1 push, 2 pull
 *   "twohop.alpha"    auto: pull when the middle vertices' edges exceed m / alpha
 *   "serve.max_batch" largest number of queries the serving runtime runs together (1..64)
 *   "serve.hipgraph"  1 (default): serving sessions replay their rounds of steps from
 *                     hipGraphs captured once per session; 0: plain launches
 *   "batch.min_bfs", "batch.min_sssp"  batches smaller than this run as sequential
 *                     single-source solves (same results, lower cost for few sources)
 *   "profile.kernels" 1: time every launch of the level kernels with HIP events
 *                     (statistics "t.<kernel>.ms" and "t.<kernel>.n"); 2: only the advance
 *                     kernels (bfs_level, sssp_relax, msbfs_level, bsssp_relax and their pull
 *                     and mark-byte forms), two event records per timed launch instead of per
 *                     launch; 0 (default): none
 *   "serve.budget_bytes"  device bytes the serving runtime's batching sessions may hold;
 *                     lowering it releases idle sessions beyond it (busy ones when they
 *                     finish).  The single-source workers' scratch is not counted.
 * GFR_E_INVALID for an unknown key or an out-of-range value.
 */
gfr_status gfr_set_option(gfr_ctx *ctx, const char *key, double value);
gfr_status gfr_get_option(gfr_ctx *ctx, const char *key, double *value);

/*
 * Statistics of the last solve on this context: "levels", "push_levels",
 * "pull_levels", "edges_inspected", "iterations", "relaxations", "kernel_ms"
 * (device time of the whole call), plus those a call documents with it.
 * Serving statistics since the last "serve.reset": "serve.completed",
 * "serve.batches" (session steps: one level or relaxation round of one
 * session), "serve.mean_batch" (queries in flight per step), "serve.joined"
 * (queries admitted into a session while other queries of it were running),
 * "serve.p50_ms", "serve.p99_ms" (submission to completion), "serve.queued";
 * current: "serve.sessions", "serve.session_bytes".
 */
gfr_status gfr_get_stat(gfr_ctx *ctx, const char *key, double *value);

/*
 * Host-only structural check of a CSR graph (no device work).  Checks what
 * gfr_graph_load_csr checks; with GFR_VALIDATE also symmetry, self loops and
 * sorted duplicate-free rows.  Writes a reason into msg (NUL terminated, at
 * most msg_cap bytes) when the graph is rejected.  Returns GFR_OK or
 * GFR_E_INVALID.
 */
gfr_status gfr_validate_csr(int32_t n, int64_t m, const int32_t *row_offsets,
                            const int32_t *col_idx, const uint32_t *weights, uint32_t flags,
                            char *msg, int32_t msg_cap);

/* ------------------------------------------------------------------ graphs */
/*
 * Make a CSR graph resident on the device (Sec. 3: row offsets R[n+1] and
 * column indices C[m]; per-edge weights W[m] for SSSP, Sec. 5.2).  The graph
 * must be undirected, i.e. stored symmetrically, as every graph the paper
 * evaluates is (Sec. 6).  The arrays are host memory and are copied; the
 * caller may free them on return.  `weights` may be NULL (SSSP then fails).
 * Rejected with GFR_E_INVALID: n <= 0, m < 0, m >= 2^31, R[0] != 0,
 * R[n] != m, decreasing offsets, column ids outside [0,n); with GFR_VALIDATE
 * also the symmetric/simple checks of gfr_validate_csr.
 * On success *out receives a handle owned by the context.
 */
gfr_status gfr_graph_load_csr(gfr_ctx *ctx, int32_t n, int64_t m, const int32_t *row_offsets,
                              const int32_t *col_idx, const uint32_t *weights, uint32_t flags,
                              gfr_graph *out);

/* Release a resident graph.  GFR_E_NOT_FOUND for an unknown handle;
 * GFR_E_NOT_READY while served queries on it are queued or running. */
gfr_status gfr_graph_free(gfr_ctx *ctx, gfr_graph g);

/* Vertex count, entry count and device bytes held by the graph (any may be NULL). */
gfr_status gfr_graph_info(gfr_ctx *ctx, gfr_graph g, int32_t *n, int64_t *m,
                          uint64_t *device_bytes);

/* -------------------------------------------------------------- primitives */
/*
 * Breadth-first search (Sec. 5.1): depth_out[v] = hop distance from `source`,
 * depth_out[source] = 0, unreached vertices -1.  n int32 elements.
 * Level-synchronous advance + filter with a per-level push/pull choice; on
 * mesh-class graphs the frontier stays as mark bytes, one launch per level
 * (option "bfs.frontier").  The depths are the same either way.
 * pred_out (n int32, may be NULL): a BFS tree read off the depths --
 * pred[source] = source, unreached -1, otherwise the first neighbour in v's
 * row one level up (the smallest such id when rows are sorted).
 * GFR_E_INVALID if source is outside [0,n).
 */
gfr_status gfr_bfs(gfr_ctx *ctx, gfr_graph g, int32_t source, int32_t *depth_out,
                   int32_t *pred_out, gfr_stream stream);

/*
 * gfr_bfs without any device allocation, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).  It
 * waits on the stream like every call here, so it is not for stream
 * capture.  Same depths as gfr_bfs (same kernels); no
 * predecessors.  depth_out must be device memory on the context's device
 * (n int32), else GFR_E_INVALID.  The traversal's scratch (frontier queue,
 * bitmaps, mark bytes, control words) comes from one fixed array of
 * GFR_NOALLOC_SCRATCH_BYTES per device, reserved when the library's code is
 * loaded on that device and held until the process ends; a graph whose
 * traversal needs more (about 13.25 bytes per vertex plus 4 bytes per
 * advance chunk of entries: about 5 M vertices at 32 entries per vertex)
 * gets GFR_E_CAPACITY, with nothing written.  The array keeps the last call's contents and every
 * call clears what it reads before writing it.  All contexts on one device
 * share the array: calls that overlap in time on one device (two contexts,
 * or two threads with two contexts) race and give wrong results; calls on
 * one context are serialised and safe.
 */
#define GFR_NOALLOC_SCRATCH_BYTES (64ull * 1024ull * 1024ull)
gfr_status gfr_bfs_noalloc(gfr_ctx *ctx, gfr_graph g, int32_t source, int32_t *depth_out,
                           gfr_stream stream);

/*
 * Single-source shortest paths with non-negative integer weights
 * (Sec. 4.1 Algorithm 1, Sec. 5.2): dist_out[v] = minimum path weight,
 * dist_out[source] = 0, unreached 0xFFFFFFFF.  n uint32 elements.
 * Near/far priority-queue split (Sec. 4.5).  pred_out (n int32, may be
 * NULL): pred[source] = source, unreached -1, otherwise the first neighbour u
 * in v's row with dist[u] + w(u,v) = dist[v] (with zero-weight edges the
 * pointers may form cycles among equal distances; with positive weights they
 * form a shortest-path tree).  GFR_E_INVALID if the graph has no weights, the
 * source is out of range, or a distance would not fit below 0xFFFFFFFF.
 */
gfr_status gfr_sssp(gfr_ctx *ctx, gfr_graph g, int32_t source, uint32_t *dist_out,
                    int32_t *pred_out, gfr_stream stream);

/*
 * Betweenness centrality restricted to k sources (Sec. 5.3, Brandes'
 * two-pass formulation): bc_out[v] = sum over s in sources, s != v, of the
 * dependency delta_s(v); unnormalised, summed over ordered pairs, not halved.
 * Shortest-path counts are FP64, dependencies FP32.  `sources` is host
 * memory (k distinct ids in range, else GFR_E_INVALID).  n float elements.
 */
gfr_status gfr_bc(gfr_ctx *ctx, gfr_graph g, const int32_t *sources, int32_t k, float *bc_out,
                  gfr_stream stream);

/*
 * Connected components (Sec. 5.4): label_out[v] = smallest vertex id of v's
 * component (n int32 elements); *num_components_out (host pointer, may be
 * NULL) = number of components.  Hooking over an edge frontier that is
 * filtered each round, then pointer jumping.
 */
gfr_status gfr_cc(gfr_ctx *ctx, gfr_graph g, int32_t *label_out, int32_t *num_components_out,
                  gfr_stream stream);

/*
 * PageRank by power iteration (Sec. 5.5): x_0 = 1/N,
 *   x_{k+1}(v) = (1-d)/N + d * (sum_{u in N(v)} x_k(u)/deg(u) + D_k/N),
 * D_k the rank held by zero-degree vertices.  Stops after the first iteration
 * whose L1 change is below l1_tol, or after max_iter iterations (GFR_OK in
 * both cases; compare *iters_out with max_iter).  Ranks are FP32, global sums
 * FP64.  rank_out: n floats; iters_out / final_l1_out: host pointers, may be
 * NULL.  GFR_E_INVALID if damping is not in (0,1) or max_iter < 1.
 */
gfr_status gfr_pagerank(gfr_ctx *ctx, gfr_graph g, float damping, double l1_tol,
                        int32_t max_iter, float *rank_out, int32_t *iters_out,
                        double *final_l1_out, gfr_stream stream);

/*
 * PageRank with per-vertex convergence filtering (Sec. 5.5, the frontier
 * form): the frontier starts with every vertex; each iteration recomputes
 * the rank of the frontier's vertices by the update above, from the ranks of
 * the previous iterate (vertices outside the frontier keep their last rank),
 * then keeps in the frontier only the vertices whose rank changed by at least
 * vertex_tol.  Stops when the frontier is empty or after max_iter iterations
 * (GFR_OK in both cases).  An approximation of the fixed point whose error
 * grows with vertex_tol; vertex_tol = 0 reproduces plain power iteration.
 * Everything is FP64, including the filter decision.
 *   rank_out      n doubles (device or host memory)
 *   active_out    n bytes, 1 = still in the frontier at the end; may be NULL
 *   iters_out     iterations run; final_l1_out: summed change of the last
 *                 iteration over the vertices it updated (host, may be NULL)
 * GFR_E_INVALID if damping is not in (0,1), vertex_tol < 0 or max_iter < 1.
 * Statistics: iterations, l1, vertex_updates, edges_gathered, final_frontier.
 */
gfr_status gfr_pagerank_filtered(gfr_ctx *ctx, gfr_graph g, double damping, double vertex_tol,
                                 int32_t max_iter, double *rank_out, uint8_t *active_out,
                                 int32_t *iters_out, double *final_l1_out, gfr_stream stream);

/* ------------------------------------------------------------- operators */
/*
 * The advance operator on its own (Sec. 4.1): the edge frontier of a vertex
 * frontier.  For every entry u of `frontier` (nf ids, host or device memory,
 * any order, duplicates allowed), in frontier order, every edge e of u in CSR
 * order: out_src[i] = u, out_edge[i] = e, out_dst[i] = C[e], i counting from 0
 * in that order.  The degrees are scanned into output offsets and the
 * load-balanced advance (Sec. 4.4) writes every edge at its offset.
 * Outputs: device memory, each may be NULL, out_cap elements each.
 * *count_out (host) = number of edges.  GFR_E_CAPACITY (nothing written) if
 * that exceeds out_cap or 2^31 - 1; GFR_E_INVALID for an id outside [0,n) or a
 * host output pointer.
 */
gfr_status gfr_advance(gfr_ctx *ctx, gfr_graph g, const int32_t *frontier, int32_t nf,
                       int32_t *out_src, int32_t *out_edge, int32_t *out_dst, int64_t out_cap,
                       int64_t *count_out, gfr_stream stream);

/*
 * The advance operator from an edge frontier (Sec. 4.1: advance may start
 * from edges as well as from vertices): edge to edge, and edge to vertex.
 * For every entry e of `edges` (ne edge ids in [0,m), host or device memory,
 * any order, duplicates allowed), in input order, every edge f of v = C[e] in
 * CSR order: out_src[i] = e, out_edge[i] = f, out_dst[i] = C[f].  So out_edge
 * is the edge frontier and out_dst the vertex frontier that the edges lead
 * to.  Outputs, capacity, *count_out and errors as for gfr_advance
 * (GFR_E_INVALID for an id outside [0,m), which every id is when m = 0).
 */
gfr_status gfr_advance_edges(gfr_ctx *ctx, gfr_graph g, const int32_t *edges, int32_t ne,
                             int32_t *out_src, int32_t *out_edge, int32_t *out_dst, int64_t out_cap,
                             int64_t *count_out, gfr_stream stream);

/*
 * The filter operator on its own (Sec. 4.1): cull and deduplicate a vertex
 * list.  out = the distinct ids of `items` (count ids, host or device memory,
 * duplicates allowed) whose byte exclude[v] is 0 (exclude: n bytes, host or
 * device memory, NULL = keep all), in ascending order.  out: device memory,
 * out_cap elements.  *count_out (host) = number kept.  GFR_E_CAPACITY
 * (nothing written) if that exceeds out_cap; GFR_E_INVALID for an id outside
 * [0,n) or a host output pointer.
 */
gfr_status gfr_filter(gfr_ctx *ctx, gfr_graph g, const int32_t *items, int64_t count,
                      const uint8_t *exclude, int32_t *out, int64_t out_cap, int64_t *count_out,
                      gfr_stream stream);

/*
 * The scan on its own (Sec. 4.4: the exclusive prefix sum that turns a
 * frontier's degrees into output offsets): out[i] = in[0] + ... + in[i-1],
 * exact in 64 bits.  in: count uint32 values, host or device memory.  out:
 * count uint64 values, device memory.  *total_out (host, may be NULL) = the
 * sum of all values.  GFR_E_INVALID for a host `out` or missing pointers.
 */
gfr_status gfr_scan(gfr_ctx *ctx, const uint32_t *in, int64_t count, uint64_t *out, uint64_t *total_out,
                    gfr_stream stream);

/*
 * The near/far split of a frontier on its own (Sec. 4.5, the priority queue
 * that organises a frontier into a near and a far slice): near_out = the
 * entries v of `items` with dist[v] < threshold, far_out = the others, each
 * in input order (duplicates kept).  items: count vertex ids, host or device
 * memory.  dist: n values, host or device memory.  near_out, far_out: device
 * memory, out_cap entries each.  *near_count_out, *far_count_out (host) are
 * always set; GFR_E_CAPACITY (nothing written) if either exceeds out_cap;
 * GFR_E_INVALID for an id outside [0,n), a host output or missing pointers.
 */
gfr_status gfr_split(gfr_ctx *ctx, gfr_graph g, const int32_t *items, int64_t count, const uint32_t *dist,
                     uint32_t threshold, int32_t *near_out, int32_t *far_out, int64_t out_cap,
                     int64_t *near_count_out, int64_t *far_count_out, gfr_stream stream);

/* --------------------------------------------- 2-hop and node rankings */
/*
 * Walks of length two from a seed set (Sec. 4.1: advance from the seeds'
 * edges to their neighbouring edges, returning the far-end vertices):
 *   count_out[v] = number of walks s - u - v, s in seeds, u in N(s), v in N(u)
 * seeds: host array of k >= 1 distinct vertices.  count_out: n uint64 (device
 * or host memory).  The second advance pushes with 64-bit atomics, or pulls
 * over every list when the middle vertices hold more than m / alpha edges
 * (options "twohop.direction": 0 auto, 1 push, 2 pull, and "twohop.alpha",
 * default 10; the result is the same).
 * GFR_E_INVALID for an empty, out-of-range or duplicated seed set.
 */
gfr_status gfr_two_hop(gfr_ctx *ctx, gfr_graph g, const int32_t *seeds, int32_t k,
                       uint64_t *count_out, gfr_stream stream);

/*
 * Personalized PageRank (one of the rankings Sec. 5.5 lists as built on
 * advance): teleport vector p uniform over the seed set, which also receives
 * the rank held by zero-degree vertices:
 *   x_0 = p,  x_{k+1}(v) = (1-d) p(v) + d * (sum_{u in N(v)} x_k(u)/deg(u) + D_k p(v))
 * Stops after the first iteration whose L1 change is below l1_tol, or after
 * max_iter iterations.  FP64 throughout.  seeds: host, k >= 1 distinct.
 * rank_out: n doubles.  GFR_E_INVALID on bad seeds, damping outside (0,1),
 * l1_tol < 0 or max_iter < 1.
 */
gfr_status gfr_ppr(gfr_ctx *ctx, gfr_graph g, const int32_t *seeds, int32_t k, double damping,
                   double l1_tol, int32_t max_iter, double *rank_out, int32_t *iters_out,
                   double *final_l1_out, gfr_stream stream);

/*
 * Bipartite node rankings (Sec. 5.5): the graph's vertices [0, n_left) are
 * hubs and [n_left, n) authorities, and every edge must join the two sides
 * (checked on the device once per graph and split; GFR_E_INVALID otherwise).
 * SALSA (random walk): h_0 = 1/n_left on every hub; per iteration
 *   a(r) = sum_{l in N(r)} h(l)/deg(l),  then  h(l) = sum_{r in N(l)} a(r)/deg(r).
 * HITS: h_0 = 1/sqrt(n_left); per iteration a = B^T h scaled to unit L2 norm,
 * then h = B a scaled to unit L2 norm (B the biadjacency matrix; a zero
 * vector stays zero).  hub_out: n_left doubles, auth_out: n - n_left doubles
 * (device or host memory), the scores after `iters` iterations (iters >= 0).
 * FP64, fixed summation order.
 */
gfr_status gfr_salsa(gfr_ctx *ctx, gfr_graph g, int32_t n_left, int32_t iters, double *hub_out,
                     double *auth_out, gfr_stream stream);
gfr_status gfr_hits(gfr_ctx *ctx, gfr_graph g, int32_t n_left, int32_t iters, double *hub_out,
                    double *auth_out, gfr_stream stream);

/* ---------------------------------------------------------------- batching */
/*
 * k BFS (or SSSP) solves from `sources` (host memory, k >= 1) on one graph,
 * run together: the sources share every read of the graph.  Row i of the
 * output (n elements starting at out + i*n) equals the single-source result
 * for sources[i].  Duplicated sources are allowed.
 */
gfr_status gfr_bfs_batch(gfr_ctx *ctx, gfr_graph g, const int32_t *sources, int32_t k,
                         int32_t *depth_out, gfr_stream stream);
gfr_status gfr_sssp_batch(gfr_ctx *ctx, gfr_graph g, const int32_t *sources, int32_t k,
                          uint32_t *dist_out, gfr_stream stream);

/* ----------------------------------------------------------------- serving */
#define GFR_Q_BFS   1
#define GFR_Q_SSSP  2

typedef struct gfr_query {
    int32_t kind;          /* GFR_Q_BFS or GFR_Q_SSSP                                 */
    int32_t source;        /* source vertex                                           */
    gfr_graph graph;       /* resident graph                                          */
    void *out;             /* n elements (int32 depth / uint32 dist), lent until done */
    int32_t out_on_device; /* nonzero: `out` is device memory of the context's device */
    int32_t reserved;      /* must be 0                                               */
    uint64_t user_tag;     /* returned untouched                                      */
} gfr_query;

/*
 * Queue `count` queries for asynchronous execution; tickets_out[i] receives
 * the ticket of queries[i].  Queries on one graph and of one kind share a
 * 64-lane batched traversal (a session); a query joins a running session at
 * its next level boundary as soon as a lane is free and leaves it when its own
 * traversal ends (continuous batching), so a query may start while others
 * are half done.  A session is created when its device footprint fits the
 * context's budget ("serve.budget_bytes") beside the running ones; sessions
 * of different graphs or kinds run concurrently on their own streams.
 * A query that could never fit the budget -> GFR_E_CAPACITY for the whole
 * call, nothing queued.  A query with a bad source or graph is queued and
 * completes with that error status.
 */
gfr_status gfr_submit_queries(gfr_ctx *ctx, const gfr_query *queries, int32_t count,
                              gfr_ticket *tickets_out);

/*
 * Collect up to `cap` finished tickets (and their statuses) into done/status,
 * waiting up to timeout_us microseconds for at least one (0: do not wait).
 * *ndone receives the count (0 on timeout, still GFR_OK).
 */
gfr_status gfr_poll(gfr_ctx *ctx, gfr_ticket *done, gfr_status *status, int32_t cap,
                    int32_t *ndone, int32_t timeout_us);

/* Cancel a queued query; GFR_E_NOT_FOUND if unknown or already finished. */
gfr_status gfr_cancel(gfr_ctx *ctx, gfr_ticket t);

#ifdef __cplusplus
}
#endif
#endif /* GFR_H */
