/*
 * tc.h — C ABI of the MI355X (gfx950) exact triangle-counting library.
 *
 * The operations follow the problem statement of Arifuzzaman, Khan and Marathe,
 * "Distributed-Memory Parallel Algorithms for Counting and Listing Triangles in
 * Big Graphs" (arXiv 1706.05151):
 *   - the input is an undirected graph G(V,E) on vertex ids 0..n-1 (Section 2);
 *   - T is the number of triangles, T_v the number containing v (Section 2);
 *   - C_v = T_v / C(d_v,2) is the local clustering coefficient (Section 2, Section 9);
 *   - the triangle list is produced from the same intersections (Section 8);
 *   - the sparsified estimate keeps each edge with probability q and returns
 *     T_s / q^3 (Section 7).
 * The counting method is NodeIteratorN with the degree order of Eq. (1):
 * u precedes v iff d_u < d_v, or d_u == d_v and u < v.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device (HBM) pointers of the current HIP device;
 *     the caller allocates and owns them. The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). All
 *     device work is ordered on it. Calls that return host scalars synchronise it.
 *   - Functions return a tc_status and never abort. On error the outputs are
 *     left untouched (except where stated) and tc_last_error() holds a message
 *     for the calling thread.
 *   - A tc_graph is read-only after it is built. Queries on one graph may run
 *     concurrently on different streams; each call takes its own scratch memory.
 *   - Limits: n <= 2^31 - 2^25 vertices and at most 2^32 - 2^25 input edge
 *     records (32-bit counters with grid strides of up to 2^24), else TC_E_RANGE
 *     and TC_E_INVAL.
 */
#ifndef TC_H_
#define TC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_graph tc_graph;

typedef enum tc_status {
  TC_OK = 0,
  TC_E_INVAL = -1,  /* bad argument (NULL where required, negative size, ...) */
  TC_E_NOMEM = -2,  /* device allocation failed */
  TC_E_DEVICE = -3, /* HIP runtime error */
  TC_E_RANGE = -4,  /* vertex id outside [0,n), n < 0, or q outside (0,1] */
  TC_E_TRUNC = -5   /* output capacity smaller than the result */
} tc_status;

/* tc_build_csr flag: src/dst are device pointers (otherwise host pointers). */
#define TC_IN_DEVICE 1u

/*
 * Build the device graph of Section 2 from a raw edge list and prepare
 * NodeIteratorN (Section 3, the algorithm figure after Eq. (1)): drop
 * self-loops, merge duplicate and reversed pairs, compute degrees d_v, orient
 * every edge from the earlier to the later endpoint under Eq. (1), and store
 * the oriented lists N_v sorted ascending as a CSR.
 *   src, dst   : int32[num_edges] endpoint ids (host, or device with TC_IN_DEVICE).
 *                May be freed as soon as the call returns.
 *   num_edges  : 0 .. 2^32 - 2^25 raw records (loops and duplicates allowed;
 *                more gives TC_E_INVAL).
 *   n          : 0 .. 2^31 - 2^25 vertices (else TC_E_RANGE); ids must lie in
 *                [0,n) else TC_E_RANGE.
 *   out        : receives the new graph; owned by the caller until tc_graph_free.
 * Internally vertices are numbered by their position in the degree order, so
 * that every oriented list holds only later vertices in ascending order.
 * Synchronises `stream`.
 */
tc_status tc_build_csr(const int32_t* src, const int32_t* dst, int64_t num_edges, int32_t n,
                       uint32_t flags, void* stream, tc_graph** out);

/* n, m (unique undirected edges), d_max and the largest oriented list size
 * dhat_max (Definition of effective degree, Section 3). Any output may be NULL. */
tc_status tc_graph_info(const tc_graph* g, int32_t* n, int64_t* m, int32_t* d_max, int32_t* dhat_max);

/* Device bytes the graph holds now (its CSR, work plans, vertex arrays and
 * workspace, as the library's allocator reserved them), for callers that keep
 * many graphs resident under a memory budget. */
tc_status tc_graph_bytes(const tc_graph* g, uint64_t* bytes);

/* Release the graph and its device memory once the work already queued on it
 * is done (calls that return before their work ends are waited for on the host;
 * other streams of the device are not synchronised). NULL is ignored. */
void tc_graph_free(tc_graph* g);

/*
 * T = sum over oriented edges (v,u) of |N_v ∩ N_u| (NodeIteratorN, Section 3;
 * each triangle counted once by Theorem 1). 64-bit total. Synchronises `stream`.
 */
tc_status tc_count(tc_graph* g, void* stream, uint64_t* T);

/*
 * T and the per-node counts T_v: each triangle (v,u,w) adds one to T_v, T_u
 * and T_w (local-count figure, Section 9). t_dev: uint64[n] device array,
 * indexed by the caller's vertex ids, fully overwritten. T may be NULL.
 * Synchronises `stream`.
 */
tc_status tc_count_per_node(tc_graph* g, void* stream, uint64_t* T, uint64_t* t_dev);

/*
 * Local clustering coefficients C_v = T_v / C(d_v,2) (Section 2), returned as
 * the exact rational num/den and its IEEE binary64 quotient (round to nearest,
 * one true division). Vertices with d_v < 2 get num = den = 0 and c = 0.0.
 * num_dev, den_dev: uint64[n]; c_dev: double[n]; any may be NULL.
 * Synchronises `stream`.
 */
tc_status tc_clustering(tc_graph* g, void* stream, uint64_t* num_dev, uint64_t* den_dev, double* c_dev);

/*
 * The triangle list (Section 8): every triangle once, as three ids in
 * ascending order, the list sorted lexicographically. tri_dev: int32[cap][3].
 * Sizing idiom: tri_dev == NULL or cap == 0 returns TC_OK with *count = T;
 * 0 < cap < T returns TC_E_TRUNC with *count = T and writes nothing.
 * Synchronises `stream`.
 */
tc_status tc_list(tc_graph* g, void* stream, int32_t* tri_dev, int64_t cap, int64_t* count);

/*
 * Sparsified estimate (Section 7): each undirected edge {a,b} (a<b, caller ids)
 * is kept independently with probability q, decided by
 *   H = mix(mix(seed ^ 0x5350415253494659) ^ (a<<32 | b)),
 * mix = the SplitMix64 output function (Steele, Lea and Flood, 2014), keep iff
 * H < floor(q * 2^64) (q = 1 keeps all). T_sampled is the exact count on the
 * kept edges, m_kept their number and estimate = T_sampled / (q*q*q).
 * q outside (0,1] gives TC_E_RANGE. Any output may be NULL. Synchronises `stream`.
 */
tc_status tc_sparsify_count(tc_graph* g, double q, uint64_t seed, void* stream, uint64_t* T_sampled,
                            int64_t* m_kept, double* estimate);

/* ------------------------------------------------------------------ extras */

/*
 * The same total as tc_count from the plain kernel: one thread per oriented
 * edge, two-pointer merge of N_v and N_u straight from HBM (the intersection of
 * the NodeIteratorN figure, no staging). The baseline the tuned kernels are
 * measured against. Synchronises `stream`.
 */
tc_status tc_count_plain(tc_graph* g, void* stream, uint64_t* T);

/* Merge work of Theorem 2, W = sum over oriented edges (v,u) of (dhat_v + dhat_u),
 * and the wedge count P = sum_v C(dhat_v, 2). Either may be NULL. */
tc_status tc_graph_work(tc_graph* g, void* stream, uint64_t* W, uint64_t* P);

/*
 * sum_v d_v * dhat_v, the quantity Theorem 3 shows the degree order minimises,
 * for the order this graph was built with (its TC_OPT_ORDER value goes to
 * *order_kind). Either output may be NULL. Synchronises `stream`.
 */
tc_status tc_graph_order_cost(tc_graph* g, void* stream, uint64_t* cost, int32_t* order_kind);

/*
 * The static load balancing of Section 5, counted on the device: core nodes
 * in id order are split into `parts` contiguous ranges by the boundary rule
 * x_j = argmin_v F(v) >= j*alpha, alpha = F(n-1)/parts (compared exactly as
 * F(v)*parts >= j*F(n-1)), where F is the prefix sum of the cost f(v) of
 * `scheme`: 0 f = 1, 1 f = d_v, 2 f = dhat_v, 3 f = d_v*dhat_v, 4 f = dhat_v^2,
 * 5 f = sum_{u in N_v} (dhat_v + dhat_u) (the cost-function table), 6 f =
 * sum over the lower-ordered neighbours u of (dhat_v + dhat_u) (the cost of
 * the space-efficient algorithm, Section 6). Each range is counted by one
 * workgroup with the NodeIteratorN merge. Outputs: *T (host) the exact total;
 * bounds_dev int64[parts+1] the boundary nodes (0 and n at the ends);
 * work_dev uint64[parts] each range's merge work sum_v sum_{u in N_v}
 * (dhat_v + dhat_u) (Theorem 2). Either device array may be NULL. TC_E_INVAL
 * for an unknown scheme, parts < 1 or a sampled graph. Synchronises `stream`.
 */
tc_status tc_count_partitioned(tc_graph* g, void* stream, int32_t scheme, int32_t parts, uint64_t* T,
                               int64_t* bounds_dev, uint64_t* work_dev);

/*
 * Coreness of every vertex in the caller's ids (the k-core order compared in
 * Section 4, "An Optimal Node Ordering"): core_dev int32[n] gets the largest k
 * such that v lies in a subgraph whose vertices all have degree >= k, computed
 * on the device by level-synchronous peeling. core_dev is caller-owned device
 * memory. TC_E_INVAL on a sampled graph or NULL arguments. Synchronises `stream`.
 */
tc_status tc_graph_coreness(tc_graph* g, void* stream, int32_t* core_dev);

/*
 * The orientation order as positions: order_dev int32[n] gets, at position r,
 * the caller id of the vertex ranked r-th (0 first) in the total order the
 * graph was oriented by (Eq. (1) for the degree order). Caller-owned device
 * memory. Synchronises `stream`.
 */
tc_status tc_graph_order(tc_graph* g, void* stream, int32_t* order_dev);

/*
 * One GPU's share of a sharded count (the overlapping partitions of Section 5
 * with the whole oriented graph resident): shard j holds the core nodes with
 * positions [bounds[j], bounds[j+1]) in the orientation order. The boundaries
 * follow the rule x_j = argmin_v F(v) >= j*alpha, alpha = F(n-1)/k (compared
 * exactly as F(v)*k >= j*F(n-1)), over positions, with F the prefix sum of a
 * per-node cost f:
 *   cost 0: f(v) = sum_{u in N_v} (dhat_v + dhat_u), the DPD row of the
 *           cost-function table of Section 5 (the merge cost of Theorem 2);
 *   cost 1: f(v) = 2 dhat_v (dhat_v - 1) + 16 dhat_v + sum_{u in N_v} dhat_u,
 *           the pivot kernel's own work model: four times C(dhat_v, 2)
 *           probes plus 4 per in-edge record, and a quarter of the lengths of
 *           the lists those records meet.
 * bounds is host int32[k+1], with bounds[0] = 0 and bounds[k] = n. TC_E_INVAL
 * for k < 1, an unknown cost or NULL arguments. Synchronises `stream`.
 */
tc_status tc_shard_bounds(tc_graph* g, void* stream, int32_t k, int32_t cost, int32_t* bounds);

/*
 * The triangles counted by the shard whose core nodes have positions [lo, hi)
 * in the orientation order: sum over those v of sum_{u in N_v} |N_v ∩ N_u|
 * (NodeIteratorN restricted to the core nodes, each triangle counted at its
 * lowest vertex, Theorem 1), into *T (host). The shards of tc_shard_bounds
 * add up to tc_count. The shard's work plan (its in-edge records and items)
 * is built on the first call for a range and kept on the graph until a call
 * for another range. TC_E_RANGE unless 0 <= lo <= hi <= n. Works on sampled
 * graphs. Synchronises `stream`.
 */
tc_status tc_count_shard(tc_graph* g, void* stream, int32_t lo, int32_t hi, uint64_t* T);

/*
 * Sparsification with overlapping partitions (Section 7, parallel
 * sparsification; Eq. var2): the core nodes are split into `parts` shards as
 * in tc_shard_bounds with cost 0, and shard i keeps each edge it uses independently of the
 * other shards, with the keep rule of tc_sparsify_count under the seed
 * seed_i = output i+1 of SplitMix64 started at `seed` (seed + (i+1)*
 * 0x9E3779B97F4A7C15, then the SplitMix64 finaliser). Shard i counts the
 * triangles of its own sample whose lowest vertex is one of its core nodes.
 * The estimate sum_i T_i / q^3 is unbiased; its variance is
 * (1/q^3 - 1) T + 2 k' (1/q - 1) with k' the pairs of triangles sharing an
 * edge whose lowest vertices lie in one shard. Outputs (each may be NULL):
 * T_parts host uint64[parts], bounds host int32[parts+1], *T_sampled the sum,
 * *estimate. parts = 1 gives the same sample as tc_sparsify_count with seed
 * seed_0. TC_E_RANGE for q outside (0,1]; TC_E_INVAL for parts < 1 or a
 * sampled graph. Synchronises `stream`.
 */
tc_status tc_sparsify_count_partitioned(tc_graph* g, double q, uint64_t seed, int32_t parts, void* stream,
                                        uint64_t* T_parts, int32_t* bounds, uint64_t* T_sampled, double* estimate);

/*
 * The oriented CSR in rank space, the input of tc_count_streamed: off int64[n+1]
 * and adj int32[m], row r holding the ranks after r adjacent to the r-th vertex
 * of the orientation order, ascending. Either pointer may be NULL; each may be
 * host or device memory (copied with hipMemcpyDefault). For a batch, the
 * ranks of all graphs together. Synchronises `stream`.
 */
tc_status tc_graph_export_csr(tc_graph* g, void* stream, int64_t* off, int32_t* adj);

/*
 * The same rank-space CSR as tc_build_csr + tc_graph_export_csr, for a graph
 * whose edge list stays in host memory and need not fit the device: the
 * simple graph, degrees, the order of Eq. (1) and the sorted oriented lists
 * N_v (Section 3) are computed with the records streamed through the GPU in
 * pieces that fit budget_bytes (the graphs larger than one machine's memory
 * of Section 6, here larger than one device). The records are split by a hash
 * of their smaller endpoint into parts sorted and deduplicated one at a time
 * (degrees accumulate on the device); after the ranks, the unique edges
 * stream through again to count the rows. The rows are cut into ranges that
 * fit the budget; with three ranges or more the unique edges stream through
 * once more and are split by range (each range then loads only its own
 * part), with fewer they stream through once per range. Each range is sorted
 * and its entries copied out.
 *   src, dst : host int32[num_edges] ids in [0,n) (pinned memory copies fastest).
 *   off      : host int64[n+1], written: row r holds adj[off[r] .. off[r+1]).
 *   adj      : host int32 with room for the unique edges (num_edges suffices).
 *   m        : receives the number of unique undirected edges.
 *   info     : host uint64[4] or NULL: parts, row ranges, bytes copied to the
 *              device, bytes copied to the host.
 * The budget covers the library's device buffers of this call (edge pieces,
 * sort buffers, per-vertex arrays of 64 bytes per vertex); it must be at least
 * 64 n + 32 MiB, else TC_E_NOMEM, as when one part or one row does not fit.
 * TC_E_RANGE for ids outside [0,n). The result feeds tc_count_streamed.
 * Synchronises `stream`.
 */
tc_status tc_build_csr_host(const int32_t* src, const int32_t* dst, int64_t num_edges, int32_t n,
                            uint64_t budget_bytes, void* stream, int64_t* off, int32_t* adj, int64_t* m,
                            uint64_t* info);

/*
 * Exact T of an oriented CSR kept in host memory, streamed through the GPU
 * under a device-memory budget (the non-overlapping partitions of Section 6,
 * with the surrogate pairing). The rows are split into pivot partitions V_j,
 * each sized to about half of budget_bytes. The rows of each V_j are loaded
 * once and serve as their own sources. The rows before V_j are shipped to it
 * in chunks sized to the other half (N_v goes to the owner of u once per
 * chunk, not once per edge). For each source range, the in-edge records
 * (v,u), u in V_j, count |N_v after u ∩ N_u| with the pivot kernel. Each
 * triangle is counted once, at the partition of its middle vertex. The next
 * chunk is copied in while the current one is counted, and a partition is
 * loaded range by range (its last rows first) so that its first pairs are
 * counted while the rest is still being copied.
 *
 * Input: off host int64[n+1] with off[0] = 0 and off[n] = m; adj int32[m]
 * (host, pinned for full copy speed, or device memory). Row r must hold
 * strictly ascending values in (r, n): a rank-space CSR such as
 * tc_graph_export_csr writes. The offsets at the ends of every partition and
 * chunk are checked on the host, the offsets between them and the rows on the
 * device, before anything is counted. A violation gives TC_E_INVAL,
 * as do off in device memory, NULL
 * arguments and budget_bytes < 4096; n above 2^31 - 2^25 gives TC_E_RANGE.
 * TC_E_NOMEM if one row alone does not fit
 * half the budget. The budget covers the copies, records and plans; the
 * kernel's counters come on top. Output: *T. info (may be NULL) gets uint64[4]:
 * pivot partitions, chunks shipped, (partition, source range) pairs visited,
 * bytes copied to the device. Runs on the current device. Synchronises
 * `stream`.
 */
tc_status tc_count_streamed(const int64_t* off, const int32_t* adj, int32_t n, int64_t m, uint64_t budget_bytes,
                            void* stream, uint64_t* T, uint64_t* info);

/*
 * Export the degree data in the caller's ids: deg_dev int32[n] = d_v and
 * dhat_dev int32[n] = |N_v| (effective degree, Section 3). Either may be NULL.
 */
tc_status tc_graph_degrees(tc_graph* g, void* stream, int32_t* deg_dev, int32_t* dhat_dev);

/*
 * Export the oriented lists in the caller's ids: off_dev int64[n+1] and
 * adj_dev int32[m] hold N_v for v = 0..n-1, each list ascending by id (the
 * layout of the NodeIteratorN preprocessing step). Either may be NULL.
 */
tc_status tc_graph_oriented(tc_graph* g, void* stream, int64_t* off_dev, int32_t* adj_dev);

/*
 * Rebuild the graph's work plan (the in-edge records grouped by pivot and the
 * work items cut from their cost prefix by the boundary rule of Section 5,
 * load balancing) with the current TC_OPT_HUB_DHAT and TC_OPT_ITEM_WORK
 * options. Calls that count rebuild the plan themselves when those options
 * changed, except tc_batch_count, which uses the plan as it is; tuners call
 * this before timing a batch. The old plan is freed after every launch that
 * read it, ordered on `stream`. TC_E_INVAL once a tc_batch_count on this
 * graph was captured into a HIP graph: the capture holds the plan's
 * addresses, so the plan stays as it is for the graph's lifetime (calls that
 * count then use it whatever the options; results do not depend on them).
 * Synchronises `stream`.
 */
tc_status tc_graph_replan(tc_graph* g, void* stream);

/* Options the graph's current work plan was built with (TC_OPT_HUB_DHAT as
 * clamped by the library, TC_OPT_ITEM_WORK as set, 0 = automatic) and whether
 * it is frozen by a capture (1) or not (0). Any output may be NULL. TC_E_INVAL
 * if the graph has no plan. */
tc_status tc_graph_plan_info(const tc_graph* g, int64_t* hub_dhat, int64_t* item_work, int32_t* frozen);

/*
 * Tuning options (process-wide; read at the start of each call).
 *   TC_OPT_KERNEL        : 0 auto (plain merge when the wedge checks are
 *                          fewer than 16 per edge, else pivot-staged),
 *                          1 plain merge, 2 pivot-staged
 *   TC_OPT_HUB_DHAT      : lists longer than this use the block-per-pivot path
 *                          (default 256, the largest per-wave table)
 *   TC_OPT_ITEM_WORK     : target probes per work item of the partitioner;
 *                          0 (default) derives it from the graph: about 8
 *                          items per resident wave, within [4096, 65536]
 *   TC_OPT_BLOCKS_PER_CU : blocks per compute unit of the persistent launch
 *   TC_OPT_HUB_BUCKET_LOAD : target list entries per 4-slot LDS hash bucket
 *                          of the block path (1 or 2)
 *   TC_OPT_ORDER         : total order used by graphs built afterwards:
 *                          0 degree (Eq. (1), the default), 1 id, 2 a fixed
 *                          pseudo-random permutation, 3 degree descending,
 *                          4 coreness (ties by id; the build first orients by
 *                          degree to compute the coreness, then rebuilds)
 *                          (the orderings compared in Section 4)
 * Options change speed only, never results (Theorem 1: any total order counts
 * each triangle once). Returns TC_E_INVAL for an unknown key or an
 * out-of-range value.
 */
typedef enum tc_option {
  TC_OPT_KERNEL = 0,
  TC_OPT_HUB_DHAT = 1,
  TC_OPT_ITEM_WORK = 2,
  TC_OPT_BLOCKS_PER_CU = 3,
  TC_OPT_HUB_BUCKET_LOAD = 4,
  TC_OPT_ORDER = 5
} tc_option;
tc_status tc_set_option(tc_option key, int64_t value);
int64_t tc_get_option(tc_option key);

/* ---------------------------------------------------------------- batching */

/*
 * Build many independent graphs as one device graph (their disjoint union):
 * graph g has n_per_graph[g] vertices and edge records
 * [edge_off[g], edge_off[g+1]) of src/dst, with ids local to the graph.
 * All arrays are host memory unless TC_IN_DEVICE (src/dst only; edge_off and
 * n_per_graph are always host). Counting on the result gives per-graph totals
 * with tc_batch_count; per-node arrays are indexed by base[g] + local id with
 * base[g] = n_per_graph[0] + ... + n_per_graph[g-1]. More than 2^31 - 2^25
 * vertices in all gives TC_E_RANGE.
 */
tc_status tc_batch_build(const int32_t* src, const int32_t* dst, const int64_t* edge_off,
                         const int32_t* n_per_graph, int32_t num_graphs, uint32_t flags, void* stream,
                         tc_graph** out);

/* Number of graphs in a batch graph (1 for tc_build_csr graphs). */
tc_status tc_batch_size(const tc_graph* g, int32_t* num_graphs);

/*
 * Per-graph totals T_dev[num_graphs] (device uint64) and, if t_dev != NULL,
 * per-node counts t_dev[sum n] in one launch sequence. The kernel follows
 * TC_OPT_KERNEL: the plain merge (one thread per oriented edge) for 1, or for
 * 0 when the batch makes fewer than 16 probes per edge; the pivot kernel
 * otherwise. Does not synchronise
 * `stream` (results are ready when the stream reaches this point), so the call
 * can be captured in a HIP graph. Scratch memory comes from the graph's own
 * workspace: calls on one batch graph must not overlap. Uses the work plan as
 * it is (see tc_graph_replan). Capturing the call freezes the plan: the HIP
 * graph holds the addresses of the plan's and the graph's arrays, so it must
 * not be replayed after tc_graph_free.
 */
tc_status tc_batch_count(tc_graph* g, void* stream, uint64_t* T_dev, uint64_t* t_dev);

/* ------------------------------------------------------------ serving */

/*
 * Counts of several resident graphs in one launch of the persistent kernel:
 * the work items of all graphs are drained from one device queue. T_dev:
 * device uint64[k], T of graph i at index i. With per_node != 0, t_dev[i] is a
 * device uint64[n_i] array (caller ids) receiving T_v of graph i. Graphs must
 * live on one device; sampled graphs (tc_sparsify_build) are allowed for
 * totals. Does not synchronise `stream`; scratch is taken from the stream-
 * ordered allocator and released on `stream`.
 */
tc_status tc_multi_count(tc_graph* const* graphs, int32_t k, int32_t per_node, void* stream, uint64_t* T_dev,
                         uint64_t* const* t_dev);

/*
 * Clustering coefficients (Section 2) from per-node counts t_dev (caller ids,
 * e.g. from tc_multi_count) without recounting: same outputs and rules as
 * tc_clustering. Does not synchronise `stream`.
 */
tc_status tc_clustering_from_counts(tc_graph* g, void* stream, const uint64_t* t_dev, uint64_t* num_dev,
                                    uint64_t* den_dev, double* c_dev);

/*
 * 128-bit digest of a clustering answer (num, den, c as tc_clustering writes
 * them, n entries), so that servers can record and compare answers without
 * copying them to the host: with f the SplitMix64 output function and
 * h_v = f(f(f(f(v ^ 0x434C555354455221) ^ num[v]) ^ den[v]) ^ bits(c[v])),
 * digest_dev[0] = sum_v h_v and digest_dev[1] = sum_v f(h_v ^ 0x4449474553543132),
 * both modulo 2^64. digest_dev: device uint64[2]. Does not synchronise `stream`.
 */
tc_status tc_clustering_digest(const uint64_t* num_dev, const uint64_t* den_dev, const double* c_dev, int32_t n,
                               void* stream, uint64_t* digest_dev);

/*
 * The edge sample of tc_sparsify_count (Section 7: same keep rule, q, seed)
 * as a graph of its own, ready for tc_count / tc_multi_count. Orientation
 * follows the degrees of the full graph. Per-node, clustering and listing
 * calls on the result return TC_E_INVAL. Free with tc_graph_free.
 * Synchronises `stream`.
 */
tc_status tc_sparsify_build(tc_graph* g, double q, uint64_t seed, void* stream, tc_graph** out);

/* T_sampled / (q*q*q), the estimate of Section 7 (the expression tc_sparsify_count uses). */
double tc_sparsify_estimate(uint64_t T_sampled, double q);

/* ------------------------------------------------------- allocation-free */

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same results as tc_count_per_node
 * (T and the per-node counts T_v by caller id, fully overwriting t_dev
 * uint64[n]), computed without allocating or freeing any device memory.
 * The work-queue counters, the total and the per-node counts by rank live in
 * a static device array of the library, 32 MiB plus 32 bytes, which every
 * device the library runs on holds until the process ends.
 *   - At most 2^22 vertices (TC_E_RANGE above that, t_dev untouched).
 *   - Uses the graph's work plan as tc_build_csr made it (options set since
 *     then are not applied, which changes speed only); TC_E_INVAL on a
 *     sampled graph.
 *   - Every call on one device shares that device's array: calls that
 *     overlap on one device (other threads, other streams) race and must not
 *     be made. The array is cleared by each call before use.
 *   - Holds the graph's lock until its results are in, so other calls on the
 *     same graph wait for it.
 * Synchronises `stream` (not capturable).
 */
tc_status tc_count_per_node_noalloc(tc_graph* g, void* stream, uint64_t* T, uint64_t* t_dev);

/* ------------------------------------------------------------------ errors */

const char* tc_status_str(tc_status s);
/* Message for the last failing call of this thread ("" if none). */
const char* tc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
