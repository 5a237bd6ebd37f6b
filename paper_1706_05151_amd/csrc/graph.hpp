// The device graph behind the opaque tc_graph handle, and the internal entry
// points shared by the library's translation units.
#pragma once

#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tc {

// Device arrays owned by a graph, taken from the library's block cache on the
// building stream. They are freed only after a device synchronisation, so the
// free is recorded on the null stream.
template <typename T>
struct Owned {
  T* p = nullptr;
  size_t n = 0;
  Owned() = default;
  Owned(const Owned&) = delete;
  Owned& operator=(const Owned&) = delete;
  ~Owned() { reset(); }
  // Callers free only when no stream still uses the array (after a device
  // synchronisation).
  void reset() {
    if (p) dev_free(p, nullptr);
    p = nullptr;
    n = 0;
  }
  // Free ordered on stream s: the block is reused only after the work queued
  // on s before this call (callers first make s wait for every reader).
  void reset_on(hipStream_t s) {
    if (p) dev_free(p, s);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count, hipStream_t s = nullptr) {
    reset();
    n = count;
    if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T), s));
  }
  // take over a stream-ordered buffer
  void adopt(DevBuf<T>& b) {
    reset();
    n = b.size();
    p = b.detach();
  }
};

// Work item of the pivot-staged intersection: pivot u (a rank), the slice
// [nbeg, nend) of the CSR entries of N_u to stage, and the slice [ibeg, iend)
// of u's in-edge records to probe against it.
struct PivotItem {
  int32_t u;
  uint32_t ibeg, iend;
  uint32_t nbeg_rel;  // offset of the staged slice inside N_u
  uint32_t nlen;      // length of the staged slice
  uint32_t pad;
};

// In-edge record for pivot u: the oriented edge (v,u) sits at CSR index e of
// N_v; the candidates for third vertices are N_v[e+1 .. end of row v).
struct InRec {
  uint32_t a_begin;  // e + 1
  uint32_t a_len;    // entries of N_v after u
};

// Launches that read a plan's arrays: an event is recorded after each launch,
// so that replacing or freeing the plan can wait for them (on a stream, or on
// the host) instead of synchronising the whole device. Completed events are
// pruned at the next record.
struct PlanUsers {
  std::mutex mu;
  std::vector<hipEvent_t> events;
  PlanUsers() = default;
  PlanUsers(const PlanUsers&) = delete;
  PlanUsers& operator=(const PlanUsers&) = delete;
  ~PlanUsers() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
  void record(hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu);
    size_t keep = 0;
    for (hipEvent_t e : events) {
      if (hipEventQuery(e) == hipSuccess) (void)hipEventDestroy(e);
      else events[keep++] = e;
    }
    (void)hipGetLastError();  // a pending query leaves hipErrorNotReady behind
    events.resize(keep);
    hipEvent_t e;
    TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (hipEventRecord(e, s) != hipSuccess) {
      (void)hipEventDestroy(e);
      TC_HIP(hipGetLastError());
    }
    events.push_back(e);
  }
  // Makes stream s wait for every recorded launch; the events are then released.
  void wait_on(hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu);
    for (hipEvent_t e : events) {
      TC_HIP(hipStreamWaitEvent(s, e, 0));
      (void)hipEventDestroy(e);
    }
    events.clear();
  }
  // Host wait for every recorded launch.
  void sync() {
    std::lock_guard<std::mutex> lk(mu);
    for (hipEvent_t e : events) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
    events.clear();
  }
};

// The pivot work plan of one oriented CSR (built lazily, cached on the graph):
// the in-edge records of the oriented edges whose source rank lies in
// [src_lo, src_hi) (all edges for the graph's own plan), grouped by pivot, and
// the work items over them.
struct PivotPlan {
  bool ready = false;
  int32_t src_lo = 0, src_hi = 0;
  Owned<InRec> inrec;        // in-edge records grouped by pivot
  Owned<int64_t> in_off;     // [n+1]
  Owned<PivotItem> items;    // hub items first, then wave items
  uint64_t n_hub_items = 0;  // items processed by whole blocks
  uint64_t n_wave_items = 0; // items processed by single waves
  Owned<int32_t> grouped;    // small pivots served from a shared queue
  uint64_t n_grouped = 0;
  int64_t hub_dhat = 0, item_work = 0;  // options the plan was built with
  uint64_t probes = 0;       // sum of suffix lengths |A| over records whose pivot has a non-empty N_u
  // Set when a launch reading the plan was captured into a HIP graph: the
  // graph holds the arrays' addresses, so the plan is never rebuilt or freed
  // before the graph (tc_graph) itself.
  bool frozen = false;
  PlanUsers users;
  uint64_t n_split_items() const { return n_wave_items; }
  void reset() {
    ready = false;
    frozen = false;
    inrec.reset();
    in_off.reset();
    items.reset();
    grouped.reset();
    n_hub_items = n_wave_items = n_grouped = probes = 0;
    hub_dhat = item_work = 0;
    src_lo = src_hi = 0;
  }
  // Frees the arrays on stream s after s has waited for every launch that read them.
  void release_on(hipStream_t s) {
    users.wait_on(s);
    inrec.reset_on(s);
    in_off.reset_on(s);
    items.reset_on(s);
    grouped.reset_on(s);
    reset();
  }
};

// An oriented CSR in rank space: vertices are numbered by their position in
// the degree order (Eq. (1)), so N_v holds only ranks > v, ascending.
struct Csr {
  int32_t n = 0;
  int64_t m = 0;
  int32_t dhat_max = 0;
  Owned<int64_t> off;  // [n+1]
  Owned<int32_t> adj;  // [m]
  Owned<int32_t> src;  // [m] row of each entry
  PivotPlan plan;      // all oriented edges
  PivotPlan shard;     // the edges of one range of source ranks (tc_count_shard)
};

}  // namespace tc

struct tc_graph {
  int device = 0;
  int32_t n = 0;   // vertices (all graphs of a batch together)
  int64_t m = 0;   // unique undirected edges
  int32_t d_max = 0;
  int bits = 1;    // bits of a vertex id
  int order_kind = 0;  // total order the orientation used (TC_OPT_ORDER at build time)
  tc::Csr csr;
  tc::Owned<int32_t> order;  // [n] rank -> caller id
  tc::Owned<int32_t> rank;   // [n] caller id -> rank
  tc::Owned<int32_t> deg;    // [n] d_v by caller id
  // batches
  int32_t num_graphs = 1;
  tc::Owned<int32_t> graph_of_rank;  // [n] graph index of each rank (batches only)
  std::vector<int32_t> vbase;        // [num_graphs+1] first caller id of each graph
  // workspace for the capturable batched count
  tc::Owned<unsigned char> workspace;
  size_t workspace_bytes = 0;
  // sampled graphs (tc_sparsify_build): edges kept and the keep probability
  bool sampled = false;
  double q = 1.0;
  std::mutex mu;  // guards lazy plan construction
};

namespace tc {

struct Options {
  int64_t kernel = 0;        // 0 auto, 1 plain, 2 pivot
  int64_t hub_dhat = 256;    // pivots with |N_u| > hub_dhat use the block path
  int64_t item_work = 0;     // target probes per work item (0: from the graph's total)
  int64_t blocks_per_cu = 8; // persistent launch occupancy
  int64_t hub_bucket_load = 2;  // entries per 4-slot bucket of a hub table (1 or 2)
  int64_t order = 0;            // total order of the orientation (0 degree, 1 id, 2 random, 3 degree descending, 4 coreness)
};
Options get_options();

// build.hip
// order: TC_OPT_ORDER value recorded on the graph; key_by_id (device, optional)
// replaces the degree as the ascending order key (ties by id). tail (pinned
// host words, optional): the last readback [look-back failure, dhat_max,
// d_max] is copied there and left for the caller to read with
// build_graph_finish after its next synchronisation of s; without it
// build_graph synchronises and finishes itself.
void build_graph(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, const int64_t* edge_off_host,
                 const int32_t* n_per_graph_host, int32_t num_graphs, bool on_device, hipStream_t s, tc_graph* g,
                 int order, const int32_t* key_by_id, uint64_t* tail = nullptr);
void build_graph_finish(tc_graph* g, const uint64_t* tail);
// the longest row of a CSR, copied (as a 64-bit word) into pinned host memory without synchronising
void row_max_to_host(const int64_t* off, int32_t n, hipStream_t s, uint64_t* host);

// The rank-space oriented CSR of a host edge list built under a device budget
// into host memory: off_h[n+1], adj_h[>= m]; info = {parts, row ranges, bytes
// copied to the device, bytes copied to the host}
void build_host_csr(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, uint64_t budget, hipStream_t s,
                    int64_t* off_h, int32_t* adj_h, int64_t* m_out, uint64_t info[4]);

// count.hip
enum CountMode { kCountTotal = 0, kCountPerNode = 1, kCountList = 2 };
struct CountArgs {
  int mode = kCountTotal;
  unsigned long long* total = nullptr;     // device, one counter (whole graph)
  unsigned long long* per_graph = nullptr; // device [num_graphs] (optional)
  const int32_t* graph_of_rank = nullptr;  // device [n] (with per_graph)
  unsigned long long* t_rank = nullptr;    // device [n] per-node counts by rank
  const int32_t* order = nullptr;          // rank -> caller id (listing)
  int32_t* tri = nullptr;                  // device [cap][3] (listing)
  unsigned long long* cursor = nullptr;    // device listing cursor
  int64_t cap = 0;
  unsigned long long* queues = nullptr;    // device [3] work-queue counters (optional)
  // Record the launch as a user of the plan (see note_plan_use). Callers that
  // hold the graph's lock until the launch has finished may skip it.
  bool note_use = true;
};
// Builds the graph's plan unless one matching the options is ready; a frozen
// plan (captured in a HIP graph) is kept whatever the options.
void ensure_plan(Csr& c, hipStream_t s, const Options& o);
// Rebuilds the graph's plan with the options (TC_E_INVAL if frozen).
void rebuild_plan(Csr& c, hipStream_t s, const Options& o);
// After work reading P was queued on s: freezes P if s is capturing a HIP
// graph, else records an event that replacing or freeing P waits on.
void note_plan_use(PivotPlan& P, hipStream_t s);
// Plan steps from in-edge keys (pivot << 32 | e) sorted by pivot (stable in e):
// the records and their cost prefix fin (lens: suffix lengths in key order, or
// null to take them from c.off / c.src; filled: P.inrec already holds the
// records, and the cost prefix is taken from lens, or from the records when
// lens is null), then the classification and items.
void plan_records(Csr& c, PivotPlan& P, const uint64_t* sk, const uint32_t* sl, uint64_t mi, DevBuf<int64_t>& fin,
                  hipStream_t s, bool filled = false);
// sort_fail (device, optional): a sort failure flag checked at plan_items' first synchronisation
void plan_items(Csr& c, PivotPlan& P, const int64_t* fin, uint64_t mi, hipStream_t s, const Options& o,
                const uint32_t* sort_fail = nullptr);
// the plan of the oriented edges whose source rank lies in [lo, hi), into c.shard
void ensure_shard_plan(Csr& c, int32_t lo, int32_t hi, hipStream_t s, const Options& o);
// triangles whose lowest vertex (in the orientation order) has rank in [lo, hi), added to *total
void count_shard(Csr& c, int32_t lo, int32_t hi, unsigned long long* total, hipStream_t s, const Options& o);
// ranks [bounds[j], bounds[j+1]) of shard j: the boundary rule over the cost
// (0: sum_{u in N_v} (dhat_v + dhat_u); 1: 2 dhat_v (dhat_v - 1) + 16 dhat_v +
// sum_{u in N_v} dhat_u); bounds int64[k+1] (device)
void shard_bounds(const Csr& c, int32_t k, int cost, int64_t* bounds, hipStream_t s);
// one persistent launch of the pivot kernel over the records and items of P (a plan of c)
void launch_pivot(const Csr& c, PivotPlan& P, const CountArgs& a, hipStream_t s, const Options& o);
// allow_rebuild = false: use the cached plan as is (capturable; fails if absent)
void count_pivot(Csr& c, const CountArgs& a, hipStream_t s, const Options& o, bool allow_rebuild = true);
void fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);
void count_multi(const std::vector<Csr*>& gs, const std::vector<unsigned long long*>& t_rank, int mode,
                 unsigned long long* T_dev, hipStream_t s, const Options& o);
void count_plain(const Csr& c, unsigned long long* total, hipStream_t s);
// Whether the plain merge serves this graph (TC_OPT_KERNEL 1, or 0 with fewer than 16 probes per edge)
bool plain_is_best(const Csr& c, const Options& o);
// Totals (a.mode kCountTotal), per-node counts (kCountPerNode: a.t_rank) or the triangle list
// (kCountList: a.order, a.tri, a.cursor, a.cap) by the plain merge, with a.total and, when set,
// a.per_graph (by a.graph_of_rank)
void count_plain_mode(const Csr& c, const CountArgs& a, hipStream_t s);
void graph_work(const Csr& c, unsigned long long* W, unsigned long long* P, hipStream_t s);
// sum_v d_v * dhat_v (the objective of Theorem 3); deg by caller id, order rank -> id
void order_cost(const Csr& c, const int32_t* deg, const int32_t* order, unsigned long long* out, hipStream_t s);
// Section 5 partitioning by a cost scheme (0..6) into `parts` id ranges, each
// counted by one workgroup; bounds int64[parts+1], work uint64[parts] (merge cost)
void count_partitioned(const Csr& c, const int32_t* order, const int32_t* rank, const int32_t* deg, int scheme,
                       int32_t parts, unsigned long long* T_dev, int64_t* bounds, unsigned long long* work,
                       hipStream_t s);
// coreness of every rank of the CSR (neighbours: out-entries and in-edge records; needs the plan)
void coreness_rank(const Csr& c, hipStream_t s, int32_t* core);
// keeps each edge with probability q (Section 7); rows of ranks below first_rank are left empty
// stream.hip: exact T of a rank-space oriented CSR held in host memory, streamed
// through the device under a memory budget; info: {partitions, chunks, pairs, bytes copied in}
uint64_t count_streamed(const int64_t* off, const int32_t* adj, int32_t n, int64_t m, uint64_t budget,
                        hipStream_t s, const Options& o, uint64_t info[4]);
// dhat_host (pinned host word, optional): the sample's dhat_max is copied there for the
// caller to read after its next synchronisation, instead of being read here
void build_sampled_csr(const tc_graph* g, double q, uint64_t seed, Csr& out, hipStream_t s, int32_t first_rank = 0,
                       uint64_t* dhat_host = nullptr);
void sort_triangles(int32_t* tri, int64_t count, int bits, hipStream_t s);
// off[r] = first index whose row is >= r, for rows sorted ascending (length m); off has n+1 entries
void offsets_from_rows(const int32_t* row, uint64_t m, int32_t n, int64_t* off, hipStream_t s);
// Same, for keys sorted by their high 32 bits (the row).
void offsets_from_key_rows(const uint64_t* keys, uint64_t m, int32_t n, int64_t* off, hipStream_t s);
// largest off[r+1]-off[r] (0 if n == 0); synchronises s
int32_t max_row_length(const int64_t* off, int32_t n, hipStream_t s);

}  // namespace tc
