// Intersection kernels of NodeIteratorN on MI355X.
//
// The graph is an oriented CSR in rank space (ranks follow the degree order of
// Eq. (1)), so for an oriented edge (v,u) every w of N_v ∩ N_u satisfies
// u < w, and the intersection equals A ∩ N_u with A the part of N_v after u.
//
//  * count_plain: the intersection exactly as the NodeIteratorN figure states
//    it (one thread per oriented edge, two-pointer merge of the full N_v and
//    N_u straight from HBM). Kept as the in-binary baseline.
//
//  * count_pivot: the same |N_v ∩ N_u| terms grouped by the middle vertex u
//    (the "pivot"): N_u is staged once in an LDS hash table and the suffix A
//    of each in-edge (v,u) is streamed through it. Work items come from a
//    cost prefix sum and the boundary rule of Section 5 (load balancing),
//    with per-item cost |A| plus fixed overheads, instead of per-processor
//    partitions. Large lists are staged by whole blocks, small ones by single
//    waves. Per-node counts accumulate in LDS beside the table and leave with
//    one atomic per (pivot, w).
#include <cmath>

#include "graph.hpp"
#include "pivot_kernel.hpp"
#include "primitives.hpp"

namespace tc {

namespace {

constexpr int kBlock = 256;
constexpr int kCostPerRecord = 4;        // fixed probe-equivalents per in-edge record
constexpr int kCostPerStaged = 2;        // probe-equivalents per staged list entry

// ------------------------------------------------------------- plain ---

__global__ __launch_bounds__(kBlock) void k_count_plain(const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                         const int32_t* __restrict__ src, uint64_t m,
                                                         unsigned long long* __restrict__ total) {
  unsigned long long cnt = 0;
  for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    // N_u holds only ranks above u, and u sits at entry e of the ascending row v,
    // so only the suffix of N_v after e can meet N_u
    const int32_t v = src[e], u = adj[e];
    int64_t i = static_cast<int64_t>(e) + 1, ie = off[v + 1], j = off[u], je = off[u + 1];
    while (i < ie && j < je) {
      const int32_t a = adj[i], b = adj[j];
      cnt += (a == b);
      i += (a <= b);
      j += (b <= a);
    }
  }
  cnt = wave_sum(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(total, cnt);
}

// dst[key] += val summed over each run of equal keys among the lanes of a wave
// (keys ascend with the lane; lanes with valid false take no part): one atomic
// per run, by its last lane, instead of one per lane on the same address.
__device__ __forceinline__ void run_add(unsigned long long* dst, int32_t key, unsigned long long val, bool valid) {
  const int lane = lane_id();
  const int32_t k = valid ? key : -1;
  unsigned long long x = valid ? val : 0ull;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d, kWave);
    const int32_t ky = __shfl_up(k, d, kWave);
    if (lane >= d && ky == k) x += y;  // keys ascend: an equal key d lanes back means one run
  }
  const int32_t next = __shfl_down(k, 1, kWave);
  const bool last = lane == kWave - 1 || next != k;
  if (valid && last && x) atomicAdd(&dst[k], x);
}

// The same merge for totals per graph of a batch (MODE kCountTotal), per-node
// counts (kCountPerNode) or the triangle list (kCountList): every w in
// N_v ∩ N_u adds one to t_w and, once per edge, the edge's matches to t_v and
// t_u (rank space); or the triangle goes to tri as caller ids, ascending, at a
// slot taken from the cursor (slots past cap are dropped, the cursor still
// counts them). With per_graph, each edge's matches also go to the total of
// the graph its source belongs to (graph_of_rank, or graph 0). The lanes of a
// wave take consecutive edges, so their sources (and graphs) ascend and the
// additions to t_v and to the graph totals are summed over runs first.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_plain_mode(const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                       const int32_t* __restrict__ src, uint64_t m,
                                                       unsigned long long* __restrict__ total,
                                                       unsigned long long* __restrict__ t_rank,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ tri,
                                                       unsigned long long* __restrict__ cursor, int64_t cap,
                                                       unsigned long long* __restrict__ per_graph,
                                                       const int32_t* __restrict__ graph_of_rank) {
  unsigned long long cnt = 0;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * blockDim.x; base < m;
       base += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t e = base + threadIdx.x;
    const bool valid = e < m;  // every lane of the wave runs the same iterations
    int32_t v = 0;
    unsigned long long here = 0;
    if (valid) {
      v = src[e];
      const int32_t u = adj[e];
      int64_t i = static_cast<int64_t>(e) + 1, ie = off[v + 1], j = off[u], je = off[u + 1];
      while (i < ie && j < je) {
        const int32_t a = adj[i], b = adj[j];
        if (a == b) {
          here++;
          if (MODE == kCountPerNode) {
            atomicAdd(&t_rank[a], 1ull);
          } else if (MODE == kCountList) {
            int32_t x = order[v], y = order[u], z = order[a], t;
            if (x > y) { t = x; x = y; y = t; }
            if (y > z) { t = y; y = z; z = t; }
            if (x > y) { t = x; x = y; y = t; }
            const unsigned long long pos = atomicAdd(cursor, 1ull);
            if (static_cast<int64_t>(pos) < cap) {
              tri[3 * pos + 0] = x;
              tri[3 * pos + 1] = y;
              tri[3 * pos + 2] = z;
            }
          }
        }
        i += (a <= b);
        j += (b <= a);
      }
      if (MODE == kCountPerNode && here) atomicAdd(&t_rank[u], here);
    }
    if (MODE == kCountPerNode) run_add(t_rank, v, here, valid);
    if (per_graph) run_add(per_graph, valid && graph_of_rank ? graph_of_rank[v] : 0, here, valid);
    cnt += here;
  }
  cnt = wave_sum(cnt);
  if (lane_id() == 0 && cnt && total) atomicAdd(total, cnt);
}

// W = sum_e (dhat_v + dhat_u) and P = sum_v C(dhat_v, 2)
__global__ __launch_bounds__(kBlock) void k_work(const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                  const int32_t* __restrict__ src, uint64_t m,
                                                  unsigned long long* __restrict__ W, unsigned long long* __restrict__ P) {
  unsigned long long w = 0, p = 0;
  for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const int32_t v = src[e], u = adj[e];
    const int64_t rv = off[v + 1];
    w += static_cast<unsigned long long>((rv - off[v]) + (off[u + 1] - off[u]));
    p += static_cast<unsigned long long>(rv - static_cast<int64_t>(e) - 1);
  }
  w = wave_sum(w);
  p = wave_sum(p);
  if (lane_id() == 0) {
    if (W) atomicAdd(W, w);
    if (P) atomicAdd(P, p);
  }
}

// -------------------------------------------------------- plan building ---

// The in-edge record of oriented edge e = e0 + i, (v, u) with u = adj[e], as
// the first pass of its sort reads it: key (u << 32) | e, value the length of
// the suffix of N_v after u, off[v + 1] - e - 1. Pivots with an empty N_u and
// records with an empty suffix stay in the list; they are given no work.
struct InEdgeSource {
  using Key = uint64_t;
  static constexpr bool kArrays = false;
  static constexpr int kHistShift = 32;  // the digits are those of u = adj[e]: counted from adj itself
  const int64_t* __restrict__ off;
  const int32_t* __restrict__ adj;
  const int32_t* __restrict__ src;
  uint64_t e0;
  __device__ __forceinline__ uint64_t key(size_t i) const {
    const uint64_t e = e0 + i;
    return (static_cast<uint64_t>(static_cast<uint32_t>(adj[e])) << 32) | e;
  }
  __device__ __forceinline__ uint32_t val(size_t i) const {
    const uint64_t e = e0 + i;
    return static_cast<uint32_t>(off[src[e] + 1] - static_cast<int64_t>(e) - 1);
  }
  ArraySource<uint32_t, NoVal> hist() const {
    return ArraySource<uint32_t, NoVal>{reinterpret_cast<const uint32_t*>(adj + e0), nullptr};
  }
};

// The last pass of the record sort writes each record in its final form:
// suffix start e + 1 (e from the key's low word) and suffix length, and the
// length alone to lens (for the cost prefix).
struct RecordSink {
  InRec* __restrict__ rec;
  uint32_t* __restrict__ lens;
  __device__ __forceinline__ void put(size_t g, uint64_t key, uint32_t len) const {
    rec[g] = InRec{static_cast<uint32_t>(key) + 1u, len};
    lens[g] = len;
  }
};

// Records in pivot order from the sorted keys and their suffix lengths (taken
// from the CSR when lens is null).
__global__ __launch_bounds__(kBlock) void k_inrec_fill(const uint64_t* __restrict__ ikeys,
                                                       const uint32_t* __restrict__ lens,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ src, uint64_t mi,
                                                       InRec* __restrict__ rec) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < mi;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t e = static_cast<uint32_t>(ikeys[i] & 0xffffffffu);
    const uint32_t len = lens ? lens[i] : static_cast<uint32_t>(off[src[e] + 1] - static_cast<int64_t>(e) - 1);
    rec[i] = InRec{e + 1, len};
  }
}

// Cost of record i, |A| + kCostPerRecord, from the sorted suffix lengths or the records.
struct LenCost {
  const uint32_t* lens;
  __device__ int64_t operator()(size_t i) const { return static_cast<int64_t>(lens[i]) + kCostPerRecord; }
};
struct RecCost {
  const InRec* rec;
  __device__ int64_t operator()(size_t i) const { return static_cast<int64_t>(rec[i].a_len) + kCostPerRecord; }
};

__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Target probe-equivalents of a wave item: the item_work option, else about 8
// items per resident wave from the plan's total cost, within [4096, 65536];
// never below 64. Block items take 8 times as much. Read on the device from
// the cost total, so the plan needs no readback before it classifies.
struct ItemWidth {
  const int64_t* total;  // the cost prefix's total
  int64_t option;        // TC_OPT_ITEM_WORK (0: from the total)
  int64_t waves;         // resident waves of the persistent launch
  __device__ int64_t wave() const {
    int64_t w = option;
    if (w <= 0) {
      w = *total / (8 * waves);
      w = w < 4096 ? 4096 : w > 65536 ? 65536 : w;
    }
    return w < 64 ? 64 : w;
  }
};

// Per pivot: number of block items, number of split wave items, and whether it
// is served from the grouped queue.
__global__ void k_pivot_classify(int32_t n, const int64_t* __restrict__ off, const int64_t* __restrict__ in_off,
                                 const int64_t* __restrict__ fin, int64_t hub_dhat, int64_t hub_cap, ItemWidth width,
                                 int64_t* __restrict__ n_hub, int64_t* __restrict__ n_split,
                                 int32_t* __restrict__ grouped, unsigned long long* __restrict__ probes) {
  const int64_t iw_wave = width.wave(), iw_hub = 8 * iw_wave;
  unsigned long long pr = 0;
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const int64_t dh = off[u + 1] - off[u];
    const int64_t i0 = in_off[u], i1 = in_off[u + 1];
    const int64_t cost = fin[i1] - fin[i0];
    const int64_t work = cost - kCostPerRecord * (i1 - i0);  // sum of the suffix lengths
    int64_t h = 0, sp = 0;
    int32_t gr = 0;
    if (dh > 0 && work > 0) {
      pr += static_cast<unsigned long long>(work);
      if (dh > hub_dhat) {
        h = ceil_div(dh, hub_cap) * ceil_div(cost, iw_hub);
      } else if (cost + kCostPerStaged * dh > iw_wave) {
        sp = ceil_div(cost, iw_wave);
      } else {
        gr = 1;
      }
    }
    n_hub[u] = h;
    n_split[u] = sp;
    grouped[u] = gr;
  }
  pr = wave_sum(pr);
  if (lane_id() == 0 && pr) atomicAdd(probes, pr);
}

// First in-edge index in [i0,i1] whose cost prefix reaches target (boundary
// rule: x_j is the first position with F >= j * alpha).
__device__ __forceinline__ int64_t boundary(const int64_t* fin, int64_t i0, int64_t i1, int64_t target) {
  int64_t lo = i0, hi = i1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (fin[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_items_fill(uint64_t n_items, const int64_t* __restrict__ item_off, int32_t n,
                             const int64_t* __restrict__ off, const int64_t* __restrict__ in_off,
                             const int64_t* __restrict__ fin, int64_t cap, ItemWidth width, int64_t scale,
                             PivotItem* __restrict__ items) {
  const int64_t iw = scale * width.wave();
  for (uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n_items;
       t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    // pivot: largest u with item_off[u] <= t (item_off holds n+1 exclusive offsets)
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int32_t mid = static_cast<int32_t>((static_cast<int64_t>(lo) + hi + 1) >> 1);
      if (item_off[mid] <= static_cast<int64_t>(t)) lo = mid;
      else hi = mid - 1;
    }
    const int32_t u = lo;
    const int64_t dh = off[u + 1] - off[u];
    const int64_t i0 = in_off[u], i1 = in_off[u + 1];
    const int64_t f0 = fin[i0], tot = fin[i1] - f0;
    const int64_t pieces = ceil_div(tot, iw);
    const int64_t local = static_cast<int64_t>(t) - item_off[u];
    const int64_t c = local / pieces, j = local % pieces;
    const int64_t b0 = j == 0 ? i0 : boundary(fin, i0, i1, f0 + (tot * j) / pieces);
    const int64_t b1 = j + 1 == pieces ? i1 : boundary(fin, i0, i1, f0 + (tot * (j + 1)) / pieces);
    const int64_t nb = c * cap;
    const int64_t nl = dh - nb < cap ? dh - nb : cap;
    items[t] = PivotItem{u, static_cast<uint32_t>(b0), static_cast<uint32_t>(b1), static_cast<uint32_t>(nb),
                         static_cast<uint32_t>(nl), 0u};
  }
}

struct GroupedPred {
  const int32_t* flag;
  __device__ bool operator()(size_t u) const { return flag[u] != 0; }
};
struct IdentityI32 {
  __device__ int32_t operator()(size_t u) const { return static_cast<int32_t>(u); }
};


__global__ void k_int32_from_u64_hi(const uint64_t* __restrict__ k, uint64_t n, int32_t* __restrict__ out) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<int32_t>(k[i] >> 32);
}

}  // namespace

// Hub items stage at most this many list entries at once (the slice size): at
// the default two entries per 4-slot bucket the table has 1024 buckets, 20 KiB
// of LDS for totals and 36 KiB with the per-node tallies.
static int64_t hub_slice_cap(int) { return 2048; }

static int device_cus() {
  int dev = 0, cus = 0;
  TC_HIP(hipGetDevice(&dev));
  TC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus > 0 ? cus : 1;
}

void count_plain(const Csr& c, unsigned long long* total, hipStream_t s) {
  if (c.m == 0) return;
  const unsigned grid = grid_for(static_cast<uint64_t>(c.m), kBlock, static_cast<unsigned>(device_cus()) * 64u);
  k_count_plain<<<grid, kBlock, 0, s>>>(c.off.p, c.adj.p, c.src.p, static_cast<uint64_t>(c.m), total);
  TC_LAUNCH_CHECK();
}

bool plain_is_best(const Csr& c, const Options& o) {
  // graphs with few wedge checks per edge (near-uniform low degrees), where the persistent
  // pivot kernel's staging costs more than the merge work
  return o.kernel == 1 || (o.kernel == 0 && c.plan.ready && c.plan.probes < 16ull * static_cast<uint64_t>(c.m));
}

void count_plain_mode(const Csr& c, const CountArgs& a, hipStream_t s) {
  if (c.m == 0) return;
  const unsigned grid = grid_for(static_cast<uint64_t>(c.m), kBlock, static_cast<unsigned>(device_cus()) * 64u);
  const uint64_t m = static_cast<uint64_t>(c.m);
  if (a.mode == kCountPerNode)
    k_plain_mode<kCountPerNode><<<grid, kBlock, 0, s>>>(c.off.p, c.adj.p, c.src.p, m, a.total, a.t_rank, nullptr,
                                                        nullptr, nullptr, 0, a.per_graph, a.graph_of_rank);
  else if (a.mode == kCountList)
    k_plain_mode<kCountList><<<grid, kBlock, 0, s>>>(c.off.p, c.adj.p, c.src.p, m, a.total, nullptr, a.order, a.tri,
                                                     a.cursor, a.cap, a.per_graph, a.graph_of_rank);
  else
    k_plain_mode<kCountTotal><<<grid, kBlock, 0, s>>>(c.off.p, c.adj.p, c.src.p, m, a.total, nullptr, nullptr, nullptr,
                                                      nullptr, 0, a.per_graph, a.graph_of_rank);
  TC_LAUNCH_CHECK();
}

void graph_work(const Csr& c, unsigned long long* W, unsigned long long* P, hipStream_t s) {
  if (c.m == 0) return;
  k_work<<<grid_for(static_cast<uint64_t>(c.m), kBlock, 16384), kBlock, 0, s>>>(c.off.p, c.adj.p, c.src.p,
                                                                                 static_cast<uint64_t>(c.m), W, P);
  TC_LAUNCH_CHECK();
}

namespace {
__global__ void k_order_cost(const int64_t* __restrict__ off, const int32_t* __restrict__ deg,
                             const int32_t* __restrict__ order, int32_t n, unsigned long long* __restrict__ out) {
  unsigned long long acc = 0;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    acc += static_cast<unsigned long long>(off[r + 1] - off[r]) * static_cast<unsigned long long>(deg[order[r]]);
  acc = wave_sum(acc);
  if (lane_id() == 0 && acc) atomicAdd(out, acc);
}
}  // namespace

void order_cost(const Csr& c, const int32_t* deg, const int32_t* order, unsigned long long* out, hipStream_t s) {
  if (c.n == 0) return;
  k_order_cost<<<grid_for(c.n, kBlock, 16384), kBlock, 0, s>>>(c.off.p, deg, order, c.n, out);
  TC_LAUNCH_CHECK();
}

// Builds the in-edge records and the work items of the pivot kernels. The
// plan depends on hub_dhat and item_work and is rebuilt when they change.
// The item lists are built for the per-node slice cap (2048 entries, see
// hub_slice_cap), which also serves the total-only mode.
static int64_t clamp_hub(int64_t h) { return h < 0 ? 0 : (h > kWaveSlots / 2 ? kWaveSlots / 2 : h); }

namespace {

// The records of the oriented edges at CSR entries [e0, e1) grouped by pivot,
// and the work items over them.
void build_plan(Csr& c, PivotPlan& P, uint64_t e0, uint64_t e1, hipStream_t s, const Options& o) {
  P.reset();
  const int32_t n = c.n;
  const uint64_t mi = e1 - e0;
  P.in_off.alloc(static_cast<size_t>(n) + 1, s);
  if (mi == 0 || n == 0) {
    if (n >= 0) TC_HIP(hipMemsetAsync(P.in_off.p, 0, (static_cast<size_t>(n) + 1) * sizeof(int64_t), s));
    P.hub_dhat = clamp_hub(o.hub_dhat);
    P.item_work = o.item_work;
    P.ready = true;
    return;
  }
  const int b = bits_for(n > 1 ? static_cast<uint64_t>(n - 1) : 1);
  // in-edge records sorted by pivot u (stable: by e within u)
  DevBuf<uint64_t> ik(mi, s), ik2(mi, s);
  DevBuf<uint32_t> il(mi, s), il2(mi, s);
  uint32_t* sl = il.get();
  DevBuf<uint32_t> sort_fail(1, s);
  TC_HIP(hipMemsetAsync(sort_fail.get(), 0, sizeof(uint32_t), s));
  // the records are read from the CSR by the sort's first pass and written in
  // their final form by its last (with one record no pass runs: the record is
  // then made from the key and value)
  const bool filled = mi > 1;
  if (filled) P.inrec.alloc(mi, s);
  // the value buffer the last pass would write (passes alternate from vtmp), free for the lengths
  uint32_t* lens_out = (((b + kRadixBits - 1) / kRadixBits) & 1) ? il2.get() : il.get();
  const RecordSink recs{P.inrec.p, lens_out};
  uint64_t* sk = radix_sort_from<uint64_t, uint32_t, InEdgeSource, NoHook, RecordSink>(
      InEdgeSource{c.off.p, c.adj.p, c.src.p, e0}, ik.get(), ik2.get(), sl, il2.get(), mi, 32, 32 + b, s,
      sort_fail.get(), NoHook(), filled ? &recs : nullptr);
  DevBuf<int64_t> fin;
  plan_records(c, P, sk, filled ? lens_out : sl, mi, fin, s, filled);
  ik.release();
  ik2.release();
  il.release();
  il2.release();
  plan_items(c, P, fin.get(), mi, s, o, sort_fail.get());
}

}  // namespace

void plan_records(Csr& c, PivotPlan& P, const uint64_t* sk, const uint32_t* sl, uint64_t mi, DevBuf<int64_t>& fin,
                  hipStream_t s, bool filled) {
  const int32_t n = c.n;
  if (!P.in_off.p) P.in_off.alloc(static_cast<size_t>(n) + 1, s);
  fin.alloc(mi + 1, s);
  if (!filled) {
    P.inrec.alloc(mi, s);
    k_inrec_fill<<<grid_for(mi, kBlock, 65536), kBlock, 0, s>>>(sk, sl, c.off.p, c.src.p, mi, P.inrec.p);
    TC_LAUNCH_CHECK();
  }
  offsets_from_key_rows(sk, mi, n, P.in_off.p, s);
  // the cost prefix F over the records (the boundary rule of Section 5 cuts items from it)
  if (sl) exclusive_scan_of<int64_t>(LenCost{sl}, fin.get(), mi, s, fin.get() + mi);
  else exclusive_scan_of<int64_t>(RecCost{P.inrec.p}, fin.get(), mi, s, fin.get() + mi);
}

void plan_items(Csr& c, PivotPlan& P, const int64_t* fin_p, uint64_t mi, hipStream_t s, const Options& o,
                const uint32_t* sort_fail) {
  const int32_t n = c.n;
  const int64_t cap = hub_slice_cap(kCountPerNode);
  const ItemWidth width{fin_p + mi, o.item_work, static_cast<int64_t>(device_cus()) * 4 * kPivotWaves};
  // control words, read back in one copy: [0] block items, [1] wave items, [2] probes,
  // [3] grouped pivots, [4] a sort's look-back gave up
  DevBuf<uint64_t> ctl(5, s);
  k_fill_words<uint64_t><<<1, 64, 0, s>>>(ctl.get(), 5, 0ull);
  TC_LAUNCH_CHECK();
  DevBuf<int64_t> nh(n, s), ns(n, s);
  DevBuf<int32_t> grp(n, s), glist(n, s);
  k_pivot_classify<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(
      n, c.off.p, P.in_off.p, fin_p, clamp_hub(o.hub_dhat), cap, width, nh.get(), ns.get(), grp.get(),
      reinterpret_cast<unsigned long long*>(ctl.get() + 2));
  TC_LAUNCH_CHECK();
  exclusive_scan<int64_t>(nh.get(), nh.get(), n, s, reinterpret_cast<int64_t*>(ctl.get()));
  exclusive_scan<int64_t>(ns.get(), ns.get(), n, s, reinterpret_cast<int64_t*>(ctl.get() + 1));
  compact_if<int32_t>(n, GroupedPred{grp.get()}, IdentityI32{}, glist.get(), ctl.get() + 3, s);
  if (sort_fail) {
    TC_HIP(hipMemcpyAsync(ctl.get() + 4, sort_fail, sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
  HostWords hw(s);
  TC_HIP(hipMemcpyAsync(hw.get(), ctl.get(), 5 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (hw[4]) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  P.n_hub_items = hw[0];
  P.n_wave_items = hw[1];
  P.probes = hw[2];
  const uint64_t ng = hw[3];
  // items: [hub items | split wave items]; the grouped pivots as int32 in a list of their own
  P.items.alloc(P.n_hub_items + P.n_wave_items, s);
  if (P.n_hub_items) {
    k_items_fill<<<grid_for(P.n_hub_items, kBlock, 65536), kBlock, 0, s>>>(P.n_hub_items, nh.get(), n, c.off.p,
                                                                          P.in_off.p, fin_p, cap, width, 8, P.items.p);
    TC_LAUNCH_CHECK();
  }
  if (P.n_wave_items) {
    k_items_fill<<<grid_for(P.n_wave_items, kBlock, 65536), kBlock, 0, s>>>(
        P.n_wave_items, ns.get(), n, c.off.p, P.in_off.p, fin_p, 1ll << 40, width, 1, P.items.p + P.n_hub_items);
    TC_LAUNCH_CHECK();
  }
  P.grouped.alloc(ng, s);
  if (ng) TC_HIP(hipMemcpyAsync(P.grouped.p, glist.get(), ng * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  P.n_grouped = ng;
  P.hub_dhat = clamp_hub(o.hub_dhat);
  P.item_work = o.item_work;
  P.ready = true;
}

namespace {

bool plan_matches(const PivotPlan& P, int32_t lo, int32_t hi, const Options& o) {
  return P.ready && P.src_lo == lo && P.src_hi == hi && P.hub_dhat == clamp_hub(o.hub_dhat) &&
         P.item_work == o.item_work;
}

}  // namespace

void note_plan_use(PivotPlan& P, hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  TC_HIP(hipStreamIsCapturing(s, &st));
  if (st != hipStreamCaptureStatusNone) P.frozen = true;
  else P.users.record(s);
}

void ensure_plan(Csr& c, hipStream_t s, const Options& o) {
  PivotPlan& P = c.plan;
  if (P.frozen || plan_matches(P, 0, c.n, o)) return;  // a frozen plan serves every option set
  if (P.ready) P.release_on(s);  // after every launch that read the old plan
  build_plan(c, P, 0, static_cast<uint64_t>(c.m), s, o);
  P.src_lo = 0;
  P.src_hi = c.n;
}

void rebuild_plan(Csr& c, hipStream_t s, const Options& o) {
  PivotPlan& P = c.plan;
  if (P.frozen) fail(TC_E_INVAL, "the work plan is held by a captured HIP graph and cannot be rebuilt");
  if (P.ready) P.release_on(s);
  build_plan(c, P, 0, static_cast<uint64_t>(c.m), s, o);
  P.src_lo = 0;
  P.src_hi = c.n;
}

void ensure_shard_plan(Csr& c, int32_t lo, int32_t hi, hipStream_t s, const Options& o) {
  if (lo < 0 || hi > c.n || lo > hi) fail(TC_E_RANGE, "shard rank range outside [0, n]");
  PivotPlan& P = c.shard;
  if (plan_matches(P, lo, hi, o)) return;
  if (P.ready) P.release_on(s);
  int64_t e[2] = {0, 0};
  if (c.n > 0) {
    TC_HIP(hipMemcpyAsync(&e[0], c.off.p + lo, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&e[1], c.off.p + hi, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
  }
  build_plan(c, P, static_cast<uint64_t>(e[0]), static_cast<uint64_t>(e[1]), s, o);
  P.src_lo = lo;
  P.src_hi = hi;
}

namespace {
__global__ void k_fill_u64(unsigned long long* __restrict__ p, size_t n, unsigned long long v) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}
}  // namespace

// A fill kernel rather than hipMemsetAsync so that captured graphs hold no memset node.
// ---------------------------------------------------------------- coreness
//
// The k-core order of Section 4: the coreness of v is the largest k such that
// v lies in a subgraph whose vertices all have degree >= k. Level-synchronous
// peeling in rank space: at level k every live vertex with remaining degree
// <= k is removed with coreness k, its live neighbours lose one degree each,
// and a neighbour whose remaining degree falls from k+1 to k joins the next
// round of the same level. A level starts at the smallest remaining degree.

__global__ void k_core_init(const int64_t* __restrict__ off, const int64_t* __restrict__ in_off, int32_t n,
                            int32_t* __restrict__ cd, int32_t* __restrict__ core) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    cd[r] = static_cast<int32_t>((off[r + 1] - off[r]) + (in_off[r + 1] - in_off[r]));
    core[r] = -1;
  }
}

__global__ void k_core_min(const int32_t* __restrict__ cd, const int32_t* __restrict__ core, int32_t n,
                           int32_t* __restrict__ out) {
  int32_t best = INT32_MAX;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    if (core[r] < 0 && cd[r] < best) best = cd[r];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const int32_t o = __shfl_xor(best, d, kWave);
    best = o < best ? o : best;
  }
  if (lane_id() == 0 && best != INT32_MAX) atomicMin(out, best);
}

struct CoreFrontierPred {
  const int32_t* cd;
  const int32_t* core;
  int32_t k;
  __device__ bool operator()(size_t r) const { return core[r] < 0 && cd[r] <= k; }
};
struct IndexI32 {
  __device__ int32_t operator()(size_t r) const { return static_cast<int32_t>(r); }
};

__global__ void k_core_mark(const int32_t* __restrict__ f, uint32_t nf, int32_t k, int32_t* __restrict__ core) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) core[f[i]] = k;
}

// One wave per removed vertex: its out-entries and in-edge records name its neighbours.
__global__ __launch_bounds__(kBlock) void k_core_peel(const int32_t* __restrict__ f, uint32_t nf, int32_t k,
                                                      const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                      const int64_t* __restrict__ in_off,
                                                      const InRec* __restrict__ rec, const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ core, int32_t* __restrict__ cd,
                                                      int32_t* __restrict__ next, uint32_t* __restrict__ n_next) {
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  auto drop = [&](int32_t w) {
    if (core[w] >= 0) return;  // already removed (this round's vertices are marked before the round)
    const int32_t old = atomicSub(&cd[w], 1);
    if (old == k + 1) next[atomicAdd(n_next, 1u)] = w;
  };
  for (uint32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < nf; i += waves) {
    const int32_t r = f[i];
    for (int64_t j = off[r] + lane; j < off[r + 1]; j += kWave) drop(adj[j]);
    for (int64_t j = in_off[r] + lane; j < in_off[r + 1]; j += kWave) drop(src[rec[j].a_begin - 1]);
  }
}

void coreness_rank(const Csr& c, hipStream_t s, int32_t* core) {
  const int32_t n = c.n;
  if (n <= 0) return;
  if (!c.plan.ready) fail(TC_E_INVAL, "coreness needs the work plan");
  const PivotPlan& P = c.plan;
  DevBuf<int32_t> cd(n, s), fa(n, s), fb(n, s), dmin(1, s);
  DevBuf<uint32_t> dnext(1, s);
  DevBuf<uint64_t> dcnt(1, s);
  k_core_init<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(c.off.p, P.in_off.p, n, cd.get(), core);
  TC_LAUNCH_CHECK();
  int64_t alive = n;
  int32_t k = 0;
  int32_t* f = fa.get();
  int32_t* g = fb.get();
  while (alive > 0) {
    k_fill_words<int32_t><<<1, 64, 0, s>>>(dmin.get(), 1, INT32_MAX);
    TC_LAUNCH_CHECK();
    k_core_min<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(cd.get(), core, n, dmin.get());
    TC_LAUNCH_CHECK();
    int32_t lo = 0;
    TC_HIP(hipMemcpyAsync(&lo, dmin.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (lo == INT32_MAX) fail(TC_E_DEVICE, "coreness: live vertices without a degree");
    if (lo > k) k = lo;
    compact_if<int32_t>(static_cast<size_t>(n), CoreFrontierPred{cd.get(), core, k}, IndexI32{}, f, dcnt.get(), s);
    uint64_t nf = 0;
    TC_HIP(hipMemcpyAsync(&nf, dcnt.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (nf == 0) fail(TC_E_DEVICE, "coreness: empty level");
    while (nf > 0) {
      const uint32_t nfu = static_cast<uint32_t>(nf);
      k_core_mark<<<grid_for(nf, kBlock, 65536), kBlock, 0, s>>>(f, nfu, k, core);
      TC_LAUNCH_CHECK();
      alive -= static_cast<int64_t>(nf);
      k_fill_words<uint32_t><<<1, 64, 0, s>>>(dnext.get(), 1, 0u);
      TC_LAUNCH_CHECK();
      k_core_peel<<<grid_for(static_cast<uint64_t>(nf) * kWave, kBlock, 65536), kBlock, 0, s>>>(
          f, nfu, k, c.off.p, c.adj.p, P.in_off.p, P.inrec.p, c.src.p, core, cd.get(), g, dnext.get());
      TC_LAUNCH_CHECK();
      uint32_t nn = 0;
      TC_HIP(hipMemcpyAsync(&nn, dnext.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      nf = nn;
      std::swap(f, g);
    }
  }
}

// ------------------------------------------------- load-balancing schemes
//
// The partitioning of Section 5: core nodes in id order are split into
// contiguous ranges by the boundary rule x_j = argmin F(v) >= j*alpha over
// the prefix F of a cost f (the cost-function table of Section 5; scheme 6 is
// the cost of the space-efficient algorithm of Section 6), and each range is
// counted by one workgroup with the NodeIteratorN merge, so the slowest range
// sets the time.

__global__ void k_vertex_costs(const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                               const int64_t* __restrict__ in_off, const InRec* __restrict__ rec,
                               const int32_t* __restrict__ src, const int32_t* __restrict__ order,
                               const int32_t* __restrict__ deg, int32_t n, int scheme,
                               unsigned long long* __restrict__ f_id, unsigned long long* __restrict__ cost_id) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const unsigned long long dh = static_cast<unsigned long long>(off[r + 1] - off[r]);
    unsigned long long merge = 0, in = 0;
    for (int64_t j = off[r]; j < off[r + 1]; j++) {
      const int32_t u = adj[j];
      merge += dh + static_cast<unsigned long long>(off[u + 1] - off[u]);
    }
    if (scheme == 6) {
      for (int64_t j = in_off[r]; j < in_off[r + 1]; j++) {
        const int32_t u = src[rec[j].a_begin - 1];
        in += dh + static_cast<unsigned long long>(off[u + 1] - off[u]);
      }
    }
    const int32_t v = order[r];
    const unsigned long long d = static_cast<unsigned long long>(deg[v]);
    unsigned long long f;
    switch (scheme) {
      case 0: f = 1; break;
      case 1: f = d; break;
      case 2: f = dh; break;
      case 3: f = d * dh; break;
      case 4: f = dh * dh; break;
      case 5: f = merge; break;
      default: f = in; break;
    }
    f_id[v] = f;
    cost_id[v] = merge;
  }
}

// bounds[j] = first v with F(v) * parts >= j * total (F inclusive; Fx = exclusive prefix).
__global__ void k_part_bounds(const unsigned long long* __restrict__ Fx, const unsigned long long* __restrict__ f,
                              int32_t n, const unsigned long long* __restrict__ total, int32_t parts,
                              int64_t* __restrict__ bounds) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j <= parts; j += gridDim.x * blockDim.x) {
    if (j == 0) { bounds[0] = 0; continue; }
    if (j == parts) { bounds[parts] = n; continue; }
    const unsigned __int128 goal = static_cast<unsigned __int128>(*total) * static_cast<unsigned>(j);
    int32_t lo = 0, hi = n;  // first v in [0, n) with F(v) * parts >= goal, n if none
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      const unsigned __int128 F = static_cast<unsigned __int128>(Fx[mid] + f[mid]) * static_cast<unsigned>(parts);
      if (F >= goal) hi = mid;
      else lo = mid + 1;
    }
    bounds[j] = lo;
  }
}

__global__ void k_part_work(const unsigned long long* __restrict__ Cx, const int64_t* __restrict__ bounds,
                            int32_t parts, unsigned long long* __restrict__ work) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < parts; j += gridDim.x * blockDim.x)
    work[j] = Cx[bounds[j + 1]] - Cx[bounds[j]];
}

// Workgroup j counts the triangles of its core nodes [bounds[j], bounds[j+1])
// (ids): wave w takes every 4th node, its lanes take the node's oriented
// edges and merge the two full lists.
constexpr int kPartBlock = 256;
__global__ __launch_bounds__(kPartBlock) void k_count_parts(const int64_t* __restrict__ off,
                                                            const int32_t* __restrict__ adj,
                                                            const int32_t* __restrict__ rank,
                                                            const int64_t* __restrict__ bounds,
                                                            unsigned long long* __restrict__ total) {
  const int64_t v0 = bounds[blockIdx.x], v1 = bounds[blockIdx.x + 1];
  const int w = threadIdx.x / kWave, lane = lane_id();
  unsigned long long cnt = 0;
  for (int64_t v = v0 + w; v < v1; v += kPartBlock / kWave) {
    const int32_t r = rank[v];
    const int64_t a0 = off[r], a1 = off[r + 1];
    for (int64_t e = a0 + lane; e < a1; e += kWave) {
      const int32_t u = adj[e];
      int64_t i = a0, j = off[u];
      const int64_t j1 = off[u + 1];
      while (i < a1 && j < j1) {
        const int32_t x = adj[i], y = adj[j];
        cnt += x == y;
        i += x <= y;
        j += y <= x;
      }
    }
  }
  cnt = wave_sum(cnt);
  if (lane == 0 && cnt) atomicAdd(total, cnt);
}

void count_partitioned(const Csr& c, const int32_t* order, const int32_t* rank, const int32_t* deg, int scheme,
                       int32_t parts, unsigned long long* T_dev, int64_t* bounds, unsigned long long* work,
                       hipStream_t s) {
  const int32_t n = c.n;
  if (!c.plan.ready) fail(TC_E_INVAL, "no work plan on this graph");
  fill_u64(T_dev, 1, 0ull, s);
  DevBuf<unsigned long long> f(static_cast<size_t>(n) + 1, s), cost(static_cast<size_t>(n) + 1, s);
  DevBuf<unsigned long long> Fx(static_cast<size_t>(n) + 1, s), Cx(static_cast<size_t>(n) + 1, s);
  if (n > 0) {
    k_vertex_costs<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(c.off.p, c.adj.p, c.plan.in_off.p, c.plan.inrec.p,
                                                                 c.src.p, order, deg, n, scheme, f.get(), cost.get());
    TC_LAUNCH_CHECK();
  }
  exclusive_scan<unsigned long long>(f.get(), Fx.get(), static_cast<size_t>(n), s, Fx.get() + n);
  exclusive_scan<unsigned long long>(cost.get(), Cx.get(), static_cast<size_t>(n), s, Cx.get() + n);
  k_part_bounds<<<grid_for(static_cast<uint64_t>(parts) + 1, kBlock, 4096), kBlock, 0, s>>>(Fx.get(), f.get(), n,
                                                                                              Fx.get() + n, parts,
                                                                                              bounds);
  TC_LAUNCH_CHECK();
  k_part_work<<<grid_for(static_cast<uint64_t>(parts), kBlock, 4096), kBlock, 0, s>>>(Cx.get(), bounds, parts, work);
  TC_LAUNCH_CHECK();
  if (n > 0 && c.m > 0) {
    k_count_parts<<<static_cast<unsigned>(parts), kPartBlock, 0, s>>>(c.off.p, c.adj.p, rank, bounds, T_dev);
    TC_LAUNCH_CHECK();
  }
}

void fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return;
  k_fill_u64<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(p, n, v);
  TC_LAUNCH_CHECK();
}

// One persistent launch of k_pivot over the records and items of plan P of c.
void launch_pivot(const Csr& c, PivotPlan& P, const CountArgs& ca, hipStream_t s, const Options& o) {
  KernelArgs a{static_cast<int>(o.hub_bucket_load), c.off.p,     c.adj.p,          c.src.p,   P.inrec.p, P.in_off.p, ca.mode,  ca.total,
               ca.per_graph, ca.graph_of_rank, ca.t_rank, ca.order,  ca.tri,     ca.cursor, ca.cap};
  DevBuf<unsigned long long> qbuf;
  unsigned long long* q = ca.queues;
  if (!q) {
    qbuf.alloc(3, s);
    q = qbuf.get();
  }
  fill_u64(q, 3, 0ull, s);
  const unsigned cus = static_cast<unsigned>(device_cus());
  const unsigned bpc = static_cast<unsigned>(o.blocks_per_cu > 0 ? o.blocks_per_cu : 8);
  const bool per_node = ca.mode == kCountPerNode;
  int hub_log2b = 4;
  if (P.n_hub_items) {
    const int64_t cap = hub_slice_cap(kCountPerNode);
    const int64_t maxlen = c.dhat_max < cap ? c.dhat_max : cap;
    while ((1ll << hub_log2b) * o.hub_bucket_load < maxlen) hub_log2b++;
  }
  const size_t lds = static_cast<size_t>(pivot_region_words(hub_log2b, per_node)) * sizeof(int32_t);
  const uint64_t wave_units = P.n_split_items() + (P.n_grouped + kGroupChunk - 1) / kGroupChunk;
  const uint64_t blocks_needed = P.n_hub_items + (wave_units + kPivotWaves - 1) / kPivotWaves;
  if (blocks_needed == 0) return;
  const uint64_t cap_blocks = static_cast<uint64_t>(cus) * bpc;
  const unsigned grid = static_cast<unsigned>(blocks_needed < cap_blocks ? blocks_needed : cap_blocks);
  const PivotItem* hub = P.items.p;
  const PivotItem* split = P.items.p + P.n_hub_items;
  const JobList none{nullptr, nullptr, 0};
  if (ca.mode == kCountPerNode)
    k_pivot<kCountPerNode, false><<<grid, kPivotBlock, lds, s>>>(a, hub, P.n_hub_items, split, P.n_wave_items,
                                                                 P.grouped.p, P.n_grouped, q, hub_log2b, none);
  else if (ca.mode == kCountList)
    k_pivot<kCountList, false><<<grid, kPivotBlock, lds, s>>>(a, hub, P.n_hub_items, split, P.n_wave_items,
                                                              P.grouped.p, P.n_grouped, q, hub_log2b, none);
  else
    k_pivot<kCountTotal, false><<<grid, kPivotBlock, lds, s>>>(a, hub, P.n_hub_items, split, P.n_wave_items,
                                                               P.grouped.p, P.n_grouped, q, hub_log2b, none);
  TC_LAUNCH_CHECK();
  if (ca.note_use) note_plan_use(P, s);
}

namespace {

// Per-rank shard cost. cost 0: f(v) = sum_{u in N_v} (dhat_v + dhat_u), the
// merge cost of v's oriented edges (Theorem 2) and the DPD row of the
// load-balancing table of Section 5. cost 1: the pivot kernel's own model,
// four times C(dhat_v, 2) + 4 dhat_v (probes and per-record work of v's
// in-edge records) + sum_{u in N_v} dhat_u / 4 (staging the lists they meet).
__global__ void k_rank_shard_costs(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n,
                                   int cost, unsigned long long* __restrict__ f) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const unsigned long long dh = static_cast<unsigned long long>(off[r + 1] - off[r]);
    unsigned long long nb = 0;
    for (int64_t j = off[r]; j < off[r + 1]; j++) nb += static_cast<unsigned long long>(off[adj[j] + 1] - off[adj[j]]);
    f[r] = cost == 0 ? dh * dh + nb : 2 * dh * (dh > 0 ? dh - 1 : 0) + 16 * dh + nb;
  }
}

}  // namespace

void count_pivot(Csr& c, const CountArgs& ca, hipStream_t s, const Options& o, bool allow_rebuild) {
  if (c.m == 0) return;
  if (allow_rebuild) ensure_plan(c, s, o);
  else if (!c.plan.ready) fail(TC_E_INVAL, "no work plan on this graph");
  launch_pivot(c, c.plan, ca, s, o);
}

void shard_bounds(const Csr& c, int32_t k, int cost, int64_t* bounds, hipStream_t s) {
  const int32_t n = c.n;
  DevBuf<unsigned long long> f(static_cast<size_t>(n) + 1, s), Fx(static_cast<size_t>(n) + 1, s);
  if (n > 0) {
    k_rank_shard_costs<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(c.off.p, c.adj.p, n, cost, f.get());
    TC_LAUNCH_CHECK();
  }
  exclusive_scan<unsigned long long>(f.get(), Fx.get(), static_cast<size_t>(n), s, Fx.get() + n);
  k_part_bounds<<<grid_for(static_cast<uint64_t>(k) + 1, kBlock, 4096), kBlock, 0, s>>>(Fx.get(), f.get(), n,
                                                                                          Fx.get() + n, k, bounds);
  TC_LAUNCH_CHECK();
}

void count_shard(Csr& c, int32_t lo, int32_t hi, unsigned long long* total, hipStream_t s, const Options& o) {
  ensure_shard_plan(c, lo, hi, s, o);
  if (c.m == 0 || lo == hi) return;
  CountArgs ca;
  ca.mode = kCountTotal;
  ca.total = total;
  launch_pivot(c, c.shard, ca, s, o);
}

// One launch over the work of several graphs (plans must be ready). mode is
// kCountTotal or kCountPerNode; per-graph totals go to T_dev[g] (zeroed here),
// per-node counts by rank to t_rank[g] (zeroed here, per-node mode only).
void count_multi(const std::vector<Csr*>& gs, const std::vector<unsigned long long*>& t_rank, int mode,
                 unsigned long long* T_dev, hipStream_t s, const Options& o) {
  const int32_t k = static_cast<int32_t>(gs.size());
  if (k == 0) return;
  std::vector<GraphDesc> descs(k);
  std::vector<uint64_t> pre(3 * (static_cast<size_t>(k) + 1), 0);
  int32_t dmax = 0;
  for (int32_t g = 0; g < k; g++) {
    Csr& c = *gs[g];
    if (!c.plan.ready) fail(TC_E_INVAL, "graph without a work plan in a multi-graph count");
    const PivotPlan& P = c.plan;
    descs[g] = GraphDesc{c.off.p, c.adj.p, c.src.p, P.inrec.p, P.in_off.p, P.items.p, P.items.p + P.n_hub_items,
                         P.grouped.p, P.n_grouped, mode == kCountPerNode ? t_rank[g] : nullptr};
    pre[g + 1] = pre[g] + (c.m ? P.n_hub_items : 0);
    pre[(k + 1) + g + 1] = pre[(k + 1) + g] + (c.m ? P.n_wave_items : 0);
    pre[2 * (k + 1) + g + 1] = pre[2 * (k + 1) + g] + (c.m ? (P.n_grouped + kGroupChunk - 1) / kGroupChunk : 0);
    if (P.n_hub_items && c.dhat_max > dmax) dmax = c.dhat_max;
    if (mode == kCountPerNode && c.n > 0) fill_u64(t_rank[g], static_cast<size_t>(c.n), 0ull, s);
  }
  fill_u64(T_dev, static_cast<size_t>(k), 0ull, s);
  const uint64_t n_hub = pre[k], n_split = pre[2 * k + 1], n_chunks = pre[3 * k + 2];
  if (n_hub + n_split + n_chunks == 0) return;
  DevBuf<GraphDesc> d_desc(k, s);
  DevBuf<uint64_t> d_pre(pre.size(), s);
  DevBuf<unsigned long long> q(3, s);
  TC_HIP(hipMemcpyAsync(d_desc.get(), descs.data(), k * sizeof(GraphDesc), hipMemcpyHostToDevice, s));
  TC_HIP(hipMemcpyAsync(d_pre.get(), pre.data(), pre.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  fill_u64(q.get(), 3, 0ull, s);
  const bool per_node = mode == kCountPerNode;
  int hub_log2b = 4;
  const int64_t cap = hub_slice_cap(kCountPerNode);
  const int64_t maxlen = dmax < cap ? dmax : cap;
  while ((1ll << hub_log2b) * o.hub_bucket_load < maxlen) hub_log2b++;
  const size_t lds = static_cast<size_t>(pivot_region_words(hub_log2b, per_node)) * sizeof(int32_t);
  const unsigned cus = static_cast<unsigned>(device_cus());
  const unsigned bpc = static_cast<unsigned>(o.blocks_per_cu > 0 ? o.blocks_per_cu : 4);
  const uint64_t blocks_needed = n_hub + (n_split + n_chunks + kPivotWaves - 1) / kPivotWaves;
  const uint64_t cap_blocks = static_cast<uint64_t>(cus) * bpc;
  const unsigned grid = static_cast<unsigned>(blocks_needed < cap_blocks ? blocks_needed : cap_blocks);
  KernelArgs a{static_cast<int>(o.hub_bucket_load), nullptr, nullptr, nullptr, nullptr, nullptr, mode, nullptr, T_dev,
               nullptr, nullptr, nullptr, nullptr, nullptr, 0};
  const JobList jobs{d_desc.get(), d_pre.get(), k};
  if (per_node)
    k_pivot<kCountPerNode, true><<<grid, kPivotBlock, lds, s>>>(a, nullptr, n_hub, nullptr, n_split, nullptr,
                                                                n_chunks, q.get(), hub_log2b, jobs);
  else
    k_pivot<kCountTotal, true><<<grid, kPivotBlock, lds, s>>>(a, nullptr, n_hub, nullptr, n_split, nullptr, n_chunks,
                                                              q.get(), hub_log2b, jobs);
  TC_LAUNCH_CHECK();
  for (Csr* c : gs) note_plan_use(c->plan, s);
}

// --------------------------------------------------------- sparsified ---

namespace {

__device__ __forceinline__ uint64_t splitmix64_output(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

struct KeepPred {
  const int32_t* adj;
  const int32_t* src;
  const int32_t* order;
  uint64_t key;  // mix(seed ^ domain)
  uint64_t tau;
  bool all;
  uint64_t first;  // entries before this index are dropped
  __device__ bool operator()(size_t e) const {
    if (e < first) return false;
    if (all) return true;
    const uint32_t a = static_cast<uint32_t>(order[src[e]]), b = static_cast<uint32_t>(order[adj[e]]);
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    return splitmix64_output(key ^ ((lo << 32) | hi)) < tau;
  }
};

struct PackEntry {
  const int32_t* adj;
  const int32_t* src;
  __device__ uint64_t operator()(size_t e) const {
    return (static_cast<uint64_t>(static_cast<uint32_t>(src[e])) << 32) | static_cast<uint32_t>(adj[e]);
  }
};

__global__ void k_unpack_entries(const uint64_t* __restrict__ k, uint64_t n, int32_t* __restrict__ adj,
                                 int32_t* __restrict__ src) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    adj[i] = static_cast<int32_t>(k[i] & 0xffffffffu);
    src[i] = static_cast<int32_t>(k[i] >> 32);
  }
}

}  // namespace

void build_sampled_csr(const tc_graph* g, double q, uint64_t seed, Csr& out, hipStream_t s, int32_t first_rank,
                       uint64_t* dhat_host) {
  const Csr& c = g->csr;
  const uint64_t m = static_cast<uint64_t>(c.m);
  const bool all = q >= 1.0;
  const uint64_t tau = all ? ~0ull : static_cast<uint64_t>(std::ldexp(q, 64));
  HostWords hw(s);
  int64_t first = 0;
  if (first_rank > 0 && c.n > 0) {
    if (first_rank > c.n) fail(TC_E_RANGE, "first rank outside [0, n]");
    TC_HIP(hipMemcpyAsync(hw.get(), c.off.p + first_rank, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    first = static_cast<int64_t>(hw[0]);
  }
  KeepPred pred{c.adj.p, c.src.p, g->order.p, 0, tau, all, static_cast<uint64_t>(first)};
  {
    uint64_t z = seed ^ 0x5350415253494659ull;  // domain separation constant ("SPARSIFY")
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    pred.key = z ^ (z >> 31);
  }
  DevBuf<uint64_t> packed(m, s);
  DevBuf<uint64_t> d_cnt(1, s);
  compact_if<uint64_t>(m, pred, PackEntry{c.adj.p, c.src.p}, packed.get(), d_cnt.get(), s);
  TC_HIP(hipMemcpyAsync(hw.get(), d_cnt.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  const uint64_t mk = hw[0];
  out.n = c.n;
  out.m = static_cast<int64_t>(mk);
  out.off.alloc(static_cast<size_t>(c.n) + 1, s);
  out.adj.alloc(mk, s);
  out.src.alloc(mk, s);
  if (mk) {
    k_unpack_entries<<<grid_for(mk, kBlock, 65536), kBlock, 0, s>>>(packed.get(), mk, out.adj.p, out.src.p);
    TC_LAUNCH_CHECK();
  }
  offsets_from_rows(out.src.p, mk, c.n, out.off.p, s);
  if (dhat_host) row_max_to_host(out.off.p, c.n, s, dhat_host);
  else out.dhat_max = max_row_length(out.off.p, c.n, s);
}

// ------------------------------------------------------------ listing ---

namespace {

__global__ void k_pack_tri(const int32_t* __restrict__ tri, int64_t count, int bits, u128* __restrict__ k) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = static_cast<uint32_t>(tri[3 * i]), b = static_cast<uint32_t>(tri[3 * i + 1]),
                   c = static_cast<uint32_t>(tri[3 * i + 2]);
    k[i] = u128{(b << bits) | c, a};
  }
}

__global__ void k_unpack_tri(const u128* __restrict__ k, int64_t count, int bits, int32_t* __restrict__ tri) {
  const uint64_t mask = (1ull << bits) - 1;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const u128 x = k[i];
    tri[3 * i] = static_cast<int32_t>(x.hi);
    tri[3 * i + 1] = static_cast<int32_t>(x.lo >> bits);
    tri[3 * i + 2] = static_cast<int32_t>(x.lo & mask);
  }
}

}  // namespace

void sort_triangles(int32_t* tri, int64_t count, int bits, hipStream_t s) {
  if (count <= 1) return;
  DevBuf<u128> k1(count, s), k2(count, s);
  k_pack_tri<<<grid_for(count, kBlock, 65536), kBlock, 0, s>>>(tri, count, bits, k1.get());
  TC_LAUNCH_CHECK();
  u128* r = radix_sort<u128>(k1.get(), k2.get(), count, 0, 2 * bits, s);
  r = radix_sort<u128>(r, r == k1.get() ? k2.get() : k1.get(), count, 64, 64 + bits, s);
  k_unpack_tri<<<grid_for(count, kBlock, 65536), kBlock, 0, s>>>(r, count, bits, tri);
  TC_LAUNCH_CHECK();
}

}  // namespace tc
