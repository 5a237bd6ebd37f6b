// Device construction of the oriented CSR used by NodeIteratorN.
//
// Steps (the preprocessing of the NodeIteratorN figure, Section 3):
//   1. canonical keys lo<<b|hi per edge record; loops and bad ids flagged
//   2. radix sort + unique -> the simple graph of Section 2 (m edges)
//   3. degrees d_v
//   4. ranks: position of each vertex in the degree order of Eq. (1)
//      (d ascending, ties by id; graphs of a batch kept contiguous)
//   5. relabel every edge to (min rank, max rank) -- the orientation of
//      Eq. (1), because the earlier endpoint has the smaller rank -- and radix
//      sort, which yields every N_v ascending, grouped by row
//   6. CSR offsets, row ids, d_max and dhat_max
#include "graph.hpp"
#include "primitives.hpp"

namespace tc {

namespace {

constexpr int kBlock = 256;

__global__ void k_canon(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, uint32_t E, int32_t n,
                        int b, const int64_t* __restrict__ edge_off, const int32_t* __restrict__ vbase, int32_t G,
                        uint64_t* __restrict__ keys, int* __restrict__ err) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < E; i += gridDim.x * blockDim.x) {
    int64_t a = src[i], c = dst[i];
    int64_t base = 0, lim = n;
    if (edge_off) {
      int32_t lo = 0, hi = G - 1;  // graph g with edge_off[g] <= i < edge_off[g+1]
      while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (edge_off[mid] <= static_cast<int64_t>(i)) lo = mid;
        else hi = mid - 1;
      }
      base = vbase[lo];
      lim = static_cast<int64_t>(vbase[lo + 1]) - vbase[lo];
    }
    if (a < 0 || a >= lim || c < 0 || c >= lim) {
      atomicOr(err, 1);
      keys[i] = ~0ull;
      continue;
    }
    if (a == c) {
      keys[i] = ~0ull;
      continue;
    }
    a += base;
    c += base;
    const uint64_t lo = static_cast<uint64_t>(a < c ? a : c), hi = static_cast<uint64_t>(a < c ? c : a);
    keys[i] = (lo << b) | hi;
  }
}

struct UniquePred {
  const uint64_t* k;
  __device__ bool operator()(size_t i) const { return k[i] != ~0ull && (i == 0 || k[i] != k[i - 1]); }
};

struct GatherU64 {
  const uint64_t* k;
  __device__ uint64_t operator()(size_t i) const { return k[i]; }
};

// Endpoint accessors over the sorted unique keys (smaller endpoint) and over
// the sorted larger endpoints.
struct LoEnd {
  const uint64_t* k;
  int b;
  __device__ int32_t operator()(size_t i) const { return static_cast<int32_t>(k[i] >> b); }
};
struct HiEnd {
  const uint32_t* h;
  __device__ int32_t operator()(size_t i) const { return static_cast<int32_t>(h[i]); }
};

// deg[v] += number of positions i in [0, m) with get(i) == v, for a sorted
// sequence: each run inside a wave is added with one atomic.
template <typename Get>
__global__ __launch_bounds__(kBlock) void k_run_counts(Get get, uint64_t m, int32_t* __restrict__ deg) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x; i0 < m; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    const bool valid = i < m;
    const int32_t v = valid ? get(i) : -1;
    const int32_t prev = __shfl_up(v, 1, kWave);
    const bool head = valid && (lane_id() == 0 || prev != v);
    const uint64_t heads = __ballot(head);
    const uint64_t vmask = __ballot(valid);
    if (head) {
      const uint64_t above = heads & ~((2ull << lane_id()) - 1ull);  // heads after this lane (lane 63: none)
      const int end = above ? __ffsll(static_cast<long long>(above)) - 1 : 64 - __clzll(static_cast<long long>(vmask));
      atomicAdd(&deg[v], end - lane_id());
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_larger_ends(const uint64_t* __restrict__ uk, uint64_t m, int b,
                                                         uint32_t* __restrict__ out) {
  const uint64_t mask = (1ull << b) - 1;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<uint32_t>(uk[i] & mask);
}

// Rank key of a vertex: graph index (hi word), then the order key, then id.
// order 0: degree (Eq. (1)); 1: id; 2: a fixed pseudo-random permutation;
// 3: degree descending; a coreness order passes the coreness as `d` with
// order 0. Any total order counts each triangle once (Theorem 1).
__device__ __forceinline__ uint64_t order_key(int order, int32_t v, int32_t d, int b) {
  const uint64_t mask = (1ull << b) - 1;
  switch (order) {
    case 1: return 0;
    case 2: return ((static_cast<uint64_t>(static_cast<uint32_t>(v)) + 1ull) * 0x9E3779B97F4A7C15ull >> 40) & mask;
    case 3: return mask - static_cast<uint64_t>(d);
    default: return static_cast<uint64_t>(d);
  }
}

__global__ void k_rank_keys(int32_t n, int b, const int32_t* __restrict__ deg, const int32_t* __restrict__ vbase,
                            int32_t G, int order, u128* __restrict__ out) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    uint64_t g = 0;
    if (G > 1) {
      int32_t lo = 0, hi = G - 1;
      while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (vbase[mid] <= v) lo = mid;
        else hi = mid - 1;
      }
      g = static_cast<uint64_t>(lo);
    }
    out[v] = u128{(order_key(order, v, deg[v], b) << b) | static_cast<uint64_t>(v), g};
  }
}

__global__ void k_rank_from_sorted(const u128* __restrict__ sorted, int32_t n, int b, int32_t* __restrict__ order,
                                   int32_t* __restrict__ rank, int32_t* __restrict__ graph_of_rank) {
  const uint64_t mask = (1ull << b) - 1;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const u128 k = sorted[r];
    const int32_t v = static_cast<int32_t>(k.lo & mask);
    order[r] = v;
    rank[v] = r;
    if (graph_of_rank) graph_of_rank[r] = static_cast<int32_t>(k.hi);
  }
}

// Orientation of Eq. (1): the endpoint earlier in the degree order has the
// smaller rank and becomes the row.
__global__ void k_relabel(const uint64_t* __restrict__ uk, uint64_t m, int b, const int32_t* __restrict__ rank,
                          uint64_t* __restrict__ ok) {
  const uint64_t mask = (1ull << b) - 1;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t k = uk[i];
    const uint64_t ra = static_cast<uint64_t>(rank[k >> b]), rb = static_cast<uint64_t>(rank[k & mask]);
    ok[i] = ra < rb ? ((ra << b) | rb) : ((rb << b) | ra);
  }
}

__global__ void k_csr_fill(const uint64_t* __restrict__ ok, uint64_t m, int b, int32_t* __restrict__ adj,
                           int32_t* __restrict__ src) {
  const uint64_t mask = (1ull << b) - 1;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t k = ok[i];
    adj[i] = static_cast<int32_t>(k & mask);
    src[i] = static_cast<int32_t>(k >> b);
  }
}

// off[r] = first entry whose row is >= r, for sorted rows `row` of length m
// (one binary search per row, so long runs of empty rows cost nothing extra).
struct RowOfI32 {
  const int32_t* r;
  __device__ int64_t operator()(uint64_t i) const { return r[i]; }
};
struct RowOfKeyHi {
  const uint64_t* k;
  __device__ int64_t operator()(uint64_t i) const { return static_cast<int64_t>(k[i] >> 32); }
};

// off[r] = first position whose row is >= r (one binary search per row).
template <typename Row>
__global__ void k_offsets_from_rows(Row row, uint64_t m, int32_t n, int64_t* __restrict__ off) {
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r <= n;
       r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (row(mid) < r) lo = mid + 1;
      else hi = mid;
    }
    off[r] = static_cast<int64_t>(lo);
  }
}

__global__ void k_row_max(const int64_t* __restrict__ off, int32_t n, int* __restrict__ out) {
  int best = 0;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const int d = static_cast<int>(off[r + 1] - off[r]);
    best = d > best ? d : best;
  }
  best = wave_max(best);
  if (lane_id() == 0 && best > 0) atomicMax(out, best);
}

__global__ void k_array_max(const int32_t* __restrict__ a, int32_t n, int* __restrict__ out) {
  int best = 0;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) best = a[r] > best ? a[r] : best;
  best = wave_max(best);
  if (lane_id() == 0 && best > 0) atomicMax(out, best);
}

}  // namespace

void offsets_from_rows(const int32_t* row, uint64_t m, int32_t n, int64_t* off, hipStream_t s) {
  k_offsets_from_rows<<<grid_for(static_cast<uint64_t>(n) + 1, kBlock, 65536), kBlock, 0, s>>>(RowOfI32{row}, m, n, off);
  TC_LAUNCH_CHECK();
}

void offsets_from_key_rows(const uint64_t* keys, uint64_t m, int32_t n, int64_t* off, hipStream_t s) {
  k_offsets_from_rows<<<grid_for(static_cast<uint64_t>(n) + 1, kBlock, 65536), kBlock, 0, s>>>(RowOfKeyHi{keys}, m, n,
                                                                                                 off);
  TC_LAUNCH_CHECK();
}

int32_t max_row_length(const int64_t* off, int32_t n, hipStream_t s) {
  DevBuf<int> mx(1, s);
  TC_HIP(hipMemsetAsync(mx.get(), 0, sizeof(int), s));
  if (n > 0) {
    k_row_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(off, n, mx.get());
    TC_LAUNCH_CHECK();
  }
  int h = 0;
  TC_HIP(hipMemcpyAsync(&h, mx.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  return h;
}

void build_graph(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, const int64_t* edge_off_host,
                 const int32_t* n_per_graph_host, int32_t G, bool on_device, hipStream_t s, tc_graph* g, int order,
                 const int32_t* key_by_id) {
  if (E < 0 || n < 0) fail(TC_E_RANGE, "negative edge or vertex count");
  if (n > kMaxVertices) fail(TC_E_RANGE, "more than 2^31 - 2^25 vertices");
  // k_canon counts records in uint32 with strides of up to 2^24
  if (E > (1ll << 32) - (1ll << 25)) fail(TC_E_INVAL, "more than 2^32 - 2^25 edge records");
  if (E > 0 && (!src || !dst)) fail(TC_E_INVAL, "NULL edge array");
  TC_HIP(hipGetDevice(&g->device));
  g->n = n;
  g->num_graphs = G;
  g->vbase.assign(static_cast<size_t>(G) + 1, 0);
  if (n_per_graph_host) {
    int64_t acc = 0;
    for (int32_t i = 0; i < G; i++) {
      if (n_per_graph_host[i] < 0) fail(TC_E_RANGE, "negative vertex count in batch");
      g->vbase[i] = static_cast<int32_t>(acc);
      acc += n_per_graph_host[i];
    }
    if (acc != n) fail(TC_E_INVAL, "batch vertex counts do not add up");
    g->vbase[G] = n;
  } else {
    g->vbase[0] = 0;
    g->vbase[1] = n;
  }
  const int b = bits_for(n > 1 ? static_cast<uint64_t>(n - 1) : 1);
  g->bits = b;
  g->order_kind = order;
  const int gbits = G > 1 ? bits_for(static_cast<uint64_t>(G - 1)) : 0;

  // ---- inputs on the device
  DevBuf<int32_t> hsrc, hdst;
  const int32_t* dsrc = src;
  const int32_t* ddst = dst;
  if (!on_device && E > 0) {
    hsrc.alloc(E, s);
    hdst.alloc(E, s);
    TC_HIP(hipMemcpyAsync(hsrc.get(), src, E * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TC_HIP(hipMemcpyAsync(hdst.get(), dst, E * sizeof(int32_t), hipMemcpyHostToDevice, s));
    dsrc = hsrc.get();
    ddst = hdst.get();
  }
  DevBuf<int64_t> d_eoff;
  DevBuf<int32_t> d_vbase(static_cast<size_t>(G) + 1, s);
  TC_HIP(hipMemcpyAsync(d_vbase.get(), g->vbase.data(), (G + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (edge_off_host) {
    if (edge_off_host[0] != 0 || edge_off_host[G] != E) fail(TC_E_INVAL, "batch edge offsets do not span the edges");
    for (int32_t i = 0; i < G; i++)
      if (edge_off_host[i + 1] < edge_off_host[i]) fail(TC_E_INVAL, "batch edge offsets decrease");
    d_eoff.alloc(static_cast<size_t>(G) + 1, s);
    TC_HIP(hipMemcpyAsync(d_eoff.get(), edge_off_host, (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  }

  // ---- 1-2: canonical keys, sort, unique
  DevBuf<uint64_t> keys(E, s), tmp(E, s);
  DevBuf<int> err(1, s);
  DevBuf<uint64_t> d_m(1, s);
  DevBuf<uint32_t> sort_fail(1, s);  // set by any sort whose look-back gave up; checked at the syncs below
  TC_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));
  TC_HIP(hipMemsetAsync(sort_fail.get(), 0, sizeof(uint32_t), s));
  uint64_t* uniq = nullptr;
  uint64_t* spare = nullptr;
  if (E > 0) {
    k_canon<<<grid_for(E, kBlock, 65536), kBlock, 0, s>>>(dsrc, ddst, static_cast<uint32_t>(E), n, b, d_eoff.get(),
                                                          d_vbase.get(), G, keys.get(), err.get());
    TC_LAUNCH_CHECK();
    uint64_t* sorted = radix_sort<uint64_t>(keys.get(), tmp.get(), E, 0, 2 * b, s, sort_fail.get());
    spare = sorted == keys.get() ? tmp.get() : keys.get();
    compact_if<uint64_t>(E, UniquePred{sorted}, GatherU64{sorted}, spare, d_m.get(), s);
    uniq = spare;
    spare = sorted;
  } else {
    TC_HIP(hipMemsetAsync(d_m.get(), 0, sizeof(uint64_t), s));
  }
  hsrc.release();
  hdst.release();
  int h_err = 0;
  uint64_t m = 0;
  uint32_t h_fail = 0;
  TC_HIP(hipMemcpyAsync(&h_err, err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  TC_HIP(hipMemcpyAsync(&m, d_m.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipMemcpyAsync(&h_fail, sort_fail.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h_fail) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  if (h_err) fail(TC_E_RANGE, "vertex id outside [0, n)");
  g->m = static_cast<int64_t>(m);

  // ---- 3: degrees
  g->deg.alloc(n, s);
  if (n > 0) TC_HIP(hipMemsetAsync(g->deg.p, 0, n * sizeof(int32_t), s));
  if (m > 0) {
    // d_v = (edges with v as the smaller endpoint: runs of the sorted keys)
    //     + (edges with v as the larger endpoint: runs after sorting those ends);
    // the larger ends and their sort buffer live in the spare key buffer (E >= m)
    k_run_counts<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(LoEnd{uniq, b}, m, g->deg.p);
    TC_LAUNCH_CHECK();
    uint32_t* ends = reinterpret_cast<uint32_t*>(spare);
    k_larger_ends<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(uniq, m, b, ends);
    TC_LAUNCH_CHECK();
    const uint32_t* sorted_ends = radix_sort<uint32_t>(ends, ends + m, m, 0, b, s, sort_fail.get());
    k_run_counts<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(HiEnd{sorted_ends}, m, g->deg.p);
    TC_LAUNCH_CHECK();
  }

  // ---- 4: ranks in the degree order
  g->order.alloc(n, s);
  g->rank.alloc(n, s);
  if (G > 1) g->graph_of_rank.alloc(n, s);
  if (n > 0) {
    DevBuf<u128> rk(n, s), rk2(n, s);
    // a caller-supplied key (coreness) orders like the degree: ascending, ties by id
    k_rank_keys<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(n, b, key_by_id ? key_by_id : g->deg.p, d_vbase.get(),
                                                               G, key_by_id ? 0 : order, rk.get());
    TC_LAUNCH_CHECK();
    u128* r1 = radix_sort<u128>(rk.get(), rk2.get(), n, 0, 2 * b, s, sort_fail.get());
    u128* r2 = r1;
    if (G > 1) r2 = radix_sort<u128>(r1, r1 == rk.get() ? rk2.get() : rk.get(), n, 64, 64 + gbits, s, sort_fail.get());
    k_rank_from_sorted<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(r2, n, b, g->order.p, g->rank.p,
                                                                      G > 1 ? g->graph_of_rank.p : nullptr);
    TC_LAUNCH_CHECK();
  }

  // ---- 5-6: orientation, sorted rows, offsets
  Csr& c = g->csr;
  c.n = n;
  c.m = static_cast<int64_t>(m);
  c.off.alloc(static_cast<size_t>(n) + 1, s);
  c.adj.alloc(m, s);
  c.src.alloc(m, s);
  if (m > 0) {
    k_relabel<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(uniq, m, b, g->rank.p, spare);
    TC_LAUNCH_CHECK();
    uint64_t* ok = radix_sort<uint64_t>(spare, uniq, m, 0, 2 * b, s, sort_fail.get());
    k_csr_fill<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(ok, m, b, c.adj.p, c.src.p);
    TC_LAUNCH_CHECK();
  }
  offsets_from_rows(c.src.p, m, n, c.off.p, s);
  keys.release();
  tmp.release();

  DevBuf<int> mx(2, s);
  TC_HIP(hipMemsetAsync(mx.get(), 0, 2 * sizeof(int), s));
  if (n > 0) {
    k_row_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(c.off.p, n, mx.get());
    TC_LAUNCH_CHECK();
    k_array_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(g->deg.p, n, mx.get() + 1);
    TC_LAUNCH_CHECK();
  }
  int h_mx[2] = {0, 0};
  TC_HIP(hipMemcpyAsync(h_mx, mx.get(), 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  TC_HIP(hipMemcpyAsync(&h_fail, sort_fail.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h_fail) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  c.dhat_max = h_mx[0];
  g->d_max = h_mx[1];
}

}  // namespace tc
