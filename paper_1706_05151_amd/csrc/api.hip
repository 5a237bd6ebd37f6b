// The C ABI (include/tc.h): argument checks, device/stream plumbing, error
// mapping, and the small per-node epilogues (permutation to caller ids and
// clustering coefficients).
#include <atomic>
#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "graph.hpp"
#include "primitives.hpp"

namespace tc {

namespace {

thread_local std::string g_last_error;
std::atomic<int64_t> g_opt_kernel{0}, g_opt_hub{256}, g_opt_iw{0}, g_opt_bpc{4}, g_opt_load{2}, g_opt_order{0};

template <typename F>
tc_status guarded(F&& f) {
  g_last_error.clear();
  try {
    f();
    return TC_OK;
  } catch (const Failure& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return TC_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return TC_E_DEVICE;
  }
}

// Makes the graph's device current for the duration of a call.
struct DeviceScope {
  int prev = -1, want = 0;
  explicit DeviceScope(int dev) : want(dev) {
    TC_HIP(hipGetDevice(&prev));
    if (prev != dev) TC_HIP(hipSetDevice(dev));
  }
  ~DeviceScope() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
};

constexpr int kBlock = 256;

__global__ void k_scatter_by_order(const unsigned long long* __restrict__ by_rank, const int32_t* __restrict__ order,
                                   int32_t n, unsigned long long* __restrict__ by_id) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) by_id[order[r]] = by_rank[r];
}

// C_v = T_v / C(d_v,2): exact numerator and denominator, one IEEE division.
__global__ void k_clustering(const unsigned long long* __restrict__ t, const int32_t* __restrict__ deg, int32_t n,
                             uint64_t* __restrict__ num, uint64_t* __restrict__ den, double* __restrict__ c) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const uint64_t d = static_cast<uint64_t>(deg[v]);
    const uint64_t nu = t[v];
    const uint64_t de = d >= 2 ? d * (d - 1) / 2 : 0;
    if (num) num[v] = nu;
    if (den) den[v] = de;
    if (c) c[v] = de ? static_cast<double>(nu) / static_cast<double>(de) : 0.0;
  }
}

// Order-independent 128-bit digest of a clustering answer: per vertex v,
// h = f(f(f(f(v ^ K) ^ num) ^ den) ^ bits(c)) with f the SplitMix64 output
// function; digest = (sum of h, sum of f(h ^ K')) modulo 2^64. Sums commute,
// so the atomics give the same bits in any order.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_cc_digest(const uint64_t* __restrict__ num, const uint64_t* __restrict__ den,
                            const double* __restrict__ c, int32_t n, unsigned long long* __restrict__ out) {
  unsigned long long a = 0, b = 0;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const uint64_t cb = static_cast<uint64_t>(__double_as_longlong(c[v]));
    const uint64_t h = mix64(mix64(mix64(mix64(static_cast<uint64_t>(v) ^ 0x434c555354455221ull) ^ num[v]) ^ den[v]) ^ cb);
    a += h;
    b += mix64(h ^ 0x4449474553543132ull);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    atomicAdd(&out[0], a);
    atomicAdd(&out[1], b);
  }
}

__global__ void k_dhat_by_id(const int64_t* __restrict__ off, const int32_t* __restrict__ order, int32_t n,
                             int32_t* __restrict__ dhat) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    dhat[order[r]] = static_cast<int32_t>(off[r + 1] - off[r]);
}

__global__ void k_oriented_keys(const int32_t* __restrict__ adj, const int32_t* __restrict__ src,
                                const int32_t* __restrict__ order, uint64_t m, int b, uint64_t* __restrict__ keys) {
  for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    keys[e] = (static_cast<uint64_t>(order[src[e]]) << b) | static_cast<uint64_t>(order[adj[e]]);
}

__global__ void k_split_keys(const uint64_t* __restrict__ keys, uint64_t m, int b, int32_t* __restrict__ row,
                             int32_t* __restrict__ col) {
  const uint64_t mask = (1ull << b) - 1;
  for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    row[e] = static_cast<int32_t>(keys[e] >> b);
    if (col) col[e] = static_cast<int32_t>(keys[e] & mask);
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

void require(bool ok, tc_status st, const char* msg) {
  if (!ok) fail(st, msg);
}

// T (and optionally per-node counts by rank) of one CSR with the selected kernel.
uint64_t count_total(tc_graph* g, Csr& c, hipStream_t s, unsigned long long* t_rank) {
  const Options o = get_options();
  DevBuf<unsigned long long> tot(1, s);
  fill_u64(tot.get(), 1, 0ull, s);
  if (t_rank) {
    fill_u64(t_rank, static_cast<size_t>(c.n), 0ull, s);
    CountArgs a;
    a.mode = kCountPerNode;
    a.total = tot.get();
    a.t_rank = t_rank;
    std::lock_guard<std::mutex> lk(g->mu);
    if (plain_is_best(c, o)) count_plain_mode(c, a, s);
    else count_pivot(c, a, s, o);
  } else if (plain_is_best(c, o)) {
    count_plain(c, tot.get(), s);
  } else {
    CountArgs a;
    a.mode = kCountTotal;
    a.total = tot.get();
    std::lock_guard<std::mutex> lk(g->mu);
    count_pivot(c, a, s, o);
  }
  unsigned long long h = 0;
  TC_HIP(hipMemcpyAsync(&h, tot.get(), sizeof(h), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

Options get_options() {
  Options o;
  o.kernel = g_opt_kernel.load();
  o.hub_dhat = g_opt_hub.load();
  o.item_work = g_opt_iw.load();
  o.blocks_per_cu = g_opt_bpc.load();
  o.hub_bucket_load = g_opt_load.load();
  o.order = g_opt_order.load();
  return o;
}

}  // namespace tc

using namespace tc;

extern "C" {

// Coreness by caller id of a built graph (the plan must exist).
__global__ void k_i32_by_order(const int32_t* __restrict__ by_rank, const int32_t* __restrict__ order, int32_t n,
                               int32_t* __restrict__ by_id) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) by_id[order[r]] = by_rank[r];
}

static void coreness_by_id(tc_graph* g, hipStream_t s, int32_t* core_id) {
  if (g->n <= 0) return;
  DevBuf<int32_t> cr(g->n, s);
  coreness_rank(g->csr, s, cr.get());
  k_i32_by_order<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(cr.get(), g->order.p, g->n, core_id);
  TC_LAUNCH_CHECK();
}

// Builds g (and its plan) in the order of the TC_OPT_ORDER option. The
// coreness order first builds the graph in degree order, takes its coreness
// and builds again with the coreness as the order key.
static void build_in_order(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, const int64_t* edge_off,
                           const int32_t* n_per_graph, int32_t G, bool on_device, hipStream_t s, tc_graph* g) {
  const Options o = get_options();
  if (o.order == 4) {
    std::unique_ptr<tc_graph> g0(new tc_graph());
    build_graph(src, dst, E, n, edge_off, n_per_graph, G, on_device, s, g0.get(), 0, nullptr);
    ensure_plan(g0->csr, s, o);
    DevBuf<int32_t> core(static_cast<size_t>(n), s);
    coreness_by_id(g0.get(), s, core.get());
    build_graph(src, dst, E, n, edge_off, n_per_graph, G, on_device, s, g, 4, core.get());
    TC_HIP(hipStreamSynchronize(s));
    ensure_plan(g->csr, s, o);
    return;
  }
  HostWords tail(s);
  build_graph(src, dst, E, n, edge_off, n_per_graph, G, on_device, s, g, static_cast<int>(o.order), nullptr,
              tail.get());
  ensure_plan(g->csr, s, o);  // work plan of the intersection kernel (it needs no dhat_max)
  TC_HIP(hipStreamSynchronize(s));
  build_graph_finish(g, tail.get());
}

tc_status tc_build_csr(const int32_t* src, const int32_t* dst, int64_t num_edges, int32_t n, uint32_t flags,
                       void* stream, tc_graph** out) {
  return guarded([&] {
    require(out != nullptr, TC_E_INVAL, "out is NULL");
    *out = nullptr;
    auto* g = new tc_graph();
    try {
      build_in_order(src, dst, num_edges, n, nullptr, nullptr, 1, (flags & TC_IN_DEVICE) != 0, as_stream(stream), g);
    } catch (...) {
      (void)hipStreamSynchronize(as_stream(stream));
      delete g;
      throw;
    }
    *out = g;
  });
}

tc_status tc_batch_build(const int32_t* src, const int32_t* dst, const int64_t* edge_off, const int32_t* n_per_graph,
                         int32_t num_graphs, uint32_t flags, void* stream, tc_graph** out) {
  return guarded([&] {
    require(out != nullptr, TC_E_INVAL, "out is NULL");
    require(num_graphs >= 1, TC_E_INVAL, "num_graphs < 1");
    require(edge_off != nullptr && n_per_graph != nullptr, TC_E_INVAL, "NULL batch description");
    *out = nullptr;
    int64_t ntot = 0;
    for (int32_t i = 0; i < num_graphs; i++) ntot += n_per_graph[i] > 0 ? n_per_graph[i] : 0;
    require(ntot <= kMaxVertices, TC_E_RANGE, "batch has more than 2^31 - 2^25 vertices");
    const hipStream_t s = as_stream(stream);
    auto* g = new tc_graph();
    try {
      build_in_order(src, dst, edge_off[num_graphs], static_cast<int32_t>(ntot), edge_off, n_per_graph, num_graphs,
                     (flags & TC_IN_DEVICE) != 0, s, g);
      g->workspace.alloc((3 + static_cast<size_t>(g->n)) * sizeof(unsigned long long), s);
      TC_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      delete g;
      throw;
    }
    *out = g;
  });
}

tc_status tc_graph_replan(tc_graph* g, void* stream) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    {
      std::lock_guard<std::mutex> lk(g->mu);
      rebuild_plan(g->csr, s, get_options());
    }
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_graph_plan_info(const tc_graph* g, int64_t* hub_dhat, int64_t* item_work, int32_t* frozen) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    const PivotPlan& P = g->csr.plan;
    require(P.ready, TC_E_INVAL, "the graph has no work plan");
    if (hub_dhat) *hub_dhat = P.hub_dhat;
    if (item_work) *item_work = P.item_work;
    if (frozen) *frozen = P.frozen ? 1 : 0;
  });
}

static size_t plan_reserved(const PivotPlan& P) {
  return dev_reserved_bytes(P.inrec.p) + dev_reserved_bytes(P.in_off.p) + dev_reserved_bytes(P.items.p) +
         dev_reserved_bytes(P.grouped.p);
}

tc_status tc_graph_bytes(const tc_graph* g, uint64_t* bytes) {
  return guarded([&] {
    require(g != nullptr && bytes != nullptr, TC_E_INVAL, "NULL argument");
    DeviceScope ds(g->device);
    const Csr& c = g->csr;
    size_t b = dev_reserved_bytes(c.off.p) + dev_reserved_bytes(c.adj.p) + dev_reserved_bytes(c.src.p) +
               plan_reserved(c.plan) + plan_reserved(c.shard) + dev_reserved_bytes(g->order.p) +
               dev_reserved_bytes(g->rank.p) + dev_reserved_bytes(g->deg.p) +
               dev_reserved_bytes(g->graph_of_rank.p) + dev_reserved_bytes(g->workspace.p);
    *bytes = static_cast<uint64_t>(b);
  });
}

tc_status tc_batch_size(const tc_graph* g, int32_t* num_graphs) {
  return guarded([&] {
    require(g != nullptr && num_graphs != nullptr, TC_E_INVAL, "NULL argument");
    *num_graphs = g->num_graphs;
  });
}

tc_status tc_graph_info(const tc_graph* g, int32_t* n, int64_t* m, int32_t* d_max, int32_t* dhat_max) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (d_max) *d_max = g->d_max;
    if (dhat_max) *dhat_max = g->csr.dhat_max;
  });
}

void tc_graph_free(tc_graph* g) {
  if (!g) return;
  const int dev = g->device;
  int prev = -1;
  if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  // Calls that return before their work is done (batch, multi-graph and
  // clustering-from-counts) record an event on the graph's plan, and so does
  // every launch of the intersection kernel; every other call synchronised
  // its stream before returning. Waiting for those events makes the arrays
  // free, without stalling the other streams of the device.
  g->csr.plan.users.sync();
  g->csr.shard.users.sync();
  delete g;
  if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

tc_status tc_count(tc_graph* g, void* stream, uint64_t* T) {
  return guarded([&] {
    require(g != nullptr && T != nullptr, TC_E_INVAL, "NULL argument");
    DeviceScope ds(g->device);
    *T = count_total(g, g->csr, as_stream(stream), nullptr);
  });
}

tc_status tc_count_plain(tc_graph* g, void* stream, uint64_t* T) {
  return guarded([&] {
    require(g != nullptr && T != nullptr, TC_E_INVAL, "NULL argument");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> tot(1, s);
    fill_u64(tot.get(), 1, 0ull, s);
    count_plain(g->csr, tot.get(), s);
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, tot.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    *T = h;
  });
}

tc_status tc_count_per_node(tc_graph* g, void* stream, uint64_t* T, uint64_t* t_dev) {
  return guarded([&] {
    require(g != nullptr && t_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(!g->sampled, TC_E_INVAL, "per-node counts are not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> tr(g->n, s);
    const uint64_t tot = count_total(g, g->csr, s, tr.get());
    if (g->n > 0) {
      k_scatter_by_order<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(
          tr.get(), g->order.p, g->n, reinterpret_cast<unsigned long long*>(t_dev));
      TC_LAUNCH_CHECK();
    }
    TC_HIP(hipStreamSynchronize(s));
    if (T) *T = tot;
  });
}

}  // extern "C"

namespace tc {
namespace {

// Scratch of tc_count_per_node_noalloc, one copy per device held for the life
// of the process: words 0..2 are the work-queue counters of the persistent
// launch, word 3 the total, words 4.. the per-node counts by rank of at most
// kNoAllocMaxVertices vertices (32 MiB in all).
constexpr int32_t kNoAllocMaxVertices = 1 << 22;
constexpr size_t kNoAllocWords = 4 + static_cast<size_t>(kNoAllocMaxVertices);
__device__ __align__(256) unsigned long long scratch[kNoAllocWords];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on device dev, which must be current. In host
// code the array's name is only a stand-in for the symbol; kernels are given
// this address instead.
unsigned long long* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) fail(TC_E_DEVICE, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      fail(TC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_addr[dev] = static_cast<unsigned long long*>(p);
  }
  return g_scratch_addr[dev];
}

}  // namespace
}  // namespace tc

extern "C" {

tc_status tc_count_per_node_noalloc(tc_graph* g, void* stream, uint64_t* T, uint64_t* t_dev) {
  return guarded([&] {
    require(g != nullptr && t_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(!g->sampled, TC_E_INVAL, "per-node counts are not available on a sampled graph");
    require(g->n <= kNoAllocMaxVertices, TC_E_RANGE,
            "more than 2^22 vertices: the static scratch holds per-node counts of at most 2^22 vertices");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    unsigned long long* ws = scratch_on(g->device);
    const int32_t n = g->n;
    // Held until the counts are in host memory, so no other call replaces the
    // plan while the launch reads it (the launch records no plan-use event).
    std::lock_guard<std::mutex> lk(g->mu);
    fill_u64(ws, 4 + static_cast<size_t>(n), 0ull, s);  // a fill kernel: no memset node, nothing allocated
    CountArgs a;
    a.mode = kCountPerNode;
    a.queues = ws;
    a.total = ws + 3;
    a.t_rank = ws + 4;
    a.note_use = false;
    count_pivot(g->csr, a, s, get_options(), /*allow_rebuild=*/false);
    if (n > 0) {
      k_scatter_by_order<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(ws + 4, g->order.p, n,
                                                                        reinterpret_cast<unsigned long long*>(t_dev));
      TC_LAUNCH_CHECK();
    }
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, ws + 3, sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (T) *T = h;
  });
}

tc_status tc_clustering(tc_graph* g, void* stream, uint64_t* num_dev, uint64_t* den_dev, double* c_dev) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "clustering is not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> tr(g->n, s), tid(g->n, s);
    (void)count_total(g, g->csr, s, tr.get());
    if (g->n > 0) {
      k_scatter_by_order<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(tr.get(), g->order.p, g->n, tid.get());
      TC_LAUNCH_CHECK();
      k_clustering<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(tid.get(), g->deg.p, g->n, num_dev, den_dev, c_dev);
      TC_LAUNCH_CHECK();
    }
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_list(tc_graph* g, void* stream, int32_t* tri_dev, int64_t cap, int64_t* count) {
  return guarded([&] {
    require(g != nullptr && count != nullptr, TC_E_INVAL, "NULL argument");
    require(cap >= 0, TC_E_INVAL, "negative capacity");
    require(!g->sampled, TC_E_INVAL, "listing is not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    const uint64_t T = count_total(g, g->csr, s, nullptr);
    *count = static_cast<int64_t>(T);
    if (!tri_dev || cap == 0 || T == 0) return;
    if (static_cast<uint64_t>(cap) < T) fail(TC_E_TRUNC, "triangle list capacity smaller than T");
    DevBuf<unsigned long long> cur(1, s);
    fill_u64(cur.get(), 1, 0ull, s);
    CountArgs a;
    a.mode = kCountList;
    a.order = g->order.p;
    a.tri = tri_dev;
    a.cursor = cur.get();
    a.cap = static_cast<int64_t>(T);
    {
      std::lock_guard<std::mutex> lk(g->mu);
      const Options o = get_options();
      if (plain_is_best(g->csr, o)) count_plain_mode(g->csr, a, s);
      else count_pivot(g->csr, a, s, o);
    }
    unsigned long long written = 0;
    TC_HIP(hipMemcpyAsync(&written, cur.get(), sizeof(written), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (written != T) fail(TC_E_DEVICE, "listing pass disagrees with the count pass");
    sort_triangles(tri_dev, static_cast<int64_t>(T), g->bits, s);
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_sparsify_count(tc_graph* g, double q, uint64_t seed, void* stream, uint64_t* T_sampled, int64_t* m_kept,
                            double* estimate) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "cannot sample a sampled graph");
    require(q > 0.0 && q <= 1.0, TC_E_RANGE, "q outside (0, 1]");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    Csr sampled;
    build_sampled_csr(g, q, seed, sampled, s);
    const uint64_t Ts = count_total(g, sampled, s, nullptr);
    TC_HIP(hipStreamSynchronize(s));
    if (T_sampled) *T_sampled = Ts;
    if (m_kept) *m_kept = sampled.m;
    if (estimate) *estimate = static_cast<double>(Ts) / ((q * q) * q);
  });
}

tc_status tc_count_partitioned(tc_graph* g, void* stream, int32_t scheme, int32_t parts, uint64_t* T,
                               int64_t* bounds_dev, uint64_t* work_dev) {
  return guarded([&] {
    require(g != nullptr && T != nullptr, TC_E_INVAL, "NULL argument");
    require(scheme >= 0 && scheme <= 6, TC_E_INVAL, "scheme must be 0..6");
    require(parts >= 1, TC_E_INVAL, "parts < 1");
    require(!g->sampled, TC_E_INVAL, "partitioned counts are not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    std::lock_guard<std::mutex> lk(g->mu);
    ensure_plan(g->csr, s, get_options());
    DevBuf<int64_t> bb;
    DevBuf<unsigned long long> ww, tt(1, s);
    int64_t* b = bounds_dev;
    unsigned long long* w = reinterpret_cast<unsigned long long*>(work_dev);
    if (!b) {
      bb.alloc(static_cast<size_t>(parts) + 1, s);
      b = bb.get();
    }
    if (!w) {
      ww.alloc(static_cast<size_t>(parts), s);
      w = ww.get();
    }
    count_partitioned(g->csr, g->order.p, g->rank.p, g->deg.p, scheme, parts, tt.get(), b, w, s);
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, tt.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    *T = h;
  });
}

tc_status tc_graph_coreness(tc_graph* g, void* stream, int32_t* core_dev) {
  return guarded([&] {
    require(g != nullptr && core_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(!g->sampled, TC_E_INVAL, "coreness is not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    std::lock_guard<std::mutex> lk(g->mu);
    ensure_plan(g->csr, s, get_options());
    coreness_by_id(g, s, core_dev);
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_shard_bounds(tc_graph* g, void* stream, int32_t k, int32_t cost, int32_t* bounds) {
  return guarded([&] {
    require(g != nullptr && bounds != nullptr, TC_E_INVAL, "NULL argument");
    require(k >= 1, TC_E_INVAL, "k < 1");
    require(cost == 0 || cost == 1, TC_E_INVAL, "cost must be 0 or 1");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<int64_t> b(static_cast<size_t>(k) + 1, s);
    shard_bounds(g->csr, k, cost, b.get(), s);
    std::vector<int64_t> h(static_cast<size_t>(k) + 1);
    TC_HIP(hipMemcpyAsync(h.data(), b.get(), h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    for (int32_t j = 0; j <= k; j++) bounds[j] = static_cast<int32_t>(h[j]);
  });
}

tc_status tc_count_shard(tc_graph* g, void* stream, int32_t lo, int32_t hi, uint64_t* T) {
  return guarded([&] {
    require(g != nullptr && T != nullptr, TC_E_INVAL, "NULL argument");
    require(lo >= 0 && lo <= hi && hi <= g->n, TC_E_RANGE, "rank range outside [0, n]");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> tot(1, s);
    fill_u64(tot.get(), 1, 0ull, s);
    {
      std::lock_guard<std::mutex> lk(g->mu);
      count_shard(g->csr, lo, hi, tot.get(), s, get_options());
    }
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, tot.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    *T = h;
  });
}

// Output i + 1 of the SplitMix64 generator (Steele, Lea and Flood, 2014)
// started at `seed`: the seed of partition i's sample.
static uint64_t partition_seed(uint64_t seed, int32_t i) {
  uint64_t z = seed + static_cast<uint64_t>(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

tc_status tc_sparsify_count_partitioned(tc_graph* g, double q, uint64_t seed, int32_t parts, void* stream,
                                        uint64_t* T_parts, int32_t* bounds, uint64_t* T_sampled, double* estimate) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "cannot sample a sampled graph");
    require(q > 0.0 && q <= 1.0, TC_E_RANGE, "q outside (0, 1]");
    require(parts >= 1, TC_E_INVAL, "parts < 1");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    const Options o = get_options();
    std::vector<int64_t> hb(static_cast<size_t>(parts) + 1);
    {
      DevBuf<int64_t> b(hb.size(), s);
      shard_bounds(g->csr, parts, 0, b.get(), s);
      TC_HIP(hipMemcpyAsync(hb.data(), b.get(), hb.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
    }
    DevBuf<unsigned long long> t(static_cast<size_t>(parts), s);
    fill_u64(t.get(), static_cast<size_t>(parts), 0ull, s);
    for (int32_t i = 0; i < parts; i++) {
      const int32_t lo = static_cast<int32_t>(hb[i]), hi = static_cast<int32_t>(hb[i + 1]);
      if (lo == hi) continue;
      // partition i samples every edge it can reach on its own: the rows of
      // ranks >= lo (its core nodes and all later vertices)
      Csr sampled;
      build_sampled_csr(g, q, partition_seed(seed, i), sampled, s, lo);
      count_shard(sampled, lo, hi, t.get() + i, s, o);
      TC_HIP(hipStreamSynchronize(s));
    }
    std::vector<unsigned long long> ht(static_cast<size_t>(parts));
    TC_HIP(hipMemcpyAsync(ht.data(), t.get(), ht.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    unsigned long long sum = 0;
    for (int32_t i = 0; i < parts; i++) {
      sum += ht[i];
      if (T_parts) T_parts[i] = ht[i];
    }
    if (bounds)
      for (int32_t j = 0; j <= parts; j++) bounds[j] = static_cast<int32_t>(hb[j]);
    if (T_sampled) *T_sampled = sum;
    if (estimate) *estimate = static_cast<double>(sum) / ((q * q) * q);
  });
}

tc_status tc_count_streamed(const int64_t* off, const int32_t* adj, int32_t n, int64_t m, uint64_t budget_bytes,
                            void* stream, uint64_t* T, uint64_t* info) {
  return guarded([&] {
    require(off != nullptr && T != nullptr && (adj != nullptr || m == 0), TC_E_INVAL, "NULL argument");
    require(n >= 0 && m >= 0, TC_E_INVAL, "negative size");
    require(n <= kMaxVertices, TC_E_RANGE, "more than 2^31 - 2^25 vertices");
    require(budget_bytes >= 4096, TC_E_INVAL, "budget below 4096 bytes");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, off) == hipSuccess && at.type == hipMemoryTypeDevice)
      fail(TC_E_INVAL, "row offsets must be in host memory");
    (void)hipGetLastError();
    require(off[0] == 0 && off[n] == m, TC_E_INVAL, "row offsets must run from 0 to m");
    uint64_t local[4];
    *T = count_streamed(off, adj, n, m, budget_bytes, as_stream(stream), get_options(), info ? info : local);
  });
}

tc_status tc_build_csr_host(const int32_t* src, const int32_t* dst, int64_t num_edges, int32_t n,
                            uint64_t budget_bytes, void* stream, int64_t* off, int32_t* adj, int64_t* m,
                            uint64_t* info) {
  return guarded([&] {
    uint64_t inf[4] = {0, 0, 0, 0};
    build_host_csr(src, dst, num_edges, n, budget_bytes, as_stream(stream), off, adj, m, inf);
    if (info)
      for (int i = 0; i < 4; i++) info[i] = inf[i];
  });
}

tc_status tc_graph_export_csr(tc_graph* g, void* stream, int64_t* off, int32_t* adj) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    if (off) TC_HIP(hipMemcpyAsync(off, g->csr.off.p, (static_cast<size_t>(g->csr.n) + 1) * sizeof(int64_t),
                                   hipMemcpyDefault, s));
    if (adj && g->csr.m > 0)
      TC_HIP(hipMemcpyAsync(adj, g->csr.adj.p, static_cast<size_t>(g->csr.m) * sizeof(int32_t), hipMemcpyDefault, s));
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_graph_work(tc_graph* g, void* stream, uint64_t* W, uint64_t* P) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> d(2, s);
    fill_u64(d.get(), 2, 0ull, s);
    graph_work(g->csr, d.get(), d.get() + 1, s);
    unsigned long long h[2] = {0, 0};
    TC_HIP(hipMemcpyAsync(h, d.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (W) *W = h[0];
    if (P) *P = h[1];
  });
}

tc_status tc_graph_order_cost(tc_graph* g, void* stream, uint64_t* cost, int32_t* order_kind) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> d(1, s);
    fill_u64(d.get(), 1, 0ull, s);
    order_cost(g->csr, g->deg.p, g->order.p, d.get(), s);
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, d.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (cost) *cost = h;
    if (order_kind) *order_kind = g->order_kind;
  });
}

tc_status tc_graph_degrees(tc_graph* g, void* stream, int32_t* deg_dev, int32_t* dhat_dev) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    if (deg_dev && g->n > 0)
      TC_HIP(hipMemcpyAsync(deg_dev, g->deg.p, g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (dhat_dev && g->n > 0) {
      k_dhat_by_id<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(g->csr.off.p, g->order.p, g->n, dhat_dev);
      TC_LAUNCH_CHECK();
    }
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_graph_order(tc_graph* g, void* stream, int32_t* order_dev) {
  return guarded([&] {
    require(g != nullptr && order_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(!g->sampled, TC_E_INVAL, "not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    if (g->n > 0) TC_HIP(hipMemcpyAsync(order_dev, g->order.p, g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_graph_oriented(tc_graph* g, void* stream, int64_t* off_dev, int32_t* adj_dev) {
  return guarded([&] {
    require(g != nullptr, TC_E_INVAL, "graph is NULL");
    require(!g->sampled, TC_E_INVAL, "not available on a sampled graph");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    const uint64_t m = static_cast<uint64_t>(g->m);
    DevBuf<uint64_t> k1(m, s), k2(m, s);
    DevBuf<int32_t> row(m, s);
    uint64_t* sorted = k1.get();
    if (m > 0) {
      k_oriented_keys<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(g->csr.adj.p, g->csr.src.p, g->order.p, m, g->bits,
                                                                    k1.get());
      TC_LAUNCH_CHECK();
      sorted = radix_sort<uint64_t>(k1.get(), k2.get(), m, 0, 2 * g->bits, s);
      k_split_keys<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(sorted, m, g->bits, row.get(), adj_dev);
      TC_LAUNCH_CHECK();
    }
    if (off_dev) offsets_from_rows(row.get(), m, g->n, off_dev, s);
    TC_HIP(hipStreamSynchronize(s));
  });
}

tc_status tc_batch_count(tc_graph* g, void* stream, uint64_t* T_dev, uint64_t* t_dev) {
  return guarded([&] {
    require(g != nullptr && T_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(g->workspace.p != nullptr, TC_E_INVAL, "graph was not built by tc_batch_build");
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    auto* ws = reinterpret_cast<unsigned long long*>(g->workspace.p);
    auto* Tg = reinterpret_cast<unsigned long long*>(T_dev);
    fill_u64(Tg, static_cast<size_t>(g->num_graphs), 0ull, s);
    CountArgs a;
    a.mode = t_dev ? kCountPerNode : kCountTotal;
    a.per_graph = Tg;
    a.graph_of_rank = g->num_graphs > 1 ? g->graph_of_rank.p : nullptr;
    a.queues = ws;
    if (t_dev) {
      a.t_rank = ws + 3;
      fill_u64(a.t_rank, static_cast<size_t>(g->n), 0ull, s);
    }
    const Options o = get_options();
    if (plain_is_best(g->csr, o)) count_plain_mode(g->csr, a, s);  // one thread per edge, no work plan
    else count_pivot(g->csr, a, s, o, /*allow_rebuild=*/false);
    if (t_dev && g->n > 0) {
      k_scatter_by_order<<<grid_for(g->n, kBlock, 65536), kBlock, 0, s>>>(a.t_rank, g->order.p, g->n,
                                                                          reinterpret_cast<unsigned long long*>(t_dev));
      TC_LAUNCH_CHECK();
    }
    note_plan_use(g->csr.plan, s);
  });
}

tc_status tc_multi_count(tc_graph* const* graphs, int32_t k, int32_t per_node, void* stream, uint64_t* T_dev,
                         uint64_t* const* t_dev) {
  return guarded([&] {
    require(k >= 0, TC_E_INVAL, "negative graph count");
    if (k == 0) return;
    require(graphs != nullptr && T_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(!per_node || t_dev != nullptr, TC_E_INVAL, "per-node counts need t_dev");
    const int dev = graphs[0] ? graphs[0]->device : 0;
    std::vector<Csr*> cs(k);
    for (int32_t i = 0; i < k; i++) {
      require(graphs[i] != nullptr, TC_E_INVAL, "NULL graph in list");
      require(graphs[i]->device == dev, TC_E_INVAL, "graphs of one multi count must share a device");
      require(!per_node || (graphs[i]->order.p != nullptr || graphs[i]->n == 0), TC_E_INVAL,
              "per-node counts are not available on a sampled graph");
      require(!per_node || t_dev[i] != nullptr, TC_E_INVAL, "NULL per-node output");
      cs[i] = &graphs[i]->csr;
    }
    DeviceScope ds(dev);
    const hipStream_t s = as_stream(stream);
    std::vector<DevBuf<unsigned long long>> tr(per_node ? k : 0);
    std::vector<unsigned long long*> trp(k, nullptr);
    if (per_node)
      for (int32_t i = 0; i < k; i++) {
        tr[i].alloc(static_cast<size_t>(graphs[i]->n), s);
        trp[i] = tr[i].get();
      }
    count_multi(cs, trp, per_node ? kCountPerNode : kCountTotal, reinterpret_cast<unsigned long long*>(T_dev), s,
                get_options());
    if (per_node)
      for (int32_t i = 0; i < k; i++)
        if (graphs[i]->n > 0) {
          k_scatter_by_order<<<grid_for(graphs[i]->n, kBlock, 65536), kBlock, 0, s>>>(
              trp[i], graphs[i]->order.p, graphs[i]->n, reinterpret_cast<unsigned long long*>(t_dev[i]));
          TC_LAUNCH_CHECK();
        }
    for (int32_t i = 0; i < k; i++) note_plan_use(graphs[i]->csr.plan, s);
  });
}

tc_status tc_clustering_from_counts(tc_graph* g, void* stream, const uint64_t* t_dev, uint64_t* num_dev,
                                    uint64_t* den_dev, double* c_dev) {
  return guarded([&] {
    require(g != nullptr && t_dev != nullptr, TC_E_INVAL, "NULL argument");
    require(g->deg.p != nullptr || g->n == 0, TC_E_INVAL, "no degrees on a sampled graph");
    DeviceScope ds(g->device);
    if (g->n > 0) {
      k_clustering<<<grid_for(g->n, kBlock, 65536), kBlock, 0, as_stream(stream)>>>(
          reinterpret_cast<const unsigned long long*>(t_dev), g->deg.p, g->n, num_dev, den_dev, c_dev);
      TC_LAUNCH_CHECK();
    }
    note_plan_use(g->csr.plan, as_stream(stream));
  });
}

tc_status tc_clustering_digest(const uint64_t* num_dev, const uint64_t* den_dev, const double* c_dev, int32_t n,
                               void* stream, uint64_t* digest_dev) {
  return guarded([&] {
    require(digest_dev != nullptr && n >= 0, TC_E_INVAL, "bad argument");
    require(n == 0 || (num_dev && den_dev && c_dev), TC_E_INVAL, "NULL array");
    const hipStream_t s = as_stream(stream);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(digest_dev);
    fill_u64(d, 2, 0ull, s);
    if (n > 0) {
      k_cc_digest<<<grid_for(n, kBlock, 2048), kBlock, 0, s>>>(num_dev, den_dev, c_dev, n, d);
      TC_LAUNCH_CHECK();
    }
  });
}

tc_status tc_sparsify_build(tc_graph* g, double q, uint64_t seed, void* stream, tc_graph** out) {
  return guarded([&] {
    require(g != nullptr && out != nullptr, TC_E_INVAL, "NULL argument");
    require(q > 0.0 && q <= 1.0, TC_E_RANGE, "q outside (0, 1]");
    require(g->order.p != nullptr || g->n == 0, TC_E_INVAL, "cannot sample a sampled graph");
    *out = nullptr;
    DeviceScope ds(g->device);
    const hipStream_t s = as_stream(stream);
    auto* h = new tc_graph();
    try {
      h->device = g->device;
      h->n = g->n;
      h->bits = g->bits;
      h->sampled = true;
      h->q = q;
      HostWords dh(s);  // the sample's longest row, read after the synchronisation below
      build_sampled_csr(g, q, seed, h->csr, s, 0, dh.get());
      h->m = h->csr.m;
      ensure_plan(h->csr, s, get_options());
      TC_HIP(hipStreamSynchronize(s));
      h->csr.dhat_max = static_cast<int32_t>(dh[0]);
    } catch (...) {
      (void)hipStreamSynchronize(s);
      delete h;
      throw;
    }
    *out = h;
  });
}

double tc_sparsify_estimate(uint64_t T_sampled, double q) { return static_cast<double>(T_sampled) / ((q * q) * q); }

tc_status tc_set_option(tc_option key, int64_t value) {
  return guarded([&] {
    require(value >= 0, TC_E_INVAL, "negative option value");
    switch (key) {
      case TC_OPT_KERNEL:
        require(value <= 2, TC_E_INVAL, "kernel must be 0, 1 or 2");
        g_opt_kernel = value;
        break;
      case TC_OPT_HUB_DHAT: g_opt_hub = value; break;
      case TC_OPT_ITEM_WORK: g_opt_iw = value; break;
      case TC_OPT_BLOCKS_PER_CU:
        require(value >= 1, TC_E_INVAL, "blocks per CU must be >= 1");
        g_opt_bpc = value;
        break;
      case TC_OPT_HUB_BUCKET_LOAD:
        require(value == 1 || value == 2, TC_E_INVAL, "bucket load must be 1 or 2");
        g_opt_load = value;
        break;
      case TC_OPT_ORDER:
        require(value <= 4, TC_E_INVAL,
                "order must be 0 (degree), 1 (id), 2 (random), 3 (degree descending) or 4 (coreness)");
        g_opt_order = value;
        break;
      default: fail(TC_E_INVAL, "unknown option");
    }
  });
}

int64_t tc_get_option(tc_option key) {
  switch (key) {
    case TC_OPT_KERNEL: return g_opt_kernel.load();
    case TC_OPT_HUB_DHAT: return g_opt_hub.load();
    case TC_OPT_ITEM_WORK: return g_opt_iw.load();
    case TC_OPT_BLOCKS_PER_CU: return g_opt_bpc.load();
    case TC_OPT_HUB_BUCKET_LOAD: return g_opt_load.load();
    case TC_OPT_ORDER: return g_opt_order.load();
    default: return -1;
  }
}

const char* tc_status_str(tc_status s) {
  switch (s) {
    case TC_OK: return "TC_OK";
    case TC_E_INVAL: return "TC_E_INVAL";
    case TC_E_NOMEM: return "TC_E_NOMEM";
    case TC_E_DEVICE: return "TC_E_DEVICE";
    case TC_E_RANGE: return "TC_E_RANGE";
    case TC_E_TRUNC: return "TC_E_TRUNC";
    default: return "TC_E_UNKNOWN";
  }
}

const char* tc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
