// Exact triangle count of an oriented CSR that stays in host memory: the
// non-overlapping partitions of Section 6 streamed through one GPU.
//
// The oriented CSR in rank space (row r holds later ranks, ascending) stays
// on the host. The rows are split into pivot partitions V_j, each sized to
// half of the device budget. For each j, the rows of V_j are loaded once and
// serve as their own sources. The rows before V_j are then shipped to it in
// chunks sized to the other half: the surrogate pairing of Section 6, where
// N_v travels to the partition owning u once per (chunk, partition), and not
// once per edge. Triangle (v,u,w), v < u < w, is counted where u lives:
// |N_v after u ∩ N_u| from the in-edge record (v,u), by the pivot kernel of
// the in-memory path. Each (source rows, partition) pair is visited once, and
// each triangle is counted once.
//
// Device layout of one (partition, chunk) pair, one CSR with local rows:
//   rows [0, np)            the rows of V_j (adj entries [0, ep))
//   row  np                 an empty gap spanning [ep, cap_p)
//   rows (np, np + 1 + nc]  a shipped chunk's rows (adj entries from cap_p)
// Resident sources use rows [0, np) alone.
// Entries keep their global ranks, and the pivot kernel only compares them.
// Records (v,u) are keyed by u's local row. The next chunk is copied into a
// staging buffer on a second stream while the current pair is counted. A
// partition is loaded on a third stream, one resident range at a time, last
// range first: the pair of a resident range reads only its own range and the
// ones after it, so it is counted while the ranges before it are still coming.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "graph.hpp"
#include "primitives.hpp"

namespace tc {
namespace {

constexpr int kBlock = 256;

// Device bytes per entry and per row: a pivot partition holds adj, src, off,
// the in-edge offsets and the classification arrays; a chunk adds its staged
// copy, the two key and two suffix-length buffers of the record sort, the
// records and their costs.
constexpr uint64_t kPivotEntryBytes = 8;
constexpr uint64_t kPivotRowBytes = 48;
constexpr uint64_t kChunkEntryBytes = 64;
constexpr uint64_t kChunkRowBytes = 56;
constexpr int64_t kMaxRegionEntries = int64_t(1) << 31;  // record keys hold 32-bit entry indices

// dst[r] = base + clamp(off[r] - o0, c0, c1) for r in [0, rows]; flags offsets
// that decrease. The host has checked only the range's end offsets, and knows
// the entries [c0, c1) that the range spans; an offset between them that breaks
// the order is clamped into that span, so nothing reads outside the range's own
// entries before the flag is seen.
__global__ void k_rebase(const int64_t* __restrict__ off, int32_t rows, int64_t o0, int64_t c0, int64_t c1,
                         int64_t base, int64_t* __restrict__ dst, uint32_t* __restrict__ bad) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r <= rows; r += gridDim.x * blockDim.x) {
    const int64_t x = off[r] - o0;
    dst[r] = base + (x < c0 ? c0 : x > c1 ? c1 : x);
    if (r < rows && off[r + 1] < off[r]) atomicOr(bad, 1u);
  }
}

// Checks the rows [0, rows) of a region (global row of local row r: g0 + r):
// entries strictly ascending, above their own row, below n. With src, writes
// the local row (row_base + r) of every entry. Each wave takes groups of 32
// consecutive rows and walks their entries 64 at a time, so a long row is
// shared by the whole wave; an entry finds its row among the group's 33
// offsets (lane i holds the start of row i) by a 5-step search over shuffles.
// The offsets are non-decreasing (the caller checks them on the host).
__global__ void k_check_rows(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t rows,
                             int32_t row_base, int32_t g0, int32_t n, int32_t* __restrict__ src,
                             uint32_t* __restrict__ bad) {
  constexpr int kGroup = 32;
  const int lane = lane_id();
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  bool ok = true;
  for (int64_t r0 = wave * kGroup; r0 < rows; r0 += nwaves * kGroup) {
    const int rl = static_cast<int>(rows - r0 < kGroup ? rows - r0 : kGroup);
    const int64_t mine = lane <= rl ? off[row_base + r0 + lane] : 0;
    const int64_t b = __shfl(mine, 0, kWave), e = __shfl(mine, rl, kWave);
    for (int64_t base = b; base < e; base += kWave) {  // uniform: every lane takes part in the shuffles
      const int64_t k = base + lane;
      int row = 0;
#pragma unroll
      for (int step = kGroup / 2; step > 0; step >>= 1) {
        const int cand = row + step;
        const int64_t start = __shfl(mine, cand < rl ? cand : 0, kWave);
        if (cand < rl && start <= k) row = cand;
      }
      const int64_t start = __shfl(mine, row, kWave);
      if (k < e) {
        const int32_t x = adj[k];
        const int32_t prev = k == start ? g0 + static_cast<int32_t>(r0) + row : adj[k - 1];
        ok = ok && x > prev && x < n;
        if (src) src[k] = row_base + static_cast<int32_t>(r0) + row;
      }
    }
  }
  if (!ok) atomicOr(bad, 2u);
}

// Record keys of the chunk entries that point into V_j = [lo, hi):
// (u - lo) << 32 | e, e the entry's index in the combined adj.
struct IntoPivots {
  const int32_t* adj;
  int64_t e0;
  int32_t lo, hi;
  __device__ bool operator()(size_t i) const {
    const int32_t x = adj[e0 + static_cast<int64_t>(i)];
    return x >= lo && x < hi;
  }
};
struct PivotKey {
  const int32_t* adj;
  int64_t e0;
  int32_t lo;
  __device__ uint64_t operator()(size_t i) const {
    const int64_t e = e0 + static_cast<int64_t>(i);
    return (static_cast<uint64_t>(static_cast<uint32_t>(adj[e] - lo)) << 32) | static_cast<uint64_t>(e);
  }
};

// |N_v after u| of the record of entry e = e0 + i: the rest of e's row, read
// in entry order (the records are then sorted with it as their value).
struct SuffixLen {
  const int64_t* off;
  const int32_t* src;
  int64_t e0;
  __device__ uint32_t operator()(size_t i) const {
    const int64_t e = e0 + static_cast<int64_t>(i);
    return static_cast<uint32_t>(off[src[e] + 1] - e - 1);
  }
};

struct Range {
  int32_t lo, hi;
  int64_t e0, e1;  // entries [off[lo], off[hi])
};

// Splits rows [lo, hi) into consecutive ranges of cost eb * entries + rb * rows
// <= cap (greedy, each range as long as fits); fails if one row alone exceeds it.
std::vector<Range> split_rows(const int64_t* off, int32_t lo, int32_t hi, uint64_t cap, uint64_t eb, uint64_t rb) {
  std::vector<Range> out;
  auto cost = [&](int32_t a, int32_t b) {
    return eb * static_cast<uint64_t>(off[b] - off[a]) + rb * static_cast<uint64_t>(b - a);
  };
  while (lo < hi) {
    if (off[lo + 1] < off[lo]) fail(TC_E_INVAL, "row offsets must not decrease");
    if (cost(lo, lo + 1) > cap || off[lo + 1] - off[lo] >= kMaxRegionEntries)
      fail(TC_E_NOMEM, "device budget too small for one adjacency row");
    int32_t a = lo + 1, b = hi;  // the largest end in [lo+1, hi] that fits
    while (a < b) {
      const int32_t mid = a + (b - a + 1) / 2;
      if (cost(lo, mid) <= cap && off[mid] - off[lo] < kMaxRegionEntries) a = mid;
      else b = mid - 1;
    }
    // the ends of every range run from 0 to m without decreasing (the offsets inside a
    // range are checked on the device)
    if (off[a] < off[lo]) fail(TC_E_INVAL, "row offsets must not decrease");
    out.push_back(Range{lo, a, off[lo], off[a]});
    lo = a;
  }
  return out;
}

// One visit: the records (v,u) with v in rows `src` and u in pivot partition
// `part`; shipped sources come through the staging buffer, resident ones are
// rows of the partition itself.
struct Task {
  int part;
  bool shipped;
  Range src;
};

// A CSR whose arrays belong to someone else (cleared before destruction).
struct CsrView {
  Csr c;
  CsrView(int64_t* off, int32_t* adj, int32_t* src) {
    c.off.p = off;
    c.adj.p = adj;
    c.src.p = src;
  }
  ~CsrView() {
    c.off.p = nullptr;
    c.adj.p = nullptr;
    c.src.p = nullptr;
  }
};

}  // namespace

uint64_t count_streamed(const int64_t* off, const int32_t* adj, int32_t n, int64_t m, uint64_t budget,
                        hipStream_t s, const Options& o, uint64_t info[4]) {
  info[0] = info[1] = info[2] = info[3] = 0;
  if (n <= 0 || m == 0) return 0;
  const std::vector<Range> parts = split_rows(off, 0, n, budget / 2, kPivotEntryBytes, kPivotRowBytes);
  // visiting order: for each partition, its own rows (resident) from the last
  // range to the first, and then the rows before it, shipped in chunks. A
  // resident range's records point only at rows after its first row, so its
  // pair needs only the ranges visited so far: the partition is loaded in the
  // same order, range by range, and each pair starts once its own range is in.
  std::vector<Task> tasks;
  size_t own_max = 1;
  for (int j = 0; j < static_cast<int>(parts.size()); j++) {
    const std::vector<Range> own =
        split_rows(off, parts[j].lo, parts[j].hi, budget / 2, kChunkEntryBytes, kChunkRowBytes);
    own_max = std::max(own_max, own.size());
    for (auto r = own.rbegin(); r != own.rend(); ++r) tasks.push_back(Task{j, false, *r});
    for (const Range& r : split_rows(off, 0, parts[j].lo, budget / 2, kChunkEntryBytes, kChunkRowBytes))
      tasks.push_back(Task{j, true, r});
  }
  int64_t cap_p = 0, cap_c = 0;
  int32_t rows_p = 0, rows_c = 0;
  for (const Range& r : parts) {
    cap_p = std::max(cap_p, r.e1 - r.e0);
    rows_p = std::max(rows_p, r.hi - r.lo);
  }
  for (const Task& t : tasks) {
    if (!t.shipped) continue;
    cap_c = std::max(cap_c, t.src.e1 - t.src.e0);
    rows_c = std::max(rows_c, t.src.hi - t.src.lo);
    info[1]++;
  }
  info[0] = parts.size();
  info[2] = tasks.size();

  DevBuf<int32_t> adj_d(static_cast<size_t>(cap_p + cap_c), s), src_d(static_cast<size_t>(cap_p + cap_c), s);
  DevBuf<int64_t> off_d(static_cast<size_t>(rows_p) + rows_c + 3, s);
  DevBuf<int32_t> stage_adj(static_cast<size_t>(cap_c), s);
  DevBuf<int64_t> stage_off(static_cast<size_t>(rows_c) + 1, s), pin_off(static_cast<size_t>(rows_p) + 1, s);
  DevBuf<unsigned long long> total(1, s);
  DevBuf<uint32_t> bad(1, s);
  fill_u64(total.get(), 1, 0ull, s);
  k_fill_words<uint32_t><<<1, 64, 0, s>>>(bad.get(), 1, 0u);
  TC_LAUNCH_CHECK();

  // cs ships chunks into the staging buffers, ls loads the partitions
  hipStream_t cs = nullptr, ls = nullptr;
  TC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipEvent_t loaded = nullptr, freed = nullptr, part_free = nullptr;
  std::vector<hipEvent_t> range_in(own_max, nullptr);  // range k of the partition being loaded is in
  auto cleanup = [&] {
    (void)hipStreamSynchronize(cs);
    if (ls) (void)hipStreamSynchronize(ls);
    (void)hipStreamSynchronize(s);
    if (loaded) (void)hipEventDestroy(loaded);
    if (freed) (void)hipEventDestroy(freed);
    if (part_free) (void)hipEventDestroy(part_free);
    for (hipEvent_t e : range_in)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(cs);
    if (ls) (void)hipStreamDestroy(ls);
  };
  HostWords hw(s);
  try {
    TC_HIP(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
    TC_HIP(hipEventCreateWithFlags(&loaded, hipEventDisableTiming));
    TC_HIP(hipEventCreateWithFlags(&freed, hipEventDisableTiming));
    TC_HIP(hipEventCreateWithFlags(&part_free, hipEventDisableTiming));
    for (hipEvent_t& e : range_in) TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    uint64_t h2d = 0;
    auto next_shipped = [&](size_t from) {
      while (from < tasks.size() && !tasks[from].shipped) from++;
      return from;
    };
    auto prefetch = [&](size_t q) {  // task q's rows into the staging buffers, on the copy stream
      if (q >= tasks.size()) return;
      const Range& r = tasks[q].src;
      TC_HIP(hipStreamWaitEvent(cs, freed, 0));
      if (r.e1 > r.e0)
        TC_HIP(hipMemcpyAsync(stage_adj.get(), adj + r.e0, static_cast<size_t>(r.e1 - r.e0) * sizeof(int32_t),
                              hipMemcpyDefault, cs));
      TC_HIP(hipMemcpyAsync(stage_off.get(), off + r.lo, (static_cast<size_t>(r.hi - r.lo) + 1) * sizeof(int64_t),
                            hipMemcpyDefault, cs));
      TC_HIP(hipEventRecord(loaded, cs));
      h2d += static_cast<uint64_t>(r.e1 - r.e0) * sizeof(int32_t) + (static_cast<uint64_t>(r.hi - r.lo) + 1) * 8;
    };
    TC_HIP(hipEventRecord(freed, s));
    prefetch(next_shipped(0));
    int cur_part = -1;
    int32_t dhat_p = 0;  // the longest row among the partition's ranges loaded so far
    size_t own_k = 0;    // the resident range's place in the partition's loading order
    CountArgs ca;
    ca.mode = kCountTotal;
    ca.total = total.get();
    for (size_t q = 0; q < tasks.size(); q++) {
      const Task& t = tasks[q];
      const Range& P = parts[t.part];
      const Range& C = t.src;
      const int32_t np = P.hi - P.lo, nc = C.hi - C.lo;
      if (t.part != cur_part) {  // load the rows of V_j on ls, range by range in visiting order
        cur_part = t.part;
        dhat_p = 0;
        own_k = 0;
        TC_HIP(hipEventRecord(part_free, s));  // after the last count that reads the previous partition
        TC_HIP(hipStreamWaitEvent(ls, part_free, 0));
        for (size_t k = 0; q + k < tasks.size() && tasks[q + k].part == t.part && !tasks[q + k].shipped; k++) {
          const Range& R = tasks[q + k].src;
          const int32_t r0 = R.lo - P.lo;
          const size_t nrow = static_cast<size_t>(R.hi - R.lo) + (R.hi == P.hi ? 1 : 0);  // the end once
          if (R.e1 > R.e0)
            TC_HIP(hipMemcpyAsync(adj_d.get() + (R.e0 - P.e0), adj + R.e0,
                                  static_cast<size_t>(R.e1 - R.e0) * sizeof(int32_t), hipMemcpyDefault, ls));
          TC_HIP(hipMemcpyAsync(pin_off.get() + r0, off + R.lo, nrow * sizeof(int64_t), hipMemcpyDefault, ls));
          TC_HIP(hipEventRecord(range_in[k], ls));
          h2d += static_cast<uint64_t>(R.e1 - R.e0) * sizeof(int32_t) + nrow * 8;
        }
      }
      CsrView w(off_d.get(), adj_d.get(), src_d.get());
      int64_t e_begin = 0;  // the source entries in the combined adj
      uint64_t ec = static_cast<uint64_t>(C.e1 - C.e0);
      if (t.shipped) {  // the staged rows after the gap row np
        TC_HIP(hipStreamWaitEvent(s, loaded, 0));
        if (ec)
          TC_HIP(hipMemcpyAsync(adj_d.get() + cap_p, stage_adj.get(), ec * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                s));
        k_rebase<<<grid_for(static_cast<uint64_t>(nc) + 1, kBlock, 65536), kBlock, 0, s>>>(
            stage_off.get(), nc, C.e0, 0, C.e1 - C.e0, cap_p, off_d.get() + np + 1, bad.get());
        TC_LAUNCH_CHECK();
        TC_HIP(hipEventRecord(freed, s));
        prefetch(next_shipped(q + 1));
        k_check_rows<<<grid_for(nc, kBlock, 65536), kBlock, 0, s>>>(off_d.get(), adj_d.get(), nc, np + 1, C.lo, n,
                                                                    src_d.get(), bad.get());
        TC_LAUNCH_CHECK();
        w.c.n = np + 1 + nc;
        w.c.m = cap_p + static_cast<int64_t>(ec);
        e_begin = cap_p;
      } else {  // rows of the partition itself: its range (the ranges after it are in and checked)
        w.c.n = np;
        w.c.m = P.e1 - P.e0;
        e_begin = C.e0 - P.e0;
        const int32_t r0 = C.lo - P.lo;
        TC_HIP(hipStreamWaitEvent(s, range_in[own_k++], 0));
        k_rebase<<<grid_for(static_cast<uint64_t>(nc) + 1, kBlock, 65536), kBlock, 0, s>>>(
            pin_off.get() + r0, nc, P.e0, C.e0 - P.e0, C.e1 - P.e0, 0, off_d.get() + r0, bad.get());
        TC_LAUNCH_CHECK();
        k_check_rows<<<grid_for(nc, kBlock, 65536), kBlock, 0, s>>>(off_d.get(), adj_d.get(), nc, r0, C.lo, n,
                                                                    src_d.get(), bad.get());
        TC_LAUNCH_CHECK();
        row_max_to_host(off_d.get() + r0, nc, s, hw.get() + 2);
      }
      // records (v,u) with u in V_j, sorted by u's local row (the row check is read back
      // with their count, before anything indexes by an entry's value)
      DevBuf<uint64_t> keys(ec, s), keys2(ec, s), cnt(2, s);
      DevBuf<uint32_t> lens(ec, s), lens2(ec, s);
      const IntoPivots into{adj_d.get(), e_begin, P.lo, P.hi};
      compact_if<uint64_t>(ec, into, PivotKey{adj_d.get(), e_begin, P.lo}, keys.get(), cnt.get(), s);
      compact_if<uint32_t>(ec, into, SuffixLen{off_d.get(), src_d.get(), e_begin}, lens.get(), cnt.get() + 1, s);
      hw.get()[1] = 0;
      TC_HIP(hipMemcpyAsync(hw.get(), cnt.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipMemcpyAsync(hw.get() + 1, bad.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      if (hw[1]) fail(TC_E_INVAL, "rows must hold ascending ranks above their own row, below n");
      if (!t.shipped) dhat_p = std::max(dhat_p, static_cast<int32_t>(hw[2]));
      w.c.dhat_max = dhat_p;  // pivots of this pair lie in the ranges loaded so far
      const uint64_t mi = hw[0];
      if (mi == 0) continue;
      const int b = bits_for(np > 1 ? static_cast<uint64_t>(np - 1) : 1);
      uint32_t* sl = lens.get();
      uint64_t* sk = radix_sort_pairs<uint64_t, uint32_t>(keys.get(), keys2.get(), sl, lens2.get(), mi, 32, 32 + b, s);
      PivotPlan plan;
      DevBuf<int64_t> fin;
      plan_records(w.c, plan, sk, sl, mi, fin, s);
      keys.release();
      keys2.release();
      lens.release();
      lens2.release();
      plan_items(w.c, plan, fin.get(), mi, s, o);
      fin.release();
      launch_pivot(w.c, plan, ca, s, o);
      plan.release_on(s);  // freed in stream order after the count: no host wait per pair
    }
    info[3] = h2d;
    unsigned long long T = 0;
    TC_HIP(hipMemcpyAsync(&T, total.get(), sizeof(T), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    cleanup();
    return T;
  } catch (...) {
    cleanup();
    throw;
  }
}

}  // namespace tc
