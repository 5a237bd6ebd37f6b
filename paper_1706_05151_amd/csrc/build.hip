// Device construction of the oriented CSR used by NodeIteratorN.
//
// Steps (the preprocessing of the NodeIteratorN figure, Section 3):
//   1. canonical keys lo<<b|hi per edge record; loops and bad ids flagged
//   2. radix sort; duplicates are found as equal neighbours -> the simple
//      graph of Section 2 (m edges)
//   3. degrees d_v: the larger endpoints are counted halfway through the sort,
//      when the keys are ordered by their low bits (duplicates included, taken
//      off once the sort is done); the smaller endpoints from runs of the
//      sorted unique keys
//   4. ranks: position of each vertex in the degree order of Eq. (1)
//      (d ascending, ties by id; graphs of a batch kept contiguous)
//   5. relabel every unique edge to (min rank, max rank) while compacting --
//      the orientation of Eq. (1), because the earlier endpoint has the
//      smaller rank -- and radix sort, which yields every N_v ascending,
//      grouped by row
//   6. CSR offsets, row ids, d_max and dhat_max
#include <vector>

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

// Adds sign times the run's length to deg[v] with one atomic, for each run of
// lanes holding the same value v >= 0 (values < 0 break runs and are not counted).
__device__ __forceinline__ void add_runs(int32_t v, int32_t* __restrict__ deg, int sign = 1) {
  const int lane = lane_id();
  const int32_t prev = __shfl_up(v, 1, kWave);
  const uint64_t bounds = __ballot(lane == 0 || prev != v);
  if (v >= 0 && (lane == 0 || prev != v)) {
    const uint64_t above = bounds & ~((2ull << lane) - 1ull);  // run starts after this lane (lane 63: none)
    const int end = above ? __ffsll(static_cast<long long>(above)) - 1 : kWave;
    atomicAdd(&deg[v], sign * (end - lane));
  }
}

// Larger endpoints of the canonical keys, which are ordered by their low bits
// (the larger endpoint comes first in them): each run adds its length to the
// endpoint's degree. Duplicate records are counted here and taken off by
// k_dedup_degrees; flagged records (~0) are skipped.
__global__ __launch_bounds__(kBlock) void k_larger_end_runs(const uint64_t* __restrict__ keys, uint64_t E,
                                                             uint64_t hmask, int32_t* __restrict__ deg) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x; i0 < E; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    const uint64_t k = i < E ? keys[i] : ~0ull;
    add_runs(k != ~0ull ? static_cast<int32_t>(k & hmask) : -1, deg);
  }
}

// Over the sorted canonical keys, in the layout of the compaction flags
// (wave w of block x covers words (4x + w) * kFlagWords ... of 64 keys):
// a key is kept iff it is valid and differs from its predecessor; the ballot
// of each word and the block's kept count are stored for k_flag_compact.
// Each run of equal smaller endpoints adds its kept keys to that endpoint's
// degree with one atomic. The larger endpoint of every repeat (a valid key
// that is not kept) is written to dup_hi (one reservation per block): those
// were counted once too often by k_larger_end_runs and are taken off after a
// sort (k_sub_sorted_runs), which groups the repeats of hub vertices instead of
// sending each to the same counter.
__global__ __launch_bounds__(kScanBlock) void k_dedup_degrees(const uint64_t* __restrict__ keys, uint64_t E, int b,
                                                             int32_t* __restrict__ deg, uint64_t* __restrict__ flags,
                                                             uint64_t* __restrict__ counts,
                                                             uint32_t* __restrict__ dup_hi,
                                                             unsigned long long* __restrict__ dup_count) {
  __shared__ uint64_t sm[kFlagWaves];
  __shared__ uint32_t sdup[kFlagWaves * kFlagWords * kWave];
  __shared__ uint32_t sdn;
  __shared__ unsigned long long sbase;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const uint64_t hmask = (1ull << b) - 1;
  const size_t word0 = (static_cast<size_t>(blockIdx.x) * kFlagWaves + w) * kFlagWords;
  if (threadIdx.x == 0) sdn = 0;
  __syncthreads();
  uint64_t c = 0;
  for (int j = 0; j < kFlagWords; j++) {
    const size_t i = (word0 + j) * kWave + lane;
    const uint64_t k = i < E ? keys[i] : ~0ull;
    uint64_t prev = __shfl_up(k, 1, kWave);
    if (lane == 0) prev = i > 0 && i - 1 < E ? keys[i - 1] : ~0ull;
    const bool valid = k != ~0ull;
    const bool kept = valid && (i == 0 || k != prev);
    const uint64_t bal = __ballot(kept);
    if (lane == 0) flags[word0 + j] = bal;
    c += static_cast<uint64_t>(__popcll(bal));
    const uint64_t dups = __ballot(valid && !kept);
    if (dups) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&sdn, static_cast<uint32_t>(__popcll(dups)));
      base = __shfl(base, 0, kWave);
      if (valid && !kept) sdup[base + __popcll(dups & lanemask_lt())] = static_cast<uint32_t>(k & hmask);
    }
    // runs of equal smaller endpoints over the valid keys, counting the kept ones
    const int32_t v = valid ? static_cast<int32_t>(k >> b) : -1;
    const int32_t pv = __shfl_up(v, 1, kWave);
    const bool head = lane == 0 || pv != v;
    const uint64_t bounds = __ballot(head);
    if (v >= 0 && head) {
      const uint64_t above = bounds & ~((2ull << lane) - 1ull);
      const int end = above ? __ffsll(static_cast<long long>(above)) - 1 : kWave;
      const uint64_t run = (end == kWave ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull);
      const int kept_in_run = __popcll(bal & run);
      if (kept_in_run) atomicAdd(&deg[v], kept_in_run);
    }
  }
  if (lane == 0) sm[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int x = 0; x < kFlagWaves; x++) t += sm[x];
    counts[blockIdx.x] = t;
    sbase = sdn ? atomicAdd(dup_count, static_cast<unsigned long long>(sdn)) : 0ull;
  }
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < sdn; x += kScanBlock) dup_hi[sbase + x] = sdup[x];
}

// deg[v] -= number of entries equal to v, over sorted 32-bit values
__global__ __launch_bounds__(kBlock) void k_sub_sorted_runs(const uint32_t* __restrict__ vals, uint64_t N,
                                                            int32_t* __restrict__ deg) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x; i0 < N; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    add_runs(i < N ? static_cast<int32_t>(vals[i]) : -1, deg, -1);
  }
}

// The repeats' larger endpoints (ndup of them at dup, with room for as many
// again after them) sorted and taken off the degrees.
void take_off_repeats(uint32_t* dup, uint64_t ndup, int b, int32_t* deg, hipStream_t s, uint32_t* fail) {
  if (ndup == 0) return;
  const uint32_t* sorted = radix_sort<uint32_t>(dup, dup + ndup, ndup, 0, b, s, fail);
  k_sub_sorted_runs<<<grid_for(ndup, kBlock, 65536), kBlock, 0, s>>>(sorted, ndup, deg);
  TC_LAUNCH_CHECK();
}

// The orientation of Eq. (1) for kept key i: the endpoint earlier in the
// degree order has the smaller rank and becomes the row.
struct RelabelKey {
  const uint64_t* k;
  int b;
  const int32_t* rank;
  __device__ uint64_t operator()(size_t i) const {
    const uint64_t key = k[i];
    const uint64_t mask = (1ull << b) - 1;
    const uint64_t ra = static_cast<uint64_t>(rank[key >> b]), rb = static_cast<uint64_t>(rank[key & mask]);
    return ra < rb ? ((ra << b) | rb) : ((rb << b) | ra);
  }
};

// Queues the degree count of the larger endpoints after the sort pass that
// completes their bits.
struct LargerEndHook {
  int last_pass;
  uint64_t E;
  uint64_t hmask;
  int32_t* deg;
  hipStream_t s;
  void operator()(int p, const uint64_t* keys) const {
    if (p != last_pass) return;
    k_larger_end_runs<<<grid_for(E, kBlock, 65536), kBlock, 0, s>>>(keys, E, hmask, deg);
    TC_LAUNCH_CHECK();
  }
};

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

// ---- the oriented lists sorted in place. The keys (row << b | col) are
// grouped by row (rows ascending, columns in any order); each row's columns
// are sorted and written out as the row's CSR entries (adj = column, src =
// row). A row holds at most dhat_max entries, so it fits one wave or one
// block's LDS and needs no global pass over the column bits.

int device_cus() {
  int dev = 0, cus = 0;
  TC_HIP(hipGetDevice(&dev));
  TC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus > 0 ? cus : 1;
}

constexpr int kSegBlock = 256;
constexpr int kSegBlockMax = 4096;  // longest row a block sorts in LDS

// Bitonic sort of one value per lane, ascending with the lane index.
__device__ __forceinline__ uint32_t wave_bitonic_sort(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t y = __shfl_xor(x, j, kWave);
      // the lower lane of an ascending pair, or the upper lane of a descending one, keeps the minimum
      x = (((lane & j) == 0) == ((lane & k) == 0)) ? (x < y ? x : y) : (x < y ? y : x);
    }
  }
  return x;
}

// Sorting network of 8 inputs (Batcher's odd-even merge sort, 19 comparators), ascending.
__device__ __forceinline__ void sort8(uint32_t (&x)[8]) {
  constexpr int kPairs[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                 {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int c = 0; c < 19; c++) {
    const uint32_t a = x[kPairs[c][0]], b = x[kPairs[c][1]];
    x[kPairs[c][0]] = a < b ? a : b;
    x[kPairs[c][1]] = a < b ? b : a;
  }
}

// Rows of at most 64 entries: each wave takes rpw consecutive rows (rpw a
// power of two up to 64, smaller for small graphs so that their rows spread
// over more waves); a row of 1..8 entries is sorted by its own lane in
// registers, a row of 9..64 entries by the whole wave (one entry per lane).
// Longer rows are left to k_seg_rows_wide and k_seg_rows_block.
__global__ __launch_bounds__(kSegBlock) void k_seg_rows_wave(const uint64_t* __restrict__ keys,
                                                           const int64_t* __restrict__ off, int32_t n, int b, int rpw,
                                                           int32_t* __restrict__ adj, int32_t* __restrict__ src) {
  const uint32_t mask = static_cast<uint32_t>((1ull << b) - 1);
  const int lane = lane_id();
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kSegBlock / kWave) + threadIdx.x / kWave;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (kSegBlock / kWave) * rpw;
  for (int64_t r0 = wave * rpw; r0 < n; r0 += stride) {
    const int64_t r = r0 + lane;
    int64_t o = 0, len = 0;
    if (lane < rpw && r < n) {
      o = off[r];
      len = off[r + 1] - o;
    }
    if (len >= 1 && len <= 8) {
      uint32_t x[8];
#pragma unroll
      for (int e = 0; e < 8; e++) x[e] = e < len ? (static_cast<uint32_t>(keys[o + e]) & mask) : 0xFFFFFFFFu;
      sort8(x);
#pragma unroll
      for (int e = 0; e < 8; e++) {
        if (e < len) {
          adj[o + e] = static_cast<int32_t>(x[e]);
          src[o + e] = static_cast<int32_t>(r);
        }
      }
    }
    uint64_t todo = __ballot(len > 8 && len <= kWave);
    while (todo) {
      const int l = __ffsll(static_cast<long long>(todo)) - 1;
      todo &= todo - 1;
      const int64_t ro = __shfl(o, l, kWave);
      const int rl = __shfl(static_cast<int>(len), l, kWave);
      uint32_t x = lane < rl ? (static_cast<uint32_t>(keys[ro + lane]) & mask) : 0xFFFFFFFFu;
      x = wave_bitonic_sort(x);
      if (lane < rl) {
        adj[ro + lane] = static_cast<int32_t>(x);
        src[ro + lane] = static_cast<int32_t>(r0 + l);
      }
    }
  }
}

// Bitonic sort of one row of at most 64 R entries held by one wave, entry
// s * 64 + lane in x[s] of that lane: pairs closer than 64 exchange through
// lane shuffles, farther ones within a lane's registers. Padding (all ones)
// sorts last: columns are below 2^31.
template <int R>
__device__ __forceinline__ void wave_sort_row(const uint64_t* __restrict__ keys, int64_t o, int len, uint32_t mask,
                                              int32_t row, int32_t* __restrict__ adj, int32_t* __restrict__ src) {
  constexpr int P = R * kWave;
  const int lane = lane_id();
  uint32_t x[R];
#pragma unroll
  for (int s = 0; s < R; s++) {
    const int e = s * kWave + lane;
    x[s] = e < len ? (static_cast<uint32_t>(keys[o + e]) & mask) : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= kWave) {
        const int js = j / kWave;
#pragma unroll
        for (int s = 0; s < R; s++) {
          if ((s & js) == 0) {  // slots s and s | js hold the pair
            const bool up = ((s * kWave + lane) & k) == 0;
            const uint32_t a = x[s], c = x[s | js];
            const bool sw = (a > c) == up;
            x[s] = sw ? c : a;
            x[s | js] = sw ? a : c;
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < R; s++) {
          const uint32_t y = __shfl_xor(x[s], j, kWave);
          const bool up = ((s * kWave + lane) & k) == 0;
          x[s] = (((lane & j) == 0) == up) ? (x[s] < y ? x[s] : y) : (x[s] < y ? y : x[s]);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < R; s++) {
    const int e = s * kWave + lane;
    if (e < len) {
      adj[o + e] = static_cast<int32_t>(x[s]);
      src[o + e] = row;
    }
  }
}

constexpr int kSegWideMax = 16 * kWave;  // longest row one wave sorts in registers

// Rows of 65..kSegWideMax entries, from a list: one wave per row.
__global__ __launch_bounds__(kSegBlock) void k_seg_rows_wide(const uint64_t* __restrict__ keys,
                                                           const int64_t* __restrict__ off,
                                                           const int32_t* __restrict__ rows,
                                                           const uint64_t* __restrict__ nrows, int b,
                                                           int32_t* __restrict__ adj, int32_t* __restrict__ src) {
  const uint32_t mask = static_cast<uint32_t>((1ull << b) - 1);
  const uint64_t cnt = *nrows;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * (kSegBlock / kWave);
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * (kSegBlock / kWave) + threadIdx.x / kWave; i < cnt;
       i += stride) {
    const int32_t r = rows[i];
    const int64_t o = off[r];
    const int len = static_cast<int>(off[r + 1] - o);
    if (len <= 2 * kWave) wave_sort_row<2>(keys, o, len, mask, r, adj, src);
    else if (len <= 4 * kWave) wave_sort_row<4>(keys, o, len, mask, r, adj, src);
    else if (len <= 8 * kWave) wave_sort_row<8>(keys, o, len, mask, r, adj, src);
    else wave_sort_row<16>(keys, o, len, mask, r, adj, src);
  }
}

// Rows of kSegWideMax+1..kSegBlockMax entries, from a list: one block per row,
// bitonic sort in LDS over the row padded to a power of two.
__global__ __launch_bounds__(kSegBlock) void k_seg_rows_block(const uint64_t* __restrict__ keys,
                                                            const int64_t* __restrict__ off,
                                                            const int32_t* __restrict__ rows,
                                                            const uint64_t* __restrict__ nrows, int b,
                                                            int32_t* __restrict__ adj, int32_t* __restrict__ src) {
  __shared__ uint32_t t[kSegBlockMax];
  const uint32_t mask = static_cast<uint32_t>((1ull << b) - 1);
  const uint64_t cnt = *nrows;
  for (uint64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int32_t r = rows[i];
    const int64_t o = off[r];
    const int len = static_cast<int>(off[r + 1] - o);
    int P = 2 * kSegWideMax;
    while (P < len) P <<= 1;
    for (int x = threadIdx.x; x < P; x += kSegBlock)
      t[x] = x < len ? (static_cast<uint32_t>(keys[o + x]) & mask) : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int x = threadIdx.x; x < P / 2; x += kSegBlock) {
          const int lo = ((x & ~(j - 1)) << 1) | (x & (j - 1));  // pair (lo, lo + j), bit j of lo clear
          const uint32_t a = t[lo], c = t[lo + j];
          if ((a > c) == ((lo & k) == 0)) {
            t[lo] = c;
            t[lo + j] = a;
          }
        }
        __syncthreads();
      }
    }
    for (int x = threadIdx.x; x < len; x += kSegBlock) {
      adj[o + x] = static_cast<int32_t>(t[x]);
      src[o + x] = r;
    }
    __syncthreads();
  }
}

struct RowsBetween {  // rows with lo < length <= hi
  const int64_t* off;
  int64_t lo, hi;
  __device__ bool operator()(size_t r) const {
    const int64_t d = off[r + 1] - off[r];
    return d > lo && d <= hi;
  }
};
struct RowIndex {
  __device__ int32_t operator()(size_t r) const { return static_cast<int32_t>(r); }
};

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
struct RowOfKey {
  const uint64_t* k;
  int b;
  __device__ int64_t operator()(uint64_t i) const { return static_cast<int64_t>(k[i] >> b); }
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

void row_max_to_host(const int64_t* off, int32_t n, hipStream_t s, uint64_t* host) {
  DevBuf<uint64_t> mx(1, s);
  k_fill_words<uint64_t><<<1, 64, 0, s>>>(mx.get(), 1, 0ull);
  TC_LAUNCH_CHECK();
  if (n > 0) {
    k_row_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(off, n, reinterpret_cast<int*>(mx.get()));
    TC_LAUNCH_CHECK();
  }
  TC_HIP(hipMemcpyAsync(host, mx.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
}

int32_t max_row_length(const int64_t* off, int32_t n, hipStream_t s) {
  HostWords h(s);
  row_max_to_host(off, n, s, h.get());
  TC_HIP(hipStreamSynchronize(s));
  return static_cast<int32_t>(h[0]);
}

void build_graph_finish(tc_graph* g, const uint64_t* tail) {
  if (tail[0]) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  g->csr.dhat_max = static_cast<int32_t>(tail[1]);
  g->d_max = static_cast<int32_t>(tail[2]);
}

void build_graph(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, const int64_t* edge_off_host,
                 const int32_t* n_per_graph_host, int32_t G, bool on_device, hipStream_t s, tc_graph* g, int order,
                 const int32_t* key_by_id, uint64_t* tail) {
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

  // ---- 1-3: canonical keys, sort, duplicates and degrees
  DevBuf<uint64_t> keys(E, s), tmp(E, s);
  // control words, read back in one copy per synchronisation: [0] kept keys m,
  // [1] repeated keys, [2] vertex id out of range, [3] a sort's look-back gave
  // up, [4] dhat_max, [5] d_max
  DevBuf<uint64_t> ctl(8, s);
  k_fill_words<uint64_t><<<1, 64, 0, s>>>(ctl.get(), 8, 0ull);
  TC_LAUNCH_CHECK();
  uint64_t* d_m = ctl.get();
  unsigned long long* d_dup = reinterpret_cast<unsigned long long*>(ctl.get() + 1);
  int* err = reinterpret_cast<int*>(ctl.get() + 2);
  uint32_t* sort_fail = reinterpret_cast<uint32_t*>(ctl.get() + 3);
  HostWords hw(s);
  g->deg.alloc(n, s);
  if (n > 0) TC_HIP(hipMemsetAsync(g->deg.p, 0, n * sizeof(int32_t), s));
  const uint64_t hmask = (1ull << b) - 1;
  // kept-key flags and per-block counts over the sorted keys (the compaction layout)
  const size_t nfb = (static_cast<size_t>(E) + kFlagChunk - 1) / kFlagChunk;
  DevBuf<uint64_t> kflags(nfb * kFlagWaves * kFlagWords, s), kcnt(nfb, s);
  uint64_t* sorted = nullptr;
  uint64_t* spare = nullptr;
  if (E > 0) {
    k_canon<<<grid_for(E, kBlock, 65536), kBlock, 0, s>>>(dsrc, ddst, static_cast<uint32_t>(E), n, b, d_eoff.get(),
                                                          d_vbase.get(), G, keys.get(), err);
    TC_LAUNCH_CHECK();
    // d_v of the larger endpoints once the passes over their bits [0, b) are done
    const LargerEndHook larger{(b + kRadixBits - 1) / kRadixBits - 1, static_cast<uint64_t>(E), hmask, g->deg.p, s};
    sorted = radix_sort<uint64_t>(keys.get(), tmp.get(), E, 0, 2 * b, s, sort_fail, larger);
    if (E == 1) larger(larger.last_pass, sorted);  // one key is sorted without a pass
    spare = sorted == keys.get() ? tmp.get() : keys.get();
    // repeats' larger endpoints go to the spare key buffer (room for 2E of them)
    k_dedup_degrees<<<static_cast<unsigned>(nfb), kScanBlock, 0, s>>>(
        sorted, static_cast<uint64_t>(E), b, g->deg.p, kflags.get(), kcnt.get(), reinterpret_cast<uint32_t*>(spare),
        d_dup);
    TC_LAUNCH_CHECK();
    exclusive_scan<uint64_t>(kcnt.get(), kcnt.get(), nfb, s, d_m);
  }
  hsrc.release();
  hdst.release();
  TC_HIP(hipMemcpyAsync(hw.get(), ctl.get(), 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (hw[3]) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  if (hw[2]) fail(TC_E_RANGE, "vertex id outside [0, n)");
  const uint64_t m = hw[0], ndup = hw[1];
  g->m = static_cast<int64_t>(m);
  take_off_repeats(reinterpret_cast<uint32_t*>(spare), ndup, b, g->deg.p, s, sort_fail);

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
    // the keys are made in id order, so a stable sort of the order-key bits
    // [b, 2b) alone leaves equal order keys in id order
    u128* r1 = radix_sort<u128>(rk.get(), rk2.get(), n, b, 2 * b, s, sort_fail);
    u128* r2 = r1;
    if (G > 1) r2 = radix_sort<u128>(r1, r1 == rk.get() ? rk2.get() : rk.get(), n, 64, 64 + gbits, s, sort_fail);
    k_rank_from_sorted<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(r2, n, b, g->order.p, g->rank.p,
                                                                      G > 1 ? g->graph_of_rank.p : nullptr);
    TC_LAUNCH_CHECK();
  }

  // ---- 5-6: orientation (with the compaction of the kept keys), sorted rows, offsets
  Csr& c = g->csr;
  c.n = n;
  c.m = static_cast<int64_t>(m);
  c.off.alloc(static_cast<size_t>(n) + 1, s);
  c.adj.alloc(m, s);
  c.src.alloc(m, s);
  if (m > 0) {
    k_flag_compact<uint64_t, RelabelKey><<<static_cast<unsigned>(nfb), kScanBlock, 0, s>>>(
        static_cast<size_t>(E), kflags.get(), RelabelKey{sorted, b, g->rank.p}, spare, kcnt.get());
    TC_LAUNCH_CHECK();
    // group the entries by row: a stable sort of the row bits [b, 2b)
    uint64_t* rows = radix_sort<uint64_t>(spare, sorted, m, b, 2 * b, s, sort_fail);
    uint64_t* other = rows == spare ? sorted : spare;
    k_offsets_from_rows<<<grid_for(static_cast<uint64_t>(n) + 1, kBlock, 65536), kBlock, 0, s>>>(RowOfKey{rows, b}, m,
                                                                                               n, c.off.p);
    TC_LAUNCH_CHECK();
    // In the degree order of Eq. (1) every entry u of row v has d_u >= d_v >= dhat_v, and
    // the degrees of a row's entries sum to at most 2m, so no row is longer than sqrt(2m):
    // small enough graphs skip reading the longest row back.
    const bool short_rows = order == 0 && key_by_id == nullptr &&
                            2 * m <= static_cast<uint64_t>(kSegBlockMax) * static_cast<uint64_t>(kSegBlockMax);
    if (short_rows || max_row_length(c.off.p, n, s) <= kSegBlockMax) {
      const unsigned cus = static_cast<unsigned>(device_cus());
      int rpw = kWave;  // rows per wave: fewer while the rows would fill fewer waves than the grid holds
      while (rpw > 1 && (static_cast<uint64_t>(n) + rpw - 1) / rpw < static_cast<uint64_t>(cus) * 16 * (kSegBlock / kWave))
        rpw >>= 1;
      const uint64_t waves = (static_cast<uint64_t>(n) + rpw - 1) / rpw;
      k_seg_rows_wave<<<grid_for(waves * kWave, kSegBlock, cus * 16), kSegBlock, 0, s>>>(rows, c.off.p, n, b, rpw,
                                                                                        c.adj.p, c.src.p);
      TC_LAUNCH_CHECK();
      DevBuf<int32_t> longrows(n, s);
      DevBuf<uint64_t> nlong(2, s);
      compact_if<int32_t>(static_cast<size_t>(n), RowsBetween{c.off.p, kWave, kSegWideMax}, RowIndex{}, longrows.get(),
                          nlong.get(), s);
      k_seg_rows_wide<<<cus * 8, kSegBlock, 0, s>>>(rows, c.off.p, longrows.get(), nlong.get(), b, c.adj.p, c.src.p);
      TC_LAUNCH_CHECK();
      compact_if<int32_t>(static_cast<size_t>(n), RowsBetween{c.off.p, kSegWideMax, kSegBlockMax}, RowIndex{},
                          longrows.get(), nlong.get() + 1, s);
      k_seg_rows_block<<<cus * 8, kSegBlock, 0, s>>>(rows, c.off.p, longrows.get(), nlong.get() + 1, b, c.adj.p,
                                                      c.src.p);
      TC_LAUNCH_CHECK();
    } else {  // some row is longer than a block sorts: sort every key by row and column instead
      uint64_t* ok = radix_sort<uint64_t>(rows, other, m, 0, 2 * b, s, sort_fail);
      k_csr_fill<<<grid_for(m, kBlock, 65536), kBlock, 0, s>>>(ok, m, b, c.adj.p, c.src.p);
      TC_LAUNCH_CHECK();
    }
  } else {
    k_offsets_from_rows<<<grid_for(static_cast<uint64_t>(n) + 1, kBlock, 65536), kBlock, 0, s>>>(RowOfI32{c.src.p}, 0,
                                                                                               n, c.off.p);
    TC_LAUNCH_CHECK();
  }
  keys.release();
  tmp.release();

  if (n > 0) {
    k_row_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(c.off.p, n, reinterpret_cast<int*>(ctl.get() + 4));
    TC_LAUNCH_CHECK();
    k_array_max<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(g->deg.p, n, reinterpret_cast<int*>(ctl.get() + 5));
    TC_LAUNCH_CHECK();
  }
  // the tail words [look-back failure, dhat_max, d_max]: the caller reads them after its next
  // synchronisation (build_graph_finish), or they are read here
  TC_HIP(hipMemcpyAsync(tail ? tail : hw.get(), ctl.get() + 3, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  if (!tail) {
    TC_HIP(hipStreamSynchronize(s));
    build_graph_finish(g, hw.get());
  }
}

// ============================================================ out of core
//
// The rank-space oriented CSR of a graph whose edge list stays in host memory,
// built under a device-memory budget (graphs larger than one device, Section
// 6): the same steps as build_graph, with the edges streamed through the
// device in pieces that fit the budget.
//
//   A1. Each chunk of records is made canonical on the device and split by a
//       hash of its smaller endpoint into P parts (a multisplit: per-block
//       LDS counts, one reservation per part and block); the grouped chunk
//       goes back to host memory. Every record of a smaller endpoint lands in
//       the same part, so duplicates and runs of equal smaller endpoints stay
//       within a part.
//   A2. Each part is gathered from the chunks, sorted, deduplicated and
//       counted into the degrees exactly as in build_graph (larger endpoints
//       halfway through the sort, smaller ones from runs of the kept keys),
//       and its unique keys go back to host memory.
//   B.  Ranks in the order of Eq. (1) from the complete degrees.
//   C1. The unique keys stream through once more to count each row (the
//       orientation's earlier endpoint); the prefix sum is the CSR offsets.
//   C2. The rows are cut into ranges whose entries fit the budget. With three
//       ranges or more, the unique keys stream through once more, are
//       oriented into rank space and split by range (the same multisplit as
//       A1, the part found by a search of the range starts), grouped per
//       chunk in host memory.
//   C3. For each range, its part is gathered from the chunks (with one or two
//       ranges: the unique keys stream through and its rows are kept), sorted
//       by (row, column) and its columns copied to their place in the host
//       adjacency array.

namespace {

constexpr int kPartLog2Max = 9;  // at most 512 parts
constexpr int kSplitTile = kBlock * 16;

// The part of a key: a multiplicative hash of its high field, or (with
// range starts rs[0..nr], in LDS) the range r with rs[r] <= field < rs[r+1].
__device__ __forceinline__ uint32_t part_of(uint64_t key, int b, int plog2, const int32_t* rs, int nr) {
  const int32_t f = static_cast<int32_t>(key >> b);
  if (rs) {
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rs[mid] <= f) lo = mid;
      else hi = mid - 1;
    }
    return static_cast<uint32_t>(lo);
  }
  return plog2 == 0 ? 0u : static_cast<uint32_t>(((key >> b) * 0x9E3779B97F4A7C15ull) >> (64 - plog2));
}

// Range starts for part_of in LDS (nr + 1 words, nr <= 512); null without ranges.
__device__ __forceinline__ const int32_t* stage_ranges(const int32_t* __restrict__ ranges, int nr, int32_t* lds) {
  if (!ranges) return nullptr;
  for (int i = threadIdx.x; i <= nr; i += blockDim.x) lds[i] = ranges[i];
  return lds;
}

// counts[p] += number of valid keys of part p in this block's tile
__global__ __launch_bounds__(kBlock) void k_part_count(const uint64_t* __restrict__ keys, uint64_t N, int b, int plog2,
                                                       const int32_t* __restrict__ ranges,
                                                       uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[1 << kPartLog2Max];
  __shared__ int32_t rl[(1 << kPartLog2Max) + 1];
  const int P = 1 << plog2;
  const int32_t* rs = stage_ranges(ranges, P, rl);
  for (int i = threadIdx.x; i < P; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSplitTile;
  for (int i = threadIdx.x; i < kSplitTile; i += kBlock) {
    const uint64_t idx = base + i;
    if (idx < N && keys[idx] != ~0ull) atomicAdd(&h[part_of(keys[idx], b, plog2, rs, P)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kBlock)
    if (h[i]) atomicAdd(&counts[i], h[i]);
}

// Each valid key to out[start[p] + its slot]: the block reserves its part
// counts with one atomic per part, then hands out slots in LDS.
__global__ __launch_bounds__(kBlock) void k_part_scatter(const uint64_t* __restrict__ keys, uint64_t N, int b,
                                                         int plog2, const int32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ start,
                                                         uint32_t* __restrict__ cursor, uint64_t* __restrict__ out) {
  __shared__ uint32_t h[1 << kPartLog2Max];
  __shared__ uint32_t base_of[1 << kPartLog2Max];
  __shared__ int32_t rl[(1 << kPartLog2Max) + 1];
  const int P = 1 << plog2;
  const int32_t* rs = stage_ranges(ranges, P, rl);
  for (int i = threadIdx.x; i < P; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSplitTile;
  for (int i = threadIdx.x; i < kSplitTile; i += kBlock) {
    const uint64_t idx = base + i;
    if (idx < N && keys[idx] != ~0ull) atomicAdd(&h[part_of(keys[idx], b, plog2, rs, P)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kBlock) {
    base_of[i] = h[i] ? start[i] + atomicAdd(&cursor[i], h[i]) : 0u;
    h[i] = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSplitTile; i += kBlock) {
    const uint64_t idx = base + i;
    if (idx < N) {
      const uint64_t k = keys[idx];
      if (k != ~0ull) {
        const uint32_t p = part_of(k, b, plog2, rs, P);
        out[base_of[p] + atomicAdd(&h[p], 1u)] = k;
      }
    }
  }
}

struct KeyAt {
  const uint64_t* k;
  __device__ uint64_t operator()(size_t i) const { return k[i]; }
};

// out[i] = the oriented key (min rank << b | max rank) of unique key i
__global__ void k_orient_keys(const uint64_t* __restrict__ keys, uint64_t N, int b, const int32_t* __restrict__ rank,
                              uint64_t* __restrict__ out) {
  const RelabelKey rk{keys, b, rank};
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    out[i] = rk(i);
}

// rows[min rank] += 1 per unique key (runs of equal rows with one atomic)
__global__ __launch_bounds__(kBlock) void k_oriented_row_counts(const uint64_t* __restrict__ keys, uint64_t N, int b,
                                                                const int32_t* __restrict__ rank,
                                                                unsigned long long* __restrict__ rows) {
  const uint64_t mask = (1ull << b) - 1;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x; i0 < N; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    int32_t r = -1;
    if (i < N) {
      const int32_t ra = rank[keys[i] >> b], rb = rank[keys[i] & mask];
      r = ra < rb ? ra : rb;
    }
    const int lane = lane_id();
    const int32_t prev = __shfl_up(r, 1, kWave);
    const uint64_t bounds = __ballot(lane == 0 || prev != r);
    if (r >= 0 && (lane == 0 || prev != r)) {
      const uint64_t above = bounds & ~((2ull << lane) - 1ull);
      const int end = above ? __ffsll(static_cast<long long>(above)) - 1 : kWave;
      atomicAdd(&rows[r], static_cast<unsigned long long>(end - lane));
    }
  }
}

struct RowRangeKeep {
  const uint64_t* k;
  int b;
  const int32_t* rank;
  int32_t r0, r1;
  __device__ bool operator()(size_t i) const {
    const uint64_t mask = (1ull << b) - 1;
    const int32_t ra = rank[k[i] >> b], rb = rank[k[i] & mask];
    const int32_t r = ra < rb ? ra : rb;
    return r >= r0 && r < r1;
  }
};

__global__ void k_cols_of(const uint64_t* __restrict__ ok, uint64_t m, int b, int32_t* __restrict__ adj) {
  const uint64_t mask = (1ull << b) - 1;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    adj[i] = static_cast<int32_t>(ok[i] & mask);
}

// Pinned host memory when it can be had (full copy speed), else pageable.
struct HostBuf {
  uint64_t* p = nullptr;
  bool pinned = false;
  std::vector<uint64_t> v;
  explicit HostBuf(size_t count) {
    if (count == 0) return;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(uint64_t), hipHostMallocDefault) == hipSuccess) {
      pinned = true;
    } else {
      (void)hipGetLastError();
      v.resize(count);
      p = v.data();
    }
  }
  ~HostBuf() {
    if (pinned) (void)hipHostFree(p);
  }
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
};

}  // namespace

void build_host_csr(const int32_t* src, const int32_t* dst, int64_t E, int32_t n, uint64_t budget, hipStream_t s,
                    int64_t* off_h, int32_t* adj_h, int64_t* m_out, uint64_t info[4]) {
  if (E < 0 || n < 0) fail(TC_E_RANGE, "negative edge or vertex count");
  if (n > kMaxVertices) fail(TC_E_RANGE, "more than 2^31 - 2^25 vertices");
  if (E > (1ll << 32) - (1ll << 25)) fail(TC_E_INVAL, "more than 2^32 - 2^25 edge records");
  if (E > 0 && (!src || !dst)) fail(TC_E_INVAL, "NULL edge array");
  if (!off_h || (E > 0 && !adj_h) || !m_out) fail(TC_E_INVAL, "NULL output");
  const int b = bits_for(n > 1 ? static_cast<uint64_t>(n - 1) : 1);
  // vertex arrays stay on the device: degrees, ranks, order, the rank sort, row counts, offsets
  const uint64_t vbytes = 64ull * static_cast<uint64_t>(n) + (16ull << 20);
  if (budget < vbytes + (16ull << 20)) fail(TC_E_NOMEM, "device budget below 64 bytes per vertex plus 32 MiB");
  const uint64_t work = budget - vbytes;
  const uint64_t C1 = work / 24;   // A1: src + dst + key + grouped key
  const uint64_t Cp = work / 20;   // A2: keys + sort buffer + look-back status + flags
  const uint64_t C2 = work / 32;   // C: a chunk of unique keys (a quarter of the work memory)
  const uint64_t Cr = (work - C2 * 8) / 24;  // C3: range keys + sort buffer + status + columns
  uint64_t bytes_in = 0, bytes_out = 0;

  // ---- A1: canonical keys split into parts by a hash of the smaller endpoint
  int plog2 = 0;
  while ((1ull << plog2) * Cp * 4 / 5 < static_cast<uint64_t>(E) && plog2 < kPartLog2Max) plog2++;
  const int P = 1 << plog2;
  const uint64_t nch = E > 0 ? (static_cast<uint64_t>(E) + C1 - 1) / C1 : 0;
  HostBuf grouped(static_cast<size_t>(E));
  std::vector<uint32_t> pcount(static_cast<size_t>(nch) * P, 0), pstart(static_cast<size_t>(nch) * P, 0);
  std::vector<uint64_t> chunk_at(nch + 1, 0);
  DevBuf<int32_t> deg(n, s);
  if (n > 0) TC_HIP(hipMemsetAsync(deg.get(), 0, n * sizeof(int32_t), s));
  DevBuf<int> err(1, s);
  DevBuf<uint32_t> sort_fail(1, s);
  TC_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));
  TC_HIP(hipMemsetAsync(sort_fail.get(), 0, sizeof(uint32_t), s));
  {
    const uint64_t c1 = E > 0 ? (static_cast<uint64_t>(E) < C1 ? static_cast<uint64_t>(E) : C1) : 0;
    DevBuf<int32_t> ds(c1, s), dd(c1, s);
    DevBuf<uint64_t> dk(c1, s), dg(c1, s);
    DevBuf<uint32_t> cnt(P, s), cur(P, s);
    DevBuf<int32_t> vb(2, s);
    const int32_t vbh[2] = {0, n};
    TC_HIP(hipMemcpyAsync(vb.get(), vbh, sizeof(vbh), hipMemcpyHostToDevice, s));
    for (uint64_t c = 0; c < nch; c++) {
      const uint64_t i0 = c * C1, N = (static_cast<uint64_t>(E) - i0) < C1 ? static_cast<uint64_t>(E) - i0 : C1;
      TC_HIP(hipMemcpyAsync(ds.get(), src + i0, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
      TC_HIP(hipMemcpyAsync(dd.get(), dst + i0, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
      bytes_in += 8 * N;
      k_canon<<<grid_for(N, kBlock, 65536), kBlock, 0, s>>>(ds.get(), dd.get(), static_cast<uint32_t>(N), n, b, nullptr,
                                                            vb.get(), 1, dk.get(), err.get());
      TC_LAUNCH_CHECK();
      TC_HIP(hipMemsetAsync(cnt.get(), 0, P * sizeof(uint32_t), s));
      const unsigned tiles = static_cast<unsigned>((N + kSplitTile - 1) / kSplitTile);
      k_part_count<<<tiles, kBlock, 0, s>>>(dk.get(), N, b, plog2, nullptr, cnt.get());
      TC_LAUNCH_CHECK();
      uint32_t* hc = &pcount[c * P];
      TC_HIP(hipMemcpyAsync(hc, cnt.get(), P * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      uint32_t acc = 0;
      for (int p = 0; p < P; p++) {
        pstart[c * P + p] = acc;
        acc += hc[p];
      }
      TC_HIP(hipMemcpyAsync(cnt.get(), &pstart[c * P], P * sizeof(uint32_t), hipMemcpyHostToDevice, s));
      TC_HIP(hipMemsetAsync(cur.get(), 0, P * sizeof(uint32_t), s));
      k_part_scatter<<<tiles, kBlock, 0, s>>>(dk.get(), N, b, plog2, nullptr, cnt.get(), cur.get(), dg.get());
      TC_LAUNCH_CHECK();
      chunk_at[c + 1] = chunk_at[c] + acc;
      if (acc) TC_HIP(hipMemcpyAsync(grouped.p + chunk_at[c], dg.get(), acc * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      bytes_out += 8ull * acc;
      TC_HIP(hipStreamSynchronize(s));  // the staging buffers are reused by the next chunk
    }
  }
  int h_err = 0;
  TC_HIP(hipMemcpyAsync(&h_err, err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h_err) fail(TC_E_RANGE, "vertex id outside [0, n)");

  // ---- A2: per part, sort, deduplicate, degrees; unique keys back to the host
  HostBuf uniq(static_cast<size_t>(E));
  uint64_t m = 0;
  {
    uint64_t big = 0;
    for (int p = 0; p < P; p++) {
      uint64_t t = 0;
      for (uint64_t c = 0; c < nch; c++) t += pcount[c * P + p];
      big = t > big ? t : big;
    }
    if (big > Cp) fail(TC_E_NOMEM, "a part of the edge list does not fit the device budget");
    DevBuf<uint64_t> k1(big, s), k2(big, s);
    const size_t nfb = (static_cast<size_t>(big) + kFlagChunk - 1) / kFlagChunk;
    DevBuf<uint64_t> flags(nfb * kFlagWaves * kFlagWords, s), bc(nfb, s), dm(2, s);
    const uint64_t hmask = (1ull << b) - 1;
    for (int p = 0; p < P; p++) {
      uint64_t M = 0;
      for (uint64_t c = 0; c < nch; c++) {
        const uint32_t k = pcount[c * P + p];
        if (!k) continue;
        TC_HIP(hipMemcpyAsync(k1.get() + M, grouped.p + chunk_at[c] + pstart[c * P + p], k * sizeof(uint64_t),
                              hipMemcpyHostToDevice, s));
        M += k;
      }
      bytes_in += 8 * M;
      if (M == 0) continue;
      const LargerEndHook larger{(b + kRadixBits - 1) / kRadixBits - 1, M, hmask, deg.get(), s};
      uint64_t* sk = radix_sort<uint64_t>(k1.get(), k2.get(), M, 0, 2 * b, s, sort_fail.get(), larger);
      if (M == 1) larger(larger.last_pass, sk);
      uint64_t* spare = sk == k1.get() ? k2.get() : k1.get();
      const size_t nb = (static_cast<size_t>(M) + kFlagChunk - 1) / kFlagChunk;
      TC_HIP(hipMemsetAsync(dm.get() + 1, 0, sizeof(uint64_t), s));
      k_dedup_degrees<<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(
          sk, M, b, deg.get(), flags.get(), bc.get(), reinterpret_cast<uint32_t*>(spare),
          reinterpret_cast<unsigned long long*>(dm.get() + 1));
      TC_LAUNCH_CHECK();
      exclusive_scan<uint64_t>(bc.get(), bc.get(), nb, s, dm.get());
      uint64_t mp_dup[2] = {0, 0};
      TC_HIP(hipMemcpyAsync(mp_dup, dm.get(), 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      take_off_repeats(reinterpret_cast<uint32_t*>(spare), mp_dup[1], b, deg.get(), s, sort_fail.get());
      k_flag_compact<uint64_t, KeyAt><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(static_cast<size_t>(M),
                                                                                       flags.get(), KeyAt{sk}, spare,
                                                                                       bc.get());
      TC_LAUNCH_CHECK();
      const uint64_t mp = mp_dup[0];
      if (mp) TC_HIP(hipMemcpyAsync(uniq.p + m, spare, mp * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      bytes_out += 8 * mp;
      m += mp;
      TC_HIP(hipStreamSynchronize(s));
    }
  }
  if (m >= (1ull << 32)) fail(TC_E_RANGE, "2^32 or more unique edges");

  // ---- B: ranks in the degree order
  DevBuf<int32_t> rank(n, s), order(n, s);
  if (n > 0) {
    DevBuf<u128> rk(n, s), rk2(n, s);
    DevBuf<int32_t> vb(2, s);
    const int32_t vbh[2] = {0, n};
    TC_HIP(hipMemcpyAsync(vb.get(), vbh, sizeof(vbh), hipMemcpyHostToDevice, s));
    k_rank_keys<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(n, b, deg.get(), vb.get(), 1, 0, rk.get());
    TC_LAUNCH_CHECK();
    u128* r1 = radix_sort<u128>(rk.get(), rk2.get(), n, b, 2 * b, s, sort_fail.get());
    k_rank_from_sorted<<<grid_for(n, kBlock, 65536), kBlock, 0, s>>>(r1, n, b, order.get(), rank.get(), nullptr);
    TC_LAUNCH_CHECK();
  }

  // ---- C1: rows of the orientation, offsets
  DevBuf<unsigned long long> rows(static_cast<size_t>(n) + 1, s);
  fill_u64(rows.get(), static_cast<size_t>(n) + 1, 0ull, s);
  const uint64_t c2 = m < C2 ? m : C2;
  DevBuf<uint64_t> dch(c2 > 0 ? c2 : 1, s);
  for (uint64_t i0 = 0; i0 < m; i0 += C2) {
    const uint64_t N = m - i0 < C2 ? m - i0 : C2;
    TC_HIP(hipMemcpyAsync(dch.get(), uniq.p + i0, N * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    bytes_in += 8 * N;
    k_oriented_row_counts<<<grid_for(N, kBlock, 65536), kBlock, 0, s>>>(dch.get(), N, b, rank.get(), rows.get());
    TC_LAUNCH_CHECK();
    TC_HIP(hipStreamSynchronize(s));  // the chunk buffer is reused
  }
  int64_t* offd = reinterpret_cast<int64_t*>(rows.get());
  exclusive_scan<int64_t>(offd, offd, static_cast<size_t>(n), s, offd + n);
  TC_HIP(hipMemcpyAsync(off_h, offd, (static_cast<size_t>(n) + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  uint32_t h_fail = 0;
  TC_HIP(hipMemcpyAsync(&h_fail, sort_fail.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h_fail) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  if (static_cast<uint64_t>(off_h[n]) != m) fail(TC_E_DEVICE, "oriented row counts do not add up to m");

  // ---- C2: row ranges [rs[r], rs[r+1]) whose entries fit the budget (each at least one row)
  std::vector<int32_t> rs(1, 0);
  while (rs.back() < n) {
    const int32_t r0 = rs.back();
    int32_t lo = r0 + 1, hi = n;  // largest r1 with off[r1] - off[r0] <= Cr
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (static_cast<uint64_t>(off_h[mid] - off_h[r0]) <= Cr) lo = mid;
      else hi = mid - 1;
    }
    if (static_cast<uint64_t>(off_h[lo] - off_h[r0]) > Cr) fail(TC_E_NOMEM, "one oriented row does not fit the device budget");
    rs.push_back(lo);
  }
  const uint64_t ranges = rs.size() - 1;
  // Splitting costs a pass in and a pass out over the keys and saves one pass in per range
  // after the first: worth it from three ranges on (up to the multisplit's 512 parts).
  const bool split = ranges >= 3 && ranges <= (1u << kPartLog2Max) && m > 0;
  int p2log = 0;
  while ((1ull << p2log) < ranges) p2log++;
  const int P2 = 1 << p2log;
  const uint64_t nch2 = split ? (m + C2 - 1) / C2 : 0;
  std::vector<uint32_t> pc2(static_cast<size_t>(nch2) * P2, 0), ps2(static_cast<size_t>(nch2) * P2, 0);
  std::vector<uint64_t> chunk2_at(nch2 + 1, 0);
  if (split) {  // the oriented keys grouped by range, per chunk, in the host buffer of the grouped records
    std::vector<int32_t> starts(static_cast<size_t>(P2) + 1, n);  // ranges past the last are empty
    for (uint64_t r = 0; r < ranges; r++) starts[r] = rs[r];
    DevBuf<int32_t> drs(static_cast<size_t>(P2) + 1, s);
    TC_HIP(hipMemcpyAsync(drs.get(), starts.data(), starts.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    DevBuf<uint64_t> dor(c2, s), dgr(c2, s);
    DevBuf<uint32_t> cnt(P2, s), cur(P2, s);
    for (uint64_t c = 0; c < nch2; c++) {
      const uint64_t i0 = c * C2, N = m - i0 < C2 ? m - i0 : C2;
      TC_HIP(hipMemcpyAsync(dch.get(), uniq.p + i0, N * sizeof(uint64_t), hipMemcpyHostToDevice, s));
      bytes_in += 8 * N;
      k_orient_keys<<<grid_for(N, kBlock, 65536), kBlock, 0, s>>>(dch.get(), N, b, rank.get(), dor.get());
      TC_LAUNCH_CHECK();
      TC_HIP(hipMemsetAsync(cnt.get(), 0, P2 * sizeof(uint32_t), s));
      const unsigned tiles = static_cast<unsigned>((N + kSplitTile - 1) / kSplitTile);
      k_part_count<<<tiles, kBlock, 0, s>>>(dor.get(), N, b, p2log, drs.get(), cnt.get());
      TC_LAUNCH_CHECK();
      uint32_t* hc = &pc2[c * P2];
      TC_HIP(hipMemcpyAsync(hc, cnt.get(), P2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      uint64_t acc = 0;
      for (int p = 0; p < P2; p++) {
        ps2[c * P2 + p] = static_cast<uint32_t>(acc);
        acc += hc[p];
      }
      if (acc != N) fail(TC_E_DEVICE, "row range counts do not add up");
      TC_HIP(hipMemcpyAsync(cnt.get(), &ps2[c * P2], P2 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
      TC_HIP(hipMemsetAsync(cur.get(), 0, P2 * sizeof(uint32_t), s));
      k_part_scatter<<<tiles, kBlock, 0, s>>>(dor.get(), N, b, p2log, drs.get(), cnt.get(), cur.get(), dgr.get());
      TC_LAUNCH_CHECK();
      chunk2_at[c + 1] = chunk2_at[c] + N;
      TC_HIP(hipMemcpyAsync(grouped.p + chunk2_at[c], dgr.get(), N * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      bytes_out += 8 * N;
      TC_HIP(hipStreamSynchronize(s));  // the chunk buffers are reused
    }
  }

  // ---- C3: each range sorted and its columns copied out
  {
    DevBuf<uint64_t> rk1(Cr, s), rk2(Cr, s);
    DevBuf<int32_t> cols(Cr, s);
    DevBuf<uint64_t> dcnt(1, s);
    for (uint64_t r = 0; r < ranges; r++) {
      const int32_t r0 = rs[r], r1 = rs[r + 1];
      const uint64_t M = static_cast<uint64_t>(off_h[r1] - off_h[r0]);
      if (M == 0) continue;
      uint64_t got = 0;
      if (split) {  // the range's part of every chunk (already oriented)
        for (uint64_t c = 0; c < nch2; c++) {
          const uint32_t k = pc2[c * P2 + r];
          if (!k) continue;
          if (got + k > M) fail(TC_E_DEVICE, "row range overflow");
          TC_HIP(hipMemcpyAsync(rk1.get() + got, grouped.p + chunk2_at[c] + ps2[c * P2 + r], k * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s));
          bytes_in += 8ull * k;
          got += k;
        }
      } else {  // every unique key streams through; the range's rows are kept, oriented
        for (uint64_t i0 = 0; i0 < m; i0 += C2) {
          const uint64_t N = m - i0 < C2 ? m - i0 : C2;
          TC_HIP(hipMemcpyAsync(dch.get(), uniq.p + i0, N * sizeof(uint64_t), hipMemcpyHostToDevice, s));
          bytes_in += 8 * N;
          compact_if<uint64_t>(N, RowRangeKeep{dch.get(), b, rank.get(), r0, r1}, RelabelKey{dch.get(), b, rank.get()},
                               rk1.get() + got, dcnt.get(), s);
          uint64_t k = 0;
          TC_HIP(hipMemcpyAsync(&k, dcnt.get(), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
          TC_HIP(hipStreamSynchronize(s));
          got += k;
          if (got > M) fail(TC_E_DEVICE, "row range overflow");
        }
      }
      if (got != M) fail(TC_E_DEVICE, "row range count mismatch");
      uint64_t* ok = radix_sort<uint64_t>(rk1.get(), rk2.get(), M, 0, 2 * b, s, sort_fail.get());
      k_cols_of<<<grid_for(M, kBlock, 65536), kBlock, 0, s>>>(ok, M, b, cols.get());
      TC_LAUNCH_CHECK();
      TC_HIP(hipMemcpyAsync(adj_h + off_h[r0], cols.get(), M * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      bytes_out += 4 * M;
      TC_HIP(hipStreamSynchronize(s));
    }
  }
  TC_HIP(hipMemcpyAsync(&h_fail, sort_fail.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h_fail) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  *m_out = static_cast<int64_t>(m);
  if (info) {
    info[0] = static_cast<uint64_t>(P);
    info[1] = ranges;
    info[2] = bytes_in;
    info[3] = bytes_out;
  }
}

}  // namespace tc
