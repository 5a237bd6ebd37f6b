// Device-wide building blocks: exclusive scan, stream compaction and an LSD
// radix sort. Header-only templates; every translation unit that uses one
// instantiates its own kernels.
#pragma once

#include <type_traits>
#include <utility>

#include "common.hpp"

namespace tc {

// ================================================================== scan ===

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Input of a scan: element i of an array, or any functor of i.
template <typename T>
struct ArrayAt {
  const T* a;
  __device__ T operator()(size_t i) const { return a[i]; }
};

template <typename T, typename Get>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(Get get, size_t N, T* __restrict__ partial) {
  __shared__ T sm[kScanBlock / kWave];
  const size_t base = static_cast<size_t>(blockIdx.x) * kScanChunk;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    size_t idx = base + static_cast<size_t>(i) * kScanBlock + threadIdx.x;
    if (idx < N) s += get(idx);
  }
  T tot;
  (void)block_excl_scan<T, kScanBlock>(s, sm, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// out[i] = carry(block) + sum of get(j) for j < i within the block's chunk.
// The input may alias `out` (the chunk is read before it is written). The
// last block stores the grand total.
template <typename T, typename Get>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(Get get, T* out, size_t N, const T* __restrict__ carry,
                                                            T* __restrict__ total_out) {
  __shared__ T sm[kScanBlock / kWave];
  __shared__ T tile[kScanChunk + kScanChunk / 32];
  auto pad = [](int j) { return j + (j >> 5); };
  const size_t base = static_cast<size_t>(blockIdx.x) * kScanChunk;
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    int j = i * kScanBlock + threadIdx.x;
    size_t idx = base + j;
    tile[pad(j)] = idx < N ? get(idx) : T(0);
  }
  __syncthreads();
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = tile[pad(threadIdx.x * kScanItems + j)];
    s += v[j];
  }
  T tot;
  T pre = block_excl_scan<T, kScanBlock>(s, sm, tot);
  T run = (carry ? carry[blockIdx.x] : T(0)) + pre;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    tile[pad(threadIdx.x * kScanItems + j)] = run;
    run += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    int j = i * kScanBlock + threadIdx.x;
    size_t idx = base + j;
    if (idx < N) out[idx] = tile[pad(j)];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) *total_out = run;
}

template <typename T>
__global__ void k_store_zero(T* p) { *p = T(0); }

// Exclusive prefix sum of get(0..N) into out; total_dev (optional) receives
// the sum of all N inputs.
template <typename T, typename Get>
void exclusive_scan_of(Get get, T* out, size_t N, hipStream_t s, T* total_dev = nullptr);

// Exclusive prefix sum of in[0..N) into out (may alias); total_dev (optional)
// receives the sum of all N inputs.
template <typename T>
void exclusive_scan(const T* in, T* out, size_t N, hipStream_t s, T* total_dev = nullptr) {
  exclusive_scan_of<T>(ArrayAt<T>{in}, out, N, s, total_dev);
}

template <typename T, typename Get>
void exclusive_scan_of(Get get, T* out, size_t N, hipStream_t s, T* total_dev) {
  if (N == 0) {
    if (total_dev) {
      k_store_zero<T><<<1, 1, 0, s>>>(total_dev);
      TC_LAUNCH_CHECK();
    }
    return;
  }
  const size_t nb = (N + kScanChunk - 1) / kScanChunk;
  if (nb == 1) {
    k_scan_apply<T, Get><<<1, kScanBlock, 0, s>>>(get, out, N, nullptr, total_dev);
    TC_LAUNCH_CHECK();
    return;
  }
  DevBuf<T> part(nb, s);
  k_scan_reduce<T, Get><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(get, N, part.get());
  TC_LAUNCH_CHECK();
  exclusive_scan<T>(part.get(), part.get(), nb, s, nullptr);
  k_scan_apply<T, Get><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(get, out, N, part.get(), total_dev);
  TC_LAUNCH_CHECK();
}

// ============================================================ compaction ===

// Pred: __device__ bool operator()(size_t i) const; Gen: __device__ T operator()(size_t i) const.
//
// Two passes over wave-strided chunks: wave w of a block takes elements
// [c, c + 64 * kFlagWords) of its block's range, word j covering
// c + 64 j + lane. The first pass evaluates pred once per element, keeps the
// ballot of every word and counts the block; the second reads the ballots back,
// so pred runs once and loads are coalesced.

constexpr int kFlagWords = 16;                               // 64-element words per wave
constexpr int kFlagWaves = kScanBlock / kWave;
constexpr size_t kFlagChunk = static_cast<size_t>(kScanBlock) * kFlagWords;  // elements per block

template <typename Pred>
__global__ __launch_bounds__(kScanBlock) void k_flag_count(size_t N, Pred pred, uint64_t* __restrict__ flags,
                                                           uint64_t* __restrict__ counts) {
  __shared__ uint64_t sm[kFlagWaves];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const size_t word0 = (static_cast<size_t>(blockIdx.x) * kFlagWaves + w) * kFlagWords;
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < kFlagWords; j++) {
    const size_t i = (word0 + j) * kWave + lane;
    const uint64_t b = __ballot(i < N && pred(i));
    if (lane == 0) flags[word0 + j] = b;
    c += static_cast<uint64_t>(__popcll(b));
  }
  if (lane == 0) sm[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int x = 0; x < kFlagWaves; x++) t += sm[x];
    counts[blockIdx.x] = t;
  }
}

template <typename T, typename Gen>
__global__ __launch_bounds__(kScanBlock) void k_flag_compact(size_t N, const uint64_t* __restrict__ flags, Gen gen,
                                                             T* __restrict__ out, const uint64_t* __restrict__ offs) {
  __shared__ uint64_t sm[kFlagWaves];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const size_t word0 = (static_cast<size_t>(blockIdx.x) * kFlagWaves + w) * kFlagWords;
  const size_t nwords = (N + kWave - 1) / kWave;
  uint64_t b[kFlagWords];
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < kFlagWords; j++) {
    b[j] = word0 + j < nwords ? flags[word0 + j] : 0ull;
    c += static_cast<uint64_t>(__popcll(b[j]));
  }
  if (lane == 0) sm[w] = c;
  __syncthreads();
  uint64_t pos = offs[blockIdx.x];
  for (int x = 0; x < w; x++) pos += sm[x];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < kFlagWords; j++) {
    if ((b[j] >> lane) & 1ull) out[pos + static_cast<uint64_t>(__popcll(b[j] & lt))] = gen((word0 + j) * kWave + lane);
    pos += static_cast<uint64_t>(__popcll(b[j]));
  }
}

// Writes gen(i) for every i in [0,N) with pred(i), in index order, to out.
// Returns nothing on the host; the kept count goes to count_dev (device uint64).
template <typename T, typename Pred, typename Gen>
void compact_if(size_t N, Pred pred, Gen gen, T* out, uint64_t* count_dev, hipStream_t s) {
  if (N == 0) {
    k_store_zero<uint64_t><<<1, 1, 0, s>>>(count_dev);
    TC_LAUNCH_CHECK();
    return;
  }
  const size_t nb = (N + kFlagChunk - 1) / kFlagChunk;
  DevBuf<uint64_t> cnt(nb, s), flags(nb * kFlagWaves * kFlagWords, s);
  k_flag_count<Pred><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(N, pred, flags.get(), cnt.get());
  TC_LAUNCH_CHECK();
  exclusive_scan<uint64_t>(cnt.get(), cnt.get(), nb, s, count_dev);
  k_flag_compact<T, Gen><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(N, flags.get(), gen, out, cnt.get());
  TC_LAUNCH_CHECK();
}

// ============================================================ radix sort ===

struct u128 {
  uint64_t lo, hi;
};

// 9-bit digits: 512 bins, one per thread of a scatter block.
constexpr int kRadixBits = 9;
constexpr uint32_t kBins = 1u << kRadixBits;

// The key's bits from `shift` up (the caller masks the digit width).
template <typename K>
struct RadixKey;

template <>
struct RadixKey<uint64_t> {
  __device__ __forceinline__ static uint32_t bits(uint64_t k, int shift) { return static_cast<uint32_t>(k >> shift); }
};

template <>
struct RadixKey<uint32_t> {
  __device__ __forceinline__ static uint32_t bits(uint32_t k, int shift) { return k >> shift; }
};

template <>
struct RadixKey<u128> {
  __device__ __forceinline__ static uint32_t bits(const u128& k, int shift) {
    if (shift >= 64) return static_cast<uint32_t>(k.hi >> (shift - 64));
    if (shift == 0) return static_cast<uint32_t>(k.lo);
    return static_cast<uint32_t>((k.lo >> shift) | (k.hi << (64 - shift)));
  }
};

// Keys per thread of the histogram pass (256 threads) and of a scatter tile.
template <typename K>
struct RadixItems;
template <>
struct RadixItems<uint64_t> {
  static constexpr int value = 32;
};
template <>
struct RadixItems<uint32_t> {
  static constexpr int value = 32;
};
template <>
struct RadixItems<u128> {
  static constexpr int value = 8;
};

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;

// Scatter passes run 512-thread blocks (thread d owns digit d) over tiles of
// 256 * RadixItems keys.
constexpr int kScatterBlock = 512;
constexpr int kScatterWaves = kScatterBlock / kWave;
static_assert(kScatterBlock == static_cast<int>(kBins), "one digit per scatter thread");
template <typename K>
struct ScatterItems {
  static constexpr int value = RadixItems<K>::value * kSortBlock / kScatterBlock;
};

// Mask of the lanes whose BITS-bit value equals this lane's (all 64 lanes active).
// Per bit: the bit as 0 / all-ones, its ballot, and the lanes whose bit differs
// (ballot xor own bit) OR-ed into a mismatch mask; the peers are the rest.
template <int BITS>
__device__ __forceinline__ uint64_t match_any(uint32_t d) {
  uint32_t mis_lo = 0, mis_hi = 0;
#pragma unroll
  for (int b = 0; b < BITS; b++) {
    const uint32_t m = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int32_t>(d), b, 1));
    const uint64_t bb = __ballot(m != 0u);
    // mis |= bb ^ m in one op per half (truth table of S0 | (S1 ^ S2))
    mis_lo = __builtin_amdgcn_bitop3_b32(mis_lo, static_cast<uint32_t>(bb), m, 0xF6);
    mis_hi = __builtin_amdgcn_bitop3_b32(mis_hi, static_cast<uint32_t>(bb >> 32), m, 0xF6);
  }
  return ~((static_cast<uint64_t>(mis_hi) << 32) | mis_lo);
}

// Single-sweep LSD radix sort. One read of the keys counts the digits of
// every pass; each pass is then one kernel that ranks a tile in LDS, finds
// the tile's global offset per digit from its predecessors' published counts
// (decoupled look-back: tiles take their index from a counter, so a tile only
// waits on tiles that are already running) and scatters the tile.

constexpr int kMaxPasses = 16;
constexpr uint64_t kKindAgg = 1ull << 62;   // status word: count of this tile only
constexpr uint64_t kKindInc = 2ull << 62;   // status word: count of all tiles up to this one
constexpr uint64_t kKindMask = 3ull << 62;
constexpr int kTagShift = 56;               // bits 56..61 hold the pass number + 1
constexpr uint64_t kValMask = (1ull << kTagShift) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;   // polls of a not-yet-published word before giving up

__host__ __device__ __forceinline__ uint32_t radix_digit_mask(int shift, int bit_hi) {
  const int w = bit_hi - shift;
  return w >= kRadixBits ? kBins - 1u : (1u << w) - 1u;
}

// Where a sort's first pass reads key i and value i: its key and value
// arrays, or (another source type) a functor that makes them on the fly.
// The digit count reads hist() instead: keys whose bits [kHistShift, ...)
// are the sort keys' bits [kHistShift, ...) seen from bit 0 (a narrower key
// type where the sort bits allow it).
template <typename K, typename V>
struct ArraySource {
  using Key = K;
  static constexpr bool kArrays = true;
  static constexpr int kHistShift = 0;
  const K* __restrict__ keys;
  const V* __restrict__ vals;
  __device__ __forceinline__ K key(size_t i) const { return keys[i]; }
  __device__ __forceinline__ V val(size_t i) const { return vals[i]; }
  ArraySource hist() const { return *this; }
};

// Where a pass writes the value that lands at output position g (with its
// key at hand): the value array, or (another sink type) a functor that
// writes something made of both.
template <typename K, typename V>
struct ArraySink {
  V* __restrict__ vals;
  __device__ __forceinline__ void put(size_t g, const K&, V v) const { vals[g] = v; }
};

// hist[p * kBins + d] += number of keys whose pass-p digit is d. The block's
// LDS counts are kept in `copies` copies (lane L adds to copy L % copies),
// each one word further along the banks than the last, so lanes with equal
// digits in different copies hit different banks, and so do lanes of one copy
// with digits that differ below 32.
template <typename K, typename Src>
__global__ __launch_bounds__(kSortBlock) void k_sweep_hist(Src keys, uint32_t N, int bit_lo, int bit_hi, int passes,
                                                            int copies, uint32_t* __restrict__ hist) {
  constexpr int ITEMS = RadixItems<K>::value;
  constexpr int TILE = kSortBlock * ITEMS;
  extern __shared__ uint32_t h[];  // copies * (passes * kBins + 1)
  const int cstride = passes * static_cast<int>(kBins) + 1;
  const int nh = cstride * copies;
  for (int i = threadIdx.x; i < nh; i += kSortBlock) h[i] = 0;
  __syncthreads();
  const uint32_t c = static_cast<uint32_t>(lane_id()) & static_cast<uint32_t>(copies - 1);
  const size_t stride = static_cast<size_t>(gridDim.x) * TILE;
  // the next tile's keys are loaded while this tile's digits are counted
  K k[ITEMS], nk[ITEMS];
  size_t base = static_cast<size_t>(blockIdx.x) * TILE;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const size_t idx = base + static_cast<size_t>(i) * kSortBlock + threadIdx.x;
    if (idx < N) k[i] = keys.key(idx);
  }
  for (; base < N; base += stride) {
    const size_t next = base + stride;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const size_t idx = next + static_cast<size_t>(i) * kSortBlock + threadIdx.x;
      if (idx < N) nk[i] = keys.key(idx);
    }
    for (int p = 0; p < passes; p++) {
      const int shift = bit_lo + kRadixBits * p;
      const uint32_t dm = radix_digit_mask(shift, bit_hi);
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const size_t idx = base + static_cast<size_t>(i) * kSortBlock + threadIdx.x;
        if (idx < N) atomicAdd(&h[c * cstride + p * kBins + (RadixKey<K>::bits(k[i], shift) & dm)], 1u);
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) k[i] = nk[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * static_cast<int>(kBins); i += kSortBlock) {
    uint32_t t = 0;
    for (int x = 0; x < copies; x++) t += h[x * cstride + i];
    if (t) atomicAdd(&hist[i], t);
  }
}

// In place: each pass's kBins counts become exclusive digit starts (one block per pass).
static __global__ __launch_bounds__(kBins) void k_sweep_starts(uint32_t* __restrict__ hist) {
  __shared__ uint32_t tmp[kBins / kWave];
  uint32_t* h = hist + static_cast<size_t>(blockIdx.x) * kBins;
  const uint32_t x = h[threadIdx.x];
  uint32_t all;
  const uint32_t ex = block_excl_scan<uint32_t, kBins>(x, tmp, all);
  h[threadIdx.x] = ex;
}

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value type of a keys-only sort.
struct NoVal {};

// One pass. Wave w ranks the contiguous chunk [w*ITEMS*64, (w+1)*ITEMS*64)
// of the tile among equal digits with wave-private 16-bit counters (ballot
// match, the lowest lane of each group updating the counter), so tile order is
// index order and the pass is stable. ctr[0] hands out tile indices; *fail
// is set if a look-back gave up. With a value type V, each key's value moves
// with it (staged through the same LDS tile after the keys are written).
template <typename K, typename V, typename Src, typename Sink>
__global__ __launch_bounds__(kScatterBlock) void k_sweep_scatter(Src in, K* __restrict__ out, Sink vout,
                                                                 uint32_t N, int shift, uint32_t dmask, uint64_t tag,
                                                                 const uint32_t* __restrict__ starts,
                                                                 uint64_t* __restrict__ status,
                                                                 uint32_t* __restrict__ ctr,
                                                                 uint32_t* __restrict__ fail) {
  constexpr bool kHasVal = !std::is_same<V, NoVal>::value;
  constexpr int ITEMS = ScatterItems<K>::value;
  constexpr int TILE = kScatterBlock * ITEMS;
  constexpr int CHUNK = kWave * ITEMS;
  static_assert(CHUNK < 65536 && TILE < 65536, "16-bit tile counters");
  static_assert(!kHasVal || sizeof(V) <= sizeof(K), "values are staged in the key tile");
  __shared__ K tile[TILE];
  __shared__ uint16_t wc[kScatterWaves][kBins];  // per-wave digit counts, then per-wave offsets inside a digit
  __shared__ uint32_t dstart[kBins];
  __shared__ uint32_t gbase[kBins];
  __shared__ uint32_t scan_tmp[kScatterWaves];
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  if (tid == 0) s_tile = atomicAdd(&ctr[0], 1u);
  for (int i = tid; i < kScatterWaves * static_cast<int>(kBins); i += kScatterBlock) (&wc[0][0])[i] = 0;
  __syncthreads();
  const uint32_t t = s_tile;
  const size_t base = static_cast<size_t>(t) * TILE;

  K key[ITEMS];
  uint32_t rk[ITEMS];
  uint32_t dg[ITEMS];
  // values are loaded with the keys, so their latency overlaps the ranking
  using VReg = typename std::conditional<kHasVal, V, uint8_t>::type;
  VReg val[kHasVal ? ITEMS : 1];
  uint16_t* cnt = wc[w];
  // All peers read the digit's count (one broadcast read), then the lowest
  // peer adds the group; LDS operations of one wave complete in order.
  auto rank_item = [&](int i, uint32_t d, uint64_t peers, bool valid) {
    const uint32_t lr = static_cast<uint32_t>(__popcll(peers & lanemask_lt()));
    const uint32_t old = valid ? static_cast<uint32_t>(cnt[d]) : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && lr == 0) cnt[d] = static_cast<uint16_t>(old + static_cast<uint32_t>(__popcll(peers)));
    dg[i] = d;
    rk[i] = old + lr;
    __builtin_amdgcn_wave_barrier();
  };
  const size_t chunk = base + static_cast<size_t>(w) * CHUNK + lane;
  if (base + TILE <= N) {  // full tile (wave-uniform): no bounds checks, one ballot per digit bit
#pragma unroll
    for (int i = 0; i < ITEMS; i++) key[i] = in.key(chunk + static_cast<size_t>(i) * kWave);
    if constexpr (kHasVal) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) val[i] = in.val(chunk + static_cast<size_t>(i) * kWave);
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t d = RadixKey<K>::bits(key[i], shift) & dmask;
      rank_item(i, d, match_any<kRadixBits>(d), true);
    }
  } else {  // partial tile: a validity bit joins the match
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const size_t idx = base + static_cast<size_t>(w) * CHUNK + static_cast<size_t>(i) * kWave + lane;
      key[i] = K{};
      if (idx < N) key[i] = in.key(idx);
      if constexpr (kHasVal) {
        val[i] = V{};
        if (idx < N) val[i] = in.val(idx);
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const size_t idx = base + static_cast<size_t>(w) * CHUNK + static_cast<size_t>(i) * kWave + lane;
      const bool valid = idx < N;
      const uint32_t d = valid ? (RadixKey<K>::bits(key[i], shift) & dmask) : kBins;
      rank_item(i, d, match_any<kRadixBits + 1>(d), valid);
    }
  }
  __syncthreads();
  // thread tid owns digit tid: per-wave offsets inside the digit, and the tile's count
  uint32_t tot = 0;
  uint64_t excl = 0;
#pragma unroll
  for (int x = 0; x < kScatterWaves; x++) {
    const uint32_t c = wc[x][tid];
    wc[x][tid] = static_cast<uint16_t>(tot);
    tot += c;
  }
  uint64_t* mine = status + static_cast<size_t>(t) * kBins + tid;
  if (t == 0) {
    status_store(mine, kKindInc | tag | tot);
  } else {
    // a predecessor already inclusive gives the prefix at once: one publication instead of two
    const uint64_t pv = status_load(status + static_cast<size_t>(t - 1) * kBins + tid);
    const bool ready = (pv & kKindMask) == kKindInc && (pv & ~kKindMask & ~kValMask) == tag;
    if (ready) excl = pv & kValMask;
    else status_store(mine, kKindAgg | tag | tot);
    uint32_t j = t - 1;
    uint32_t polls = 0;
    while (!ready) {
      const uint64_t v = status_load(status + static_cast<size_t>(j) * kBins + tid);
      const uint64_t kind = v & kKindMask;
      if (kind == 0 || (v & ~kKindMask & ~kValMask) != tag) {
        if (++polls > kSpinLimit) {
          atomicOr(fail, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += v & kValMask;
      if (kind == kKindInc || j == 0) break;
      --j;
    }
    status_store(mine, kKindInc | tag | (excl + tot));
  }
  uint32_t all;
  const uint32_t ds = block_excl_scan<uint32_t, kScatterBlock>(tot, scan_tmp, all);
  dstart[tid] = ds;
  gbase[tid] = starts[tid] + static_cast<uint32_t>(excl);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    if (dg[i] < kBins) {
      rk[i] += dstart[dg[i]] + wc[w][dg[i]];  // the key's position in the staged tile
      tile[rk[i]] = key[i];
    }
  }
  __syncthreads();
  const uint32_t count = static_cast<uint32_t>(N - base < static_cast<size_t>(TILE) ? N - base : TILE);
  // the array sink needs only the output position of staged position i * kScatterBlock + tid;
  // another sink gets the key too
  constexpr bool kKeepKey = kHasVal && !std::is_same<Sink, ArraySink<K, V>>::value;
  uint32_t gpos[kHasVal ? ITEMS : 1];
  K gkey[kKeepKey ? ITEMS : 1];
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t j = static_cast<uint32_t>(i * kScatterBlock + tid);
    if (j < count) {
      const K k = tile[j];
      const uint32_t d = RadixKey<K>::bits(k, shift) & dmask;
      const uint32_t g = gbase[d] + (j - dstart[d]);
      out[g] = k;
      if constexpr (kHasVal) gpos[i] = g;
      if constexpr (kKeepKey) gkey[i] = k;
    }
  }
  if constexpr (kHasVal) {
    __syncthreads();
    V* vt = reinterpret_cast<V*>(tile);
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      if (dg[i] < kBins) vt[rk[i]] = val[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = static_cast<uint32_t>(i * kScatterBlock + tid);
      if (j < count) {
        if constexpr (kKeepKey) vout.put(gpos[i], gkey[i], vt[j]);
        else vout.put(gpos[i], K{}, vt[j]);
      }
    }
  }
}

template <typename T>
__global__ void k_fill_words(T* __restrict__ p, size_t n, T v) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Called after each scatter pass with the pass index and the buffer that
// holds the keys sorted by the bits of that pass and the ones before it.
struct NoHook {
  template <typename K>
  void operator()(int, const K*) const {}
};

// keys[i], vals[i] = the source's key i and value i (a source that is not
// the arrays themselves, when no pass runs).
template <typename K, typename V, typename Src>
__global__ void k_materialize(Src src, uint32_t N, K* __restrict__ keys, V* __restrict__ vals) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    keys[i] = src.key(i);
    if constexpr (!std::is_same<V, NoVal>::value) vals[i] = src.val(i);
  }
}

// Sorts N keys ascending by bits [bit_lo, bit_hi) (9-bit digits, stable),
// each value moving with its key. The first pass (and the digit count) reads
// key i and value i from `first`; the passes then ping-pong between
// `tmp`/`vtmp` and `keys`/`vals`. Returns the key buffer holding the result
// and points `vals` at the value buffer holding the result. A pass whose
// look-back gave up sets *fail_dev (device word, never cleared here); the
// caller checks it at its next synchronisation. Without fail_dev the sort
// synchronises the stream and checks its own flag before returning.
// hook(p, buf) runs on the host after pass p is queued (work it queues on s
// sees the keys sorted by bits [bit_lo, bit_lo + 9 (p + 1))); no pass runs,
// and the hook is not called, when N <= 1 (the source is then copied to
// keys/vals unless it is those arrays). With `last`, the last pass hands each
// value and its key to that sink instead of writing a value buffer (the
// returned `vals` then holds nothing; `last` is not used when no pass runs).
template <typename K, typename V, typename Src, typename Hook = NoHook, typename Sink = ArraySink<K, V>>
K* radix_sort_from(Src first, K* keys, K* tmp, V*& vals, V* vtmp, size_t N, int bit_lo, int bit_hi, hipStream_t s,
                   uint32_t* fail_dev = nullptr, Hook hook = Hook(), const Sink* last = nullptr) {
  if (N <= 1 || bit_hi <= bit_lo) {
    if constexpr (!Src::kArrays) {
      if (N >= (1ull << 32)) fail(TC_E_INVAL, "radix_sort: more than 2^32 - 1 keys");
      if (N > 0) {
        k_materialize<K, V, Src><<<grid_for(N, 256, 65536), 256, 0, s>>>(first, static_cast<uint32_t>(N), keys, vals);
        TC_LAUNCH_CHECK();
      }
    }
    return keys;
  }
  if (N >= (1ull << 32)) fail(TC_E_INVAL, "radix_sort: more than 2^32 - 1 keys");
  constexpr int TILE = kScatterBlock * ScatterItems<K>::value;
  const int passes = (bit_hi - bit_lo + kRadixBits - 1) / kRadixBits;
  if (passes > kMaxPasses) fail(TC_E_INVAL, "radix_sort: bit range too wide");
  const uint32_t tiles = static_cast<uint32_t>((N + TILE - 1) / TILE);
  // words: passes*kBins histogram/starts, per pass a tile counter, then a local failure flag
  const size_t nwords = static_cast<size_t>(passes) * kBins + passes + 1;
  DevBuf<uint32_t> words(nwords, s);
  DevBuf<uint64_t> status(static_cast<size_t>(tiles) * kBins, s);
  k_fill_words<uint32_t><<<grid_for(nwords, 256, 64), 256, 0, s>>>(words.get(), nwords, 0u);
  TC_LAUNCH_CHECK();
  k_fill_words<uint64_t><<<grid_for(static_cast<uint64_t>(tiles) * kBins, 256, 8192), 256, 0, s>>>(
      status.get(), static_cast<size_t>(tiles) * kBins, 0ull);
  TC_LAUNCH_CHECK();
  uint32_t* hist = words.get();
  uint32_t* ctrs = hist + static_cast<size_t>(passes) * kBins;
  uint32_t* fail_flag = fail_dev ? fail_dev : ctrs + passes;
  int copies = 4;  // LDS: copies * (passes * kBins + 1) words <= 64 KiB
  while (copies > 1 && static_cast<size_t>(copies) * (static_cast<size_t>(passes) * kBins + 1) * 4 > 65536) copies >>= 1;
  const auto hsrc = first.hist();
  using HSrc = decltype(hsrc);
  k_sweep_hist<typename HSrc::Key, HSrc><<<tiles < 2048u ? tiles : 2048u, kSortBlock,
                                            static_cast<size_t>(copies) * (static_cast<size_t>(passes) * kBins + 1) * 4,
                                            s>>>(hsrc, static_cast<uint32_t>(N), bit_lo - Src::kHistShift,
                                                 bit_hi - Src::kHistShift, passes, copies, hist);
  TC_LAUNCH_CHECK();
  k_sweep_starts<<<passes, kBins, 0, s>>>(hist);
  TC_LAUNCH_CHECK();
  K* a = keys;
  K* b = tmp;
  V* va = vals;
  V* vb = vtmp;
  for (int p = 0; p < passes; p++) {
    const int shift = bit_lo + kRadixBits * p;
    const uint32_t dm = radix_digit_mask(shift, bit_hi);
    const uint64_t tag = static_cast<uint64_t>(p + 1) << kTagShift;
    uint32_t* hp = hist + static_cast<size_t>(p) * kBins;
    const ArraySink<K, V> to{vb};
    if (p + 1 == passes && last) {
      if (p == 0)
        k_sweep_scatter<K, V, Src, Sink><<<tiles, kScatterBlock, 0, s>>>(first, b, *last, static_cast<uint32_t>(N),
                                                                         shift, dm, tag, hp, status.get(), ctrs + p,
                                                                         fail_flag);
      else
        k_sweep_scatter<K, V, ArraySource<K, V>, Sink><<<tiles, kScatterBlock, 0, s>>>(
            ArraySource<K, V>{a, va}, b, *last, static_cast<uint32_t>(N), shift, dm, tag, hp, status.get(), ctrs + p,
            fail_flag);
    } else if (p == 0) {
      k_sweep_scatter<K, V, Src, ArraySink<K, V>><<<tiles, kScatterBlock, 0, s>>>(
          first, b, to, static_cast<uint32_t>(N), shift, dm, tag, hp, status.get(), ctrs + p, fail_flag);
    } else {
      k_sweep_scatter<K, V, ArraySource<K, V>, ArraySink<K, V>><<<tiles, kScatterBlock, 0, s>>>(
          ArraySource<K, V>{a, va}, b, to, static_cast<uint32_t>(N), shift, dm, tag, hp, status.get(), ctrs + p,
          fail_flag);
    }
    TC_LAUNCH_CHECK();
    std::swap(a, b);
    std::swap(va, vb);
    hook(p, static_cast<const K*>(a));
  }
  vals = va;
  if (!fail_dev) {
    uint32_t h_fail = 0;
    TC_HIP(hipMemcpyAsync(&h_fail, fail_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h_fail) fail(TC_E_DEVICE, "radix_sort: a tile's look-back did not complete");
  }
  return a;
}

// radix_sort_from with the first pass reading `keys` and `vals` themselves.
template <typename K, typename V, typename Hook = NoHook>
K* radix_sort_pairs(K* keys, K* tmp, V*& vals, V* vtmp, size_t N, int bit_lo, int bit_hi, hipStream_t s,
                    uint32_t* fail_dev = nullptr, Hook hook = Hook()) {
  return radix_sort_from<K, V, ArraySource<K, V>, Hook>(ArraySource<K, V>{keys, vals}, keys, tmp, vals, vtmp, N,
                                                        bit_lo, bit_hi, s, fail_dev, hook);
}

// Keys-only form of radix_sort_pairs.
template <typename K, typename Hook = NoHook>
K* radix_sort(K* keys, K* tmp, size_t N, int bit_lo, int bit_hi, hipStream_t s, uint32_t* fail_dev = nullptr,
              Hook hook = Hook()) {
  NoVal* none = nullptr;
  return radix_sort_pairs<K, NoVal, Hook>(keys, tmp, none, nullptr, N, bit_lo, bit_hi, s, fail_dev, hook);
}

}  // namespace tc
