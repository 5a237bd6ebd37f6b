// The pivot-staged intersection kernel k_pivot and its LDS tables (see
// count.hip for the method). Included by count.hip only; the launch, the work
// plan and the other kernels live there.
#pragma once

#include "graph.hpp"
#include "primitives.hpp"

namespace tc {
namespace {

#ifndef TC_PIVOT_MIN_WAVES
#define TC_PIVOT_MIN_WAVES 8  // waves per SIMD the pivot kernel is compiled for (register budget)
#endif
constexpr int kPivotBlock = 512;  // threads of a pivot-kernel block (hub items are staged once per 8 waves)
constexpr int kPivotWaves = kPivotBlock / kWave;
constexpr int32_t kEmpty = -1;
constexpr int kWaveSlots = 512;          // hash slots per wave (lists up to 256 entries)
constexpr int kGroupChunk = 8;           // grouped pivots taken per queue fetch

// ------------------------------------------------------------ hashing ---

// Orders the LDS accesses of one wave around a point (lanes of a wave share
// the hash table and the record arrays).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bucketed hash set in LDS: 2^log2b buckets of 4 int32 slots. A bucket's
// slots fill in order and a full bucket spills into the next one, so a lookup
// reads one 16-byte bucket and stops there unless that bucket is full. One
// multiplicative hash h = x * 0x9E3779B1 gives both the home bucket (top
// log2b bits) and the element's filter bit in the home bucket's filter word
// (the next 5 bits).
__device__ __forceinline__ uint32_t hash_of(int32_t x) { return static_cast<uint32_t>(x) * 0x9E3779B1u; }
__device__ __forceinline__ uint32_t home_bucket(uint32_t h, int log2b) { return h >> (32 - log2b); }
__device__ __forceinline__ uint32_t filter_shift(uint32_t h, int log2b) { return (h >> (27 - log2b)) & 31u; }

__device__ __forceinline__ void bt_insert(int32_t* T, int log2b, uint32_t b, int32_t x) {
  const uint32_t mask = (1u << log2b) - 1u;
  for (;;) {
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (atomicCAS(&T[4 * b + i], kEmpty, x) == kEmpty) return;
    b = (b + 1u) & mask;
  }
}

// Smallest of slot ^ x over a bucket's four slots: zero iff x is in it.
__device__ __forceinline__ uint32_t bucket_miss(const int4& q, int32_t x) {
  const uint32_t ux = static_cast<uint32_t>(x);
  const uint32_t a = static_cast<uint32_t>(q.x) ^ ux, b = static_cast<uint32_t>(q.y) ^ ux;
  const uint32_t c = static_cast<uint32_t>(q.z) ^ ux, d = static_cast<uint32_t>(q.w) ^ ux;
  return min(min(a, b), min(c, d));
}

// Slot index of x in the full buckets after b, or -1 (a bucket spills only
// when it is full, so the search stops at the first bucket with a free slot).
__device__ __forceinline__ int bt_find_spilled(const int32_t* T, int log2b, uint32_t b, int32_t x) {
  const uint32_t mask = (1u << log2b) - 1u;
  for (;;) {
    b = (b + 1u) & mask;
    const int4 q = *reinterpret_cast<const int4*>(T + 4 * b);
    const int s = q.x == x ? 0 : q.y == x ? 1 : q.z == x ? 2 : q.w == x ? 3 : -1;
    if (s >= 0) return static_cast<int>(4 * b) + s;
    if (q.w == kEmpty) return -1;
  }
}

// Slot index of x with home bucket b, or -1 (kAnySlot if only membership is
// asked for). The home bucket is read with one 16-byte LDS read.
constexpr int kAnySlot = 0;
template <bool kSlot>
__device__ __forceinline__ int bt_find(const int32_t* T, int log2b, uint32_t b, int32_t x) {
  const int4 q = *reinterpret_cast<const int4*>(T + 4 * b);
  if (bucket_miss(q, x) == 0) {
    if (!kSlot) return kAnySlot;
    return static_cast<int>(4 * b) + (q.x == x ? 0 : q.y == x ? 1 : q.z == x ? 2 : 3);
  }
  if (q.w == kEmpty) return -1;
  return bt_find_spilled(T, log2b, b, x);
}

__device__ __forceinline__ int log2_buckets(int64_t len, int load = 1) {
  int l = 4;
  while ((1ll << l) * load < len) l++;
  return l;
}

// A staged list: the bucket table T (4 << log2b slots), a bit filter F of one
// 32-bit word per bucket (8 bits per slot, 16 per entry at two entries per
// bucket) tested before the table, and per-slot tallies C (per-node mode). A
// probe reads one 4-byte filter word; only filter hits (true hits and ~6%
// false positives) read the 16-byte bucket.
//
// Bitmap form: when the staged entries lie in a short range [lo, lo + span),
// the region holds one bit per value of the range instead; a probe is a range
// check and one 4-byte LDS read, exact. For per-node counts each bit word is
// followed by the number of set bits before it, so a hit's entry index (its
// tally slot in C, one per staged entry) is that count plus a popcount.
struct Table {
  int32_t* T;
  uint32_t* F;
  uint32_t* C;
  int log2b;
  int32_t lo;     // bitmap form: smallest staged entry
  uint32_t span;  // bitmap form: entries lie in [lo, lo + span); 0 for the hash form
  uint32_t len;   // per-node bitmap form: staged entries (tallies C[0..len))
};

// Words of a table region of 2^log2b buckets: T, then F, then C (per-node).
__host__ __device__ __forceinline__ int table_words(int log2b, bool per_node) {
  return (4 << log2b) + (1 << log2b) + (per_node ? (4 << log2b) : 0);
}

__device__ __forceinline__ Table table_at(int32_t* base, int log2b, bool per_node) {
  Table t;
  t.log2b = log2b;
  t.T = base;
  t.F = reinterpret_cast<uint32_t*>(base + (4 << log2b));
  t.C = per_node ? reinterpret_cast<uint32_t*>(base + (4 << log2b) + (1 << log2b)) : nullptr;
  t.lo = 0;
  t.span = 0;
  t.len = 0;
  return t;
}

// The table for the sorted entries list[0..len) in a region of `words`
// 32-bit words: the bitmap form if the entries' range fits the region (with
// room for the prefix words and one tally per entry in per-node mode), else
// the hash form with 2^log2b buckets.
template <int MODE>
__device__ __forceinline__ Table table_for(int32_t* base, const int32_t* list, uint32_t len, int log2b, uint32_t words) {
  if (len > 0) {
    const int32_t lo = __builtin_amdgcn_readfirstlane(list[0]);
    const uint32_t span = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(list[len - 1]) - lo) + 1u;
    if (span <= 32u * words) {
      const uint32_t W = (span + 31u) >> 5;
      // counts and listing keep one zero word after the bitmap (read by values out of range)
      if (MODE != kCountPerNode ? W + 1u <= words : 2u * W + len <= words) {
        Table t = table_at(base, log2b, false);
        t.lo = lo;
        t.span = span;
        if (MODE == kCountPerNode) {
          t.len = len;
          t.C = reinterpret_cast<uint32_t*>(base + 2u * W);
        }
        return t;
      }
    }
  }
  return table_at(base, log2b, MODE == kCountPerNode);
}

template <int MODE>
__device__ __forceinline__ void tb_clear(const Table& t, int i0, int step) {
  if (t.span) {
    const int words = MODE == kCountPerNode ? static_cast<int>((t.span + 31u) >> 5) * 2
                                            : static_cast<int>((t.span + 31u) >> 5) + 1;  // and the zero word
    for (int w = i0; w < words; w += step) t.T[w] = 0;
    if (MODE == kCountPerNode)
      for (int i = i0; i < static_cast<int>(t.len); i += step) t.C[i] = 0;
    return;
  }
  const int S = 4 << t.log2b;
  for (int s = i0; s < S; s += step) {
    t.T[s] = kEmpty;
    if (t.C) t.C[s] = 0;
  }
  for (int w = i0; w < (1 << t.log2b); w += step) t.F[w] = 0u;
}

template <int MODE>
__device__ __forceinline__ void tb_insert(const Table& t, int32_t x) {
  if (t.span) {
    const uint32_t d = static_cast<uint32_t>(x - t.lo);
    atomicOr(reinterpret_cast<uint32_t*>(t.T) + ((d >> 5) << (MODE == kCountPerNode ? 1 : 0)), 1u << (d & 31u));
    return;
  }
  const uint32_t h = hash_of(x);
  const uint32_t b = home_bucket(h, t.log2b);
  bt_insert(t.T, t.log2b, b, x);
  atomicOr(&t.F[b], 1u << filter_shift(h, t.log2b));
}

// Slot of x or -1 (MODE == kCountTotal: kAnySlot for found).
template <int MODE>
__device__ __forceinline__ int tb_find(const Table& t, int32_t x) {
  if (t.span) {
    const uint32_t d = static_cast<uint32_t>(x - t.lo);
    const bool in = d < t.span;
    if (MODE == kCountPerNode) {  // the entry's index: prefix word plus the bits below it
      if (!in) return -1;
      const uint2 v = reinterpret_cast<const uint2*>(t.T)[d >> 5];
      const uint32_t sh = d & 31u;
      if (!((v.x >> sh) & 1u)) return -1;
      return static_cast<int>(v.y + static_cast<uint32_t>(__popc(v.x & ((1u << sh) - 1u))));
    }
    // branch-free: out-of-range values read the zero word after the bitmap
    const uint32_t w = reinterpret_cast<const uint32_t*>(t.T)[in ? d >> 5 : (t.span + 31u) >> 5];
    return ((w >> (d & 31u)) & 1u) ? kAnySlot : -1;
  }
  const uint32_t h = hash_of(x);
  const uint32_t b = home_bucket(h, t.log2b);
  if (!((t.F[b] >> filter_shift(h, t.log2b)) & 1u)) return -1;
  return bt_find<MODE != kCountTotal>(t.T, t.log2b, b, x);
}

// Per-node bitmap form: writes after each bit word the number of set bits in
// the words before it. Wave form: the calling wave's lanes take consecutive
// runs of words.
__device__ __forceinline__ void tb_prefix_wave(const Table& t) {
  const uint32_t W = (t.span + 31u) >> 5, per = (W + kWave - 1) / kWave;
  const uint32_t w0 = static_cast<uint32_t>(lane_id()) * per;
  uint32_t* R = reinterpret_cast<uint32_t*>(t.T);
  uint32_t c = 0;
  for (uint32_t w = w0; w < w0 + per && w < W; w++) c += static_cast<uint32_t>(__popc(R[2 * w]));
  uint32_t run = wave_incl_scan(c) - c;
  for (uint32_t w = w0; w < w0 + per && w < W; w++) {
    R[2 * w + 1] = run;
    run += static_cast<uint32_t>(__popc(R[2 * w]));
  }
}

// Block form of tb_prefix_wave (all threads of the block call it).
__device__ __forceinline__ void tb_prefix_block(const Table& t, uint32_t* scan_tmp) {
  const uint32_t W = (t.span + 31u) >> 5, per = (W + kPivotBlock - 1) / kPivotBlock;
  const uint32_t w0 = static_cast<uint32_t>(threadIdx.x) * per;
  uint32_t* R = reinterpret_cast<uint32_t*>(t.T);
  uint32_t c = 0;
  for (uint32_t w = w0; w < w0 + per && w < W; w++) c += static_cast<uint32_t>(__popc(R[2 * w]));
  uint32_t all;
  uint32_t run = block_excl_scan<uint32_t, kPivotBlock>(c, scan_tmp, all);
  for (uint32_t w = w0; w < w0 + per && w < W; w++) {
    R[2 * w + 1] = run;
    run += static_cast<uint32_t>(__popc(R[2 * w]));
  }
}

struct KernelArgs {
  int bucket_load;  // target entries per 4-slot bucket of a hub table (1 or 2)
  const int64_t* off;
  const int32_t* adj;
  const int32_t* src;
  const InRec* rec;
  const int64_t* in_off;
  int mode;
  unsigned long long* total;
  unsigned long long* per_graph;
  const int32_t* graph_of_rank;
  unsigned long long* t_rank;
  const int32_t* order;
  int32_t* tri;
  unsigned long long* cursor;
  int64_t cap;
};

__device__ __forceinline__ void emit_triangle(const KernelArgs& a, int32_t v, int32_t u, int32_t w) {
  int32_t x = a.order[v], y = a.order[u], z = a.order[w], t;
  if (x > y) { t = x; x = y; y = t; }
  if (y > z) { t = y; y = z; z = t; }
  if (x > y) { t = x; x = y; y = t; }
  const unsigned long long pos = atomicAdd(a.cursor, 1ull);
  if (static_cast<int64_t>(pos) < a.cap) {
    a.tri[3 * pos + 0] = x;
    a.tri[3 * pos + 1] = y;
    a.tri[3 * pos + 2] = z;
  }
}

// ------------------------------------------------------------- probing ---
//
// A batch of in-edge records (one per thread) is split in two:
//   long records (suffix >= kLongMin): cut into segments of kSeg elements; a
//     whole wave takes one segment, lane L reading elements L, L+64, ... so the
//     loads are coalesced, up to four are in flight per lane, and the owning
//     record is found once per segment;
//   short records: their elements are concatenated and each lane takes
//     kPerLane consecutive ones, finding the owner by binary search.

constexpr int kPerLane = 4;
constexpr uint32_t kLongMin = 128;
constexpr uint32_t kSeg = kWave * kPerLane;

// Record arrays of one batch of NR records (NR = 256 for a block, 64 for a wave).
template <int NR>
struct BatchLds {
  uint32_t spre[NR + 1];    // exclusive prefix of lengths (short records)
  uint32_t beg[NR];
  uint32_t len[NR];
  uint32_t hits[NR];        // per-node mode: hits of each record
};

// Probe one element against the table; counts, per-node tallies and listing.
template <int MODE>
__device__ __forceinline__ uint32_t probe_one(const KernelArgs& a, int32_t u, int32_t x, const Table& tab,
                                              uint32_t* hit_rec, uint32_t rec_begin) {
  const int s = tb_find<MODE>(tab, x);
  if (s < 0) return 0u;
  if (MODE == kCountPerNode) {
    atomicAdd(&tab.C[s], 1u);
    atomicAdd(hit_rec, 1u);
  } else if (MODE == kCountList) {
    emit_triangle(a, a.src[rec_begin - 1], u, x);
  }
  return 1u;
}

// Totals only: kPerLane probes of one lane against one table form at once,
// with no branch between them, so their LDS reads are in flight together.
// Bitmap form: an element past the staged range (the kEmpty filler lies
// below every rank, so it wraps to a large offset) reads zeros: its word
// index is clamped to the zero word kept after the bitmap. Hash form: every filter
// word is read, then every bucket (lanes without a filter hit read bucket 0,
// their result masked off); only elements whose full home bucket did not
// hold them search the buckets they spill into.
template <bool kBitmap, bool kAllValid>
__device__ __forceinline__ uint32_t count_probes(const Table& t, const int32_t (&x)[kPerLane]) {
  uint32_t c = 0;
  if constexpr (kBitmap) {
    const uint32_t* W = reinterpret_cast<const uint32_t*>(t.T);
    const uint32_t zero = (t.span + 31u) >> 5;
    uint32_t d[kPerLane], w[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; i++) d[i] = static_cast<uint32_t>(x[i] - t.lo);
    // word d / 32, clamped to the zero word: bits of the last word at or past
    // span are never set, so values in [span, 32 * zero) read zeros as well
#pragma unroll
    for (int i = 0; i < kPerLane; i++) w[i] = W[min(d[i] >> 5, zero)];
    // bit d mod 32 of w (the hardware bit-field extract reads the low 5 bits of the offset)
#pragma unroll
    for (int i = 0; i < kPerLane; i++) c += __builtin_amdgcn_ubfe(w[i], d[i], 1u);
  } else {
#pragma unroll
    for (int h0 = 0; h0 < kPerLane; h0 += 2) {
      uint32_t b[2], fs[2], f[2];
      bool hit[2];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        const uint32_t h = hash_of(x[h0 + i]);
        b[i] = home_bucket(h, t.log2b);
        fs[i] = filter_shift(h, t.log2b);
      }
#pragma unroll
      for (int i = 0; i < 2; i++) f[i] = t.F[b[i]];
#pragma unroll
      for (int i = 0; i < 2; i++) hit[i] = (kAllValid || x[h0 + i] != kEmpty) && ((f[i] >> fs[i]) & 1u);
      int4 q[2];
#pragma unroll
      for (int i = 0; i < 2; i++) q[i] = reinterpret_cast<const int4*>(t.T)[hit[i] ? b[i] : 0u];
      bool spill = false;
#pragma unroll
      for (int i = 0; i < 2; i++) {
        const bool found = hit[i] && bucket_miss(q[i], x[h0 + i]) == 0;
        c += found ? 1u : 0u;
        spill = spill || (hit[i] && !found && q[i].w != kEmpty);
      }
      if (spill) {
#pragma unroll
        for (int i = 0; i < 2; i++)
          if (hit[i] && bucket_miss(q[i], x[h0 + i]) != 0 && q[i].w != kEmpty)
            c += bt_find_spilled(t.T, t.log2b, b[i], x[h0 + i]) >= 0 ? 1u : 0u;
      }
    }
  }
  return c;
}

// Totals only: the long records of probe_long with one table form.
template <bool kBitmap, int NR>
__device__ __forceinline__ uint32_t count_long(const KernelArgs& a, const BatchLds<NR>& B, uint32_t nrec, uint32_t w0,
                                               uint32_t stride, const Table& tab) {
  const int lane = lane_id();
  uint32_t cnt = 0;
  for (uint32_t j = w0; j < nrec; j += stride) {
    const uint32_t len = __builtin_amdgcn_readfirstlane(B.len[j]);
    if (len < kLongMin) continue;
    const uint32_t beg = __builtin_amdgcn_readfirstlane(B.beg[j]);
    uint32_t k0 = 0;
    for (; k0 + kSeg <= len; k0 += kSeg) {
      const int32_t* wbase = a.adj + beg + k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) x[i] = wbase[lane + kWave * i];
      cnt += count_probes<kBitmap, true>(tab, x);
    }
    if (k0 < len) {
      const uint32_t rem = len - k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) {
        const uint32_t k = static_cast<uint32_t>(lane + kWave * i);
        x[i] = k < rem ? a.adj[beg + k0 + k] : kEmpty;
      }
      cnt += count_probes<kBitmap, false>(tab, x);
    }
  }
  return cnt;
}

// Totals only: the concatenated short-record elements of probe_short with one table form.
template <bool kBitmap, int NR>
__device__ __forceinline__ uint32_t count_short(const KernelArgs& a, const BatchLds<NR>& B, uint32_t tot, int slot,
                                                int width, const Table& tab) {
  uint32_t cnt = 0;
  for (uint32_t k0 = 0; k0 < tot; k0 += static_cast<uint32_t>(width) * kPerLane) {
    const uint32_t kb = k0 + static_cast<uint32_t>(slot) * kPerLane;
    int j = 0;
    if (kb < tot) {
#pragma unroll
      for (int step = NR / 2; step > 0; step >>= 1)
        if (B.spre[j + step] <= kb) j += step;  // j + step <= NR - 1
    }
    int32_t x[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; i++) {
      const uint32_t k = kb + i;
      x[i] = kEmpty;
      if (k < tot) {
        while (B.spre[j + 1] <= k) j++;  // stops at j = NR - 1 because spre[NR] = tot > k
        x[i] = a.adj[B.beg[j] + (k - B.spre[j])];
      }
    }
    cnt += count_probes<kBitmap, false>(tab, x);
  }
  return cnt;
}

// Per-node counts: kPerLane probes of one lane against a hash table at once
// (two in flight, as in count_probes), adding one to the tally of every slot
// found. Returns the found elements as bits 0..kPerLane-1.
template <bool kAllValid>
__device__ __forceinline__ uint32_t tally_probes(const Table& t, const int32_t (&x)[kPerLane]) {
  uint32_t found_bits = 0;
#pragma unroll
  for (int h0 = 0; h0 < kPerLane; h0 += 2) {
    uint32_t b[2], fs[2], f[2];
    bool hit[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const uint32_t h = hash_of(x[h0 + i]);
      b[i] = home_bucket(h, t.log2b);
      fs[i] = filter_shift(h, t.log2b);
    }
#pragma unroll
    for (int i = 0; i < 2; i++) f[i] = t.F[b[i]];
#pragma unroll
    for (int i = 0; i < 2; i++) hit[i] = (kAllValid || x[h0 + i] != kEmpty) && ((f[i] >> fs[i]) & 1u);
    int4 q[2];
#pragma unroll
    for (int i = 0; i < 2; i++) q[i] = reinterpret_cast<const int4*>(t.T)[hit[i] ? b[i] : 0u];
#pragma unroll
    for (int i = 0; i < 2; i++) {
      if (!hit[i]) continue;
      const int32_t v = x[h0 + i];
      int slot = -1;
      if (bucket_miss(q[i], v) == 0)
        slot = static_cast<int>(4 * b[i]) + (q[i].x == v ? 0 : q[i].y == v ? 1 : q[i].z == v ? 2 : 3);
      else if (q[i].w != kEmpty)
        slot = bt_find_spilled(t.T, t.log2b, b[i], v);
      if (slot >= 0) {
        atomicAdd(&t.C[slot], 1u);
        found_bits |= 1u << (h0 + i);
      }
    }
  }
  return found_bits;
}

// Per-node counts against the bitmap form: kPerLane probes with their LDS
// reads in flight together; a hit adds one to its entry's tally.
__device__ __forceinline__ uint32_t tally_probes_bitmap(const Table& t, const int32_t (&x)[kPerLane]) {
  const uint2* R = reinterpret_cast<const uint2*>(t.T);
  uint32_t d[kPerLane];
  bool in[kPerLane];
  uint2 v[kPerLane];
#pragma unroll
  for (int i = 0; i < kPerLane; i++) {
    d[i] = static_cast<uint32_t>(x[i] - t.lo);
    in[i] = d[i] < t.span;
  }
#pragma unroll
  for (int i = 0; i < kPerLane; i++) v[i] = R[in[i] ? d[i] >> 5 : 0u];
  uint32_t found_bits = 0;
#pragma unroll
  for (int i = 0; i < kPerLane; i++) {
    const uint32_t sh = d[i] & 31u;
    if (in[i] && ((v[i].x >> sh) & 1u)) {
      atomicAdd(&t.C[v[i].y + static_cast<uint32_t>(__popc(v[i].x & ((1u << sh) - 1u)))], 1u);
      found_bits |= 1u << i;
    }
  }
  return found_bits;
}

template <bool kBitmap, bool kAllValid>
__device__ __forceinline__ uint32_t tally4(const Table& t, const int32_t (&x)[kPerLane]) {
  if constexpr (kBitmap) return tally_probes_bitmap(t, x);
  else return tally_probes<kAllValid>(t, x);
}

// Per-node counts: the long records of probe_long. A window belongs to one
// record, so the record's hits are added once per window.
template <bool kBitmap, int NR>
__device__ __forceinline__ uint32_t tally_long(const KernelArgs& a, const BatchLds<NR>& B, uint32_t nrec, uint32_t w0,
                                               uint32_t stride, const Table& tab, uint32_t* hits) {
  const int lane = lane_id();
  uint32_t cnt = 0;
  for (uint32_t j = w0; j < nrec; j += stride) {
    const uint32_t len = __builtin_amdgcn_readfirstlane(B.len[j]);
    if (len < kLongMin) continue;
    const uint32_t beg = __builtin_amdgcn_readfirstlane(B.beg[j]);
    uint32_t rec = 0;
    uint32_t k0 = 0;
    for (; k0 + kSeg <= len; k0 += kSeg) {
      const int32_t* wbase = a.adj + beg + k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) x[i] = wbase[lane + kWave * i];
      rec += static_cast<uint32_t>(__popc(tally4<kBitmap, true>(tab, x)));
    }
    if (k0 < len) {
      const uint32_t rem = len - k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) {
        const uint32_t k = static_cast<uint32_t>(lane + kWave * i);
        x[i] = k < rem ? a.adj[beg + k0 + k] : kEmpty;
      }
      rec += static_cast<uint32_t>(__popc(tally4<kBitmap, false>(tab, x)));
    }
    const uint32_t wrec = wave_sum(rec);
    if (lane == 0 && wrec) atomicAdd(&hits[j], wrec);
    cnt += rec;
  }
  return cnt;
}

// Per-node counts: the concatenated short-record elements of probe_short.
template <bool kBitmap, int NR>
__device__ __forceinline__ uint32_t tally_short(const KernelArgs& a, const BatchLds<NR>& B, uint32_t tot, int slot,
                                                int width, const Table& tab, uint32_t* hits) {
  uint32_t cnt = 0;
  for (uint32_t k0 = 0; k0 < tot; k0 += static_cast<uint32_t>(width) * kPerLane) {
    const uint32_t kb = k0 + static_cast<uint32_t>(slot) * kPerLane;
    int j = 0;
    if (kb < tot) {
#pragma unroll
      for (int step = NR / 2; step > 0; step >>= 1)
        if (B.spre[j + step] <= kb) j += step;  // j + step <= NR - 1
    }
    int32_t x[kPerLane];
    int jj[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; i++) {
      const uint32_t k = kb + i;
      jj[i] = 0;
      x[i] = kEmpty;
      if (k < tot) {
        while (B.spre[j + 1] <= k) j++;  // stops at j = NR - 1 because spre[NR] = tot > k
        jj[i] = j;
        x[i] = a.adj[B.beg[j] + (k - B.spre[j])];
      }
    }
    const uint32_t fb = tally4<kBitmap, false>(tab, x);
#pragma unroll
    for (int i = 0; i < kPerLane; i++)
      if ((fb >> i) & 1u) atomicAdd(&hits[jj[i]], 1u);
    cnt += static_cast<uint32_t>(__popc(fb));
  }
  return cnt;
}

// Long records of the batch, wave `w0` of `stride` taking records w0,
// w0+stride, ...: the wave walks a record's suffix in windows of kSeg
// elements, lane L reading elements L, L+64, L+128, L+192 of the window.
template <int MODE, int NR>
__device__ __forceinline__ uint32_t probe_long(const KernelArgs& a, int32_t u, const BatchLds<NR>& B, uint32_t nrec,
                                               uint32_t w0, uint32_t stride, const Table& tab,
                                               uint32_t* hits) {
  if constexpr (MODE == kCountTotal)
    return tab.span ? count_long<true, NR>(a, B, nrec, w0, stride, tab) : count_long<false, NR>(a, B, nrec, w0, stride, tab);
  if constexpr (MODE == kCountPerNode)
    return tab.span ? tally_long<true, NR>(a, B, nrec, w0, stride, tab, hits)
                    : tally_long<false, NR>(a, B, nrec, w0, stride, tab, hits);
  const int lane = lane_id();
  uint32_t cnt = 0;
  for (uint32_t j = w0; j < nrec; j += stride) {
    const uint32_t len = __builtin_amdgcn_readfirstlane(B.len[j]);
    if (len < kLongMin) continue;
    const uint32_t beg = __builtin_amdgcn_readfirstlane(B.beg[j]);
    uint32_t k0 = 0;
    // full windows: unguarded loads from a wave-uniform base
    for (; k0 + kSeg <= len; k0 += kSeg) {
      const int32_t* wbase = a.adj + beg + k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) x[i] = wbase[lane + kWave * i];
      uint32_t h = 0;
#pragma unroll
      for (int i = 0; i < kPerLane; i++) h += probe_one<MODE>(a, u, x[i], tab, &hits[j], beg);
      cnt += h;
    }
    if (k0 < len) {
      const uint32_t rem = len - k0;
      int32_t x[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; i++) {
        const uint32_t k = static_cast<uint32_t>(lane + kWave * i);
        x[i] = (static_cast<uint32_t>(kWave * i) < rem && k < rem) ? a.adj[beg + k0 + k] : kEmpty;
      }
      uint32_t h = 0;
#pragma unroll
      for (int i = 0; i < kPerLane; i++)
        if (x[i] != kEmpty) h += probe_one<MODE>(a, u, x[i], tab, &hits[j], beg);
      cnt += h;
    }
  }
  return cnt;
}

// Concatenated short-record elements [k_first, tot) in windows of width*kPerLane,
// this thread taking kPerLane consecutive ones at its slot `slot` of `width`.
template <int MODE, int NR>
__device__ __forceinline__ uint32_t probe_short(const KernelArgs& a, int32_t u, const BatchLds<NR>& B, uint32_t tot,
                                                int slot, int width, const Table& tab, uint32_t* hits) {
  if constexpr (MODE == kCountTotal)
    return tab.span ? count_short<true, NR>(a, B, tot, slot, width, tab) : count_short<false, NR>(a, B, tot, slot, width, tab);
  if constexpr (MODE == kCountPerNode)
    return tab.span ? tally_short<true, NR>(a, B, tot, slot, width, tab, hits)
                    : tally_short<false, NR>(a, B, tot, slot, width, tab, hits);
  uint32_t cnt = 0;
  for (uint32_t k0 = 0; k0 < tot; k0 += static_cast<uint32_t>(width) * kPerLane) {
    const uint32_t kb = k0 + static_cast<uint32_t>(slot) * kPerLane;
    int j = 0;
    if (kb < tot) {
#pragma unroll
      for (int step = NR / 2; step > 0; step >>= 1)
        if (B.spre[j + step] <= kb) j += step;  // j + step <= NR - 1
    }
    int32_t x[kPerLane];
    int jj[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; i++) {
      const uint32_t k = kb + i;
      jj[i] = -1;
      x[i] = kEmpty;
      if (k < tot) {
        while (B.spre[j + 1] <= k) j++;  // stops at j = NR - 1 because spre[NR] = tot > k
        jj[i] = j;
        x[i] = a.adj[B.beg[j] + (k - B.spre[j])];
      }
    }
#pragma unroll
    for (int i = 0; i < kPerLane; i++)
      if (jj[i] >= 0) cnt += probe_one<MODE>(a, u, x[i], tab, &hits[jj[i]], B.beg[jj[i]]);
  }
  return cnt;
}

// Fill the batch arrays for the record this thread holds (idx in [0,NR)):
// `excl`/`tot` are the exclusive prefix and total of the short-record lengths.
template <int MODE, int NR>
__device__ __forceinline__ void batch_fill(BatchLds<NR>& B, int idx, const InRec& rc, uint32_t excl, uint32_t tot) {
  B.spre[idx] = excl;
  B.beg[idx] = rc.a_begin;
  B.len[idx] = rc.a_len;
  if (MODE != kCountTotal) B.hits[idx] = 0;
  if (idx == NR - 1) B.spre[NR] = tot;
}

__device__ __forceinline__ uint32_t short_len(uint32_t len) { return len >= kLongMin ? 0u : len; }

// Block-wide batch of up to kPivotBlock records for a hub item.
template <int MODE>
__device__ __forceinline__ uint32_t probe_batch_block(const KernelArgs& a, int32_t u, uint32_t r0, uint32_t r1,
                                                      const Table& tab, BatchLds<kPivotBlock>& B, uint32_t* scan_tmp) {
  const int tid = threadIdx.x, w = tid / kWave;
  const uint32_t r = r0 + tid;
  const bool valid = r < r1;
  InRec rc{0u, 0u};
  if (valid) rc = a.rec[r];
  uint32_t tot;
  const uint32_t excl = block_excl_scan<uint32_t, kPivotBlock>(short_len(rc.a_len), scan_tmp, tot);
  batch_fill<MODE, kPivotBlock>(B, tid, rc, excl, tot);
  __syncthreads();
  uint32_t cnt = probe_long<MODE, kPivotBlock>(a, u, B, r1 - r0, static_cast<uint32_t>(w), kPivotWaves, tab, B.hits);
  cnt += probe_short<MODE, kPivotBlock>(a, u, B, tot, tid, kPivotBlock, tab, B.hits);
  __syncthreads();
  if (MODE == kCountPerNode && valid && B.hits[tid])
    atomicAdd(&a.t_rank[a.src[rc.a_begin - 1]], static_cast<unsigned long long>(B.hits[tid]));
  __syncthreads();
  return cnt;
}

// Wave-wide batch of up to 64 records for a small pivot.
template <int MODE>
__device__ __forceinline__ uint32_t probe_batch_wave(const KernelArgs& a, int32_t u, uint32_t r0, uint32_t r1,
                                                     const Table& tab, BatchLds<kWave>& B) {
  const int lane = lane_id();
  const uint32_t r = r0 + lane;
  const bool valid = r < r1;
  InRec rc{0u, 0u};
  if (valid) rc = a.rec[r];
  const uint32_t p = short_len(rc.a_len);
  const uint32_t incl = wave_incl_scan(p);
  const uint32_t tot = __shfl(incl, kWave - 1, kWave);
  batch_fill<MODE, kWave>(B, lane, rc, incl - p, tot);
  wave_sync();
  uint32_t cnt = probe_long<MODE, kWave>(a, u, B, r1 - r0, 0u, 1u, tab, B.hits);
  cnt += probe_short<MODE, kWave>(a, u, B, tot, lane, kWave, tab, B.hits);
  if (MODE == kCountPerNode) {
    wave_sync();
    if (valid && B.hits[lane]) atomicAdd(&a.t_rank[a.src[rc.a_begin - 1]], static_cast<unsigned long long>(B.hits[lane]));
  }
  wave_sync();
  return cnt;
}

constexpr int kWaveLog2b = 7;  // per-wave tables: 128 buckets (kWaveSlots slots), lists up to 256 entries
constexpr int kRegionWords = 7680;  // least dynamic LDS of a pivot block (32-bit words; 30 KiB, 4 blocks per CU)

// Dynamic LDS words of a pivot block: one hub table of 2^hub_log2b buckets
// in phase 1, kPivotWaves equal wave regions in phase 2.
__host__ __device__ __forceinline__ uint32_t pivot_region_words(int hub_log2b, bool per_node) {
  const uint32_t hub = static_cast<uint32_t>(table_words(hub_log2b, per_node));
  const uint32_t wave = static_cast<uint32_t>(kPivotWaves * table_words(kWaveLog2b, per_node));
  uint32_t r = hub > wave ? hub : wave;
  if (r < static_cast<uint32_t>(kRegionWords)) r = kRegionWords;
  return (r + kPivotWaves * 4 - 1) / (kPivotWaves * 4) * (kPivotWaves * 4);  // whole 16-byte rows per wave
}

// Per-wave staging of one small pivot (|N_u| <= 256) into the wave's region.
template <int MODE>
__device__ __forceinline__ unsigned long long wave_pivot(const KernelArgs& a, int32_t u, uint32_t ibeg, uint32_t iend,
                                                         int32_t* region, uint32_t region_words, BatchLds<kWave>& B) {
  const int lane = lane_id();
  const int64_t nb = a.off[u];
  const uint32_t nlen = static_cast<uint32_t>(a.off[u + 1] - nb);
  int log2b = log2_buckets(nlen);
  if (log2b > kWaveLog2b) log2b = kWaveLog2b;  // >= 2 slots per entry
  const Table tab = table_for<MODE>(region, a.adj + nb, nlen, log2b, region_words);
  tb_clear<MODE>(tab, lane, kWave);
  wave_sync();
  for (uint32_t k = lane; k < nlen; k += kWave) tb_insert<MODE>(tab, a.adj[nb + k]);
  wave_sync();
  if (MODE == kCountPerNode && tab.span) {
    tb_prefix_wave(tab);
    wave_sync();
  }
  uint32_t cnt = 0;
  for (uint32_t r0 = ibeg; r0 < iend; r0 += kWave)
    cnt += probe_batch_wave<MODE>(a, u, r0, iend < r0 + kWave ? iend : r0 + kWave, tab, B);
  const unsigned long long tot = wave_sum(static_cast<unsigned long long>(cnt));
  if (MODE == kCountPerNode) {
    if (tab.span) {
      for (uint32_t i = lane; i < nlen; i += kWave)
        if (tab.C[i]) atomicAdd(&a.t_rank[a.adj[nb + i]], static_cast<unsigned long long>(tab.C[i]));
    } else {
      for (int s = lane; s < (4 << log2b); s += kWave)
        if (tab.C[s]) atomicAdd(&a.t_rank[tab.T[s]], static_cast<unsigned long long>(tab.C[s]));
    }
  }
  if (lane == 0 && tot) {
    if (a.per_graph) atomicAdd(&a.per_graph[a.graph_of_rank ? a.graph_of_rank[u] : 0], tot);
    if (MODE == kCountPerNode) atomicAdd(&a.t_rank[u], tot);
  }
  wave_sync();
  return tot;
}

// One hub item processed by the whole block: stage the slice of N_u, probe
// the item's in-edge records block-wide, flush per-node tallies. Returns the
// item's triangle count (valid in thread 0).
template <int MODE>
__device__ __forceinline__ unsigned long long hub_item(const KernelArgs& a, const PivotItem& item, int32_t* region,
                                                       uint32_t region_words, BatchLds<kPivotBlock>& bl,
                                                       uint32_t* scan_tmp, unsigned long long* red) {
  const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  constexpr bool per_node = MODE == kCountPerNode;
  const int log2b = log2_buckets(item.nlen, a.bucket_load);
  const int64_t nb = a.off[item.u] + item.nbeg_rel;
  const Table tab = table_for<MODE>(region, a.adj + nb, item.nlen, log2b, region_words);
  tb_clear<MODE>(tab, tid, kPivotBlock);
  __syncthreads();
  for (uint32_t k = tid; k < item.nlen; k += kPivotBlock) tb_insert<MODE>(tab, a.adj[nb + k]);
  __syncthreads();
  if (per_node && tab.span) {
    tb_prefix_block(tab, scan_tmp);
    __syncthreads();
  }
  uint32_t cnt = 0;
  for (uint32_t r0 = item.ibeg; r0 < item.iend; r0 += kPivotBlock)
    cnt += probe_batch_block<MODE>(a, item.u, r0, item.iend < r0 + kPivotBlock ? item.iend : r0 + kPivotBlock, tab, bl,
                                   scan_tmp);
  const unsigned long long ws = wave_sum(static_cast<unsigned long long>(cnt));
  if (lane == 0) red[w] = ws;
  __syncthreads();
  if (per_node) {
    if (tab.span) {
      for (uint32_t i = tid; i < item.nlen; i += kPivotBlock)
        if (tab.C[i]) atomicAdd(&a.t_rank[a.adj[nb + i]], static_cast<unsigned long long>(tab.C[i]));
    } else {
      for (int s = tid; s < (4 << log2b); s += kPivotBlock)
        if (tab.C[s]) atomicAdd(&a.t_rank[tab.T[s]], static_cast<unsigned long long>(tab.C[s]));
    }
  }
  unsigned long long tot = 0;
  if (tid == 0) {
    for (int x = 0; x < kPivotWaves; x++) tot += red[x];
    if (tot) {
      if (a.per_graph) atomicAdd(&a.per_graph[a.graph_of_rank ? a.graph_of_rank[item.u] : 0], tot);
      if (per_node) atomicAdd(&a.t_rank[item.u], tot);
    }
  }
  __syncthreads();
  return tot;
}

// Work of many graphs in one launch: graph g's hub items, split items and
// chunks of grouped pivots follow those of graphs 0..g-1 in three global
// queues; pre[q * (k+1) + g] is the first queue index of graph g.
struct GraphDesc {
  const int64_t* off;
  const int32_t* adj;
  const int32_t* src;
  const InRec* rec;
  const int64_t* in_off;
  const PivotItem* hub;
  const PivotItem* split;
  const int32_t* grouped;
  uint64_t n_grouped;
  unsigned long long* t_rank;  // per-node counts by rank (per-node mode)
};

struct JobList {
  const GraphDesc* descs;  // [k]
  const uint64_t* pre;     // [3][k+1]
  int32_t k;
};

__device__ __forceinline__ int32_t job_of(const uint64_t* pre, int32_t k, uint64_t idx) {
  int32_t lo = 0, hi = k - 1;  // last g with pre[g] <= idx
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ KernelArgs job_args(const KernelArgs& base, const GraphDesc& d, int32_t g) {
  KernelArgs a = base;
  a.off = d.off;
  a.adj = d.adj;
  a.src = d.src;
  a.rec = d.rec;
  a.in_off = d.in_off;
  a.t_rank = d.t_rank;
  a.per_graph = base.per_graph ? base.per_graph + g : nullptr;
  a.graph_of_rank = nullptr;
  return a;
}

// The persistent intersection kernel. Phase 1: blocks take hub items from
// queue 0 (a slice of a long N_u staged by all 512 threads, in-edge records
// probed by the eight waves). Phase 2: each wave takes split items from queue 1
// and then chunks of small pivots from queue 2, each staged by the wave alone.
// The dynamic LDS region serves as the block table in phase 1 and as eight
// per-wave tables in phase 2 (a block enters phase 2 only after its phase 1).
// With MULTI the queues run over the work of the graphs of a JobList.
template <int MODE, bool MULTI>
__global__ __launch_bounds__(kPivotBlock, TC_PIVOT_MIN_WAVES) void k_pivot(
    KernelArgs a, const PivotItem* __restrict__ hub_items, uint64_t n_hub, const PivotItem* __restrict__ split_items,
    uint64_t n_split, const int32_t* __restrict__ grouped, uint64_t n_grouped, unsigned long long* __restrict__ queues,
    int hub_log2b, JobList jobs) {
  extern __shared__ int4 smem4[];
  int32_t* smem = reinterpret_cast<int32_t*>(smem4);
  // record arrays: the block's in phase 1, one per wave in phase 2
  __shared__ union {
    BatchLds<kPivotBlock> block;
    BatchLds<kWave> wave[kPivotWaves];
  } rl;
  __shared__ uint32_t scan_tmp[kPivotWaves];
  __shared__ unsigned long long cur;
  __shared__ unsigned long long red[kPivotWaves];
  const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  constexpr bool per_node = MODE == kCountPerNode;
  unsigned long long acc = 0;
  const uint32_t region_words = pivot_region_words(hub_log2b, per_node);

  // ---- phase 1: hub items, one block each
  {
    for (;;) {
      if (tid == 0) cur = n_hub ? atomicAdd(&queues[0], 1ull) : 0ull;
      __syncthreads();
      const unsigned long long it = cur;
      if (it >= n_hub) break;
      if (MULTI) {
        const int32_t g = job_of(jobs.pre, jobs.k, it);
        const GraphDesc d = jobs.descs[g];
        acc += hub_item<MODE>(job_args(a, d, g), d.hub[it - jobs.pre[g]], smem, region_words, rl.block, scan_tmp,
                              red);
      } else {
        acc += hub_item<MODE>(a, hub_items[it], smem, region_words, rl.block, scan_tmp, red);
      }
    }
  }

  // ---- phase 2: split items and grouped small pivots, one wave each
  {
    const uint32_t wave_words = region_words / kPivotWaves;
    int32_t* region = smem + w * wave_words;
    for (;;) {
      unsigned long long it = 0;
      if (lane == 0) it = n_split ? atomicAdd(&queues[1], 1ull) : 0ull;
      it = __shfl(it, 0, kWave);
      if (it >= n_split) break;
      if (MULTI) {
        const uint64_t* pre = jobs.pre + (jobs.k + 1);
        const int32_t g = job_of(pre, jobs.k, it);
        const GraphDesc d = jobs.descs[g];
        const PivotItem item = d.split[it - pre[g]];
        acc += wave_pivot<MODE>(job_args(a, d, g), item.u, item.ibeg, item.iend, region, wave_words, rl.wave[w]);
      } else {
        const PivotItem item = split_items[it];
        acc += wave_pivot<MODE>(a, item.u, item.ibeg, item.iend, region, wave_words, rl.wave[w]);
      }
    }
    for (;;) {
      unsigned long long c = 0;
      if (lane == 0) c = n_grouped ? atomicAdd(&queues[2], 1ull) : 0ull;  // one chunk of kGroupChunk pivots
      c = __shfl(c, 0, kWave);
      const uint64_t n_chunks = MULTI ? n_grouped : (n_grouped + kGroupChunk - 1) / kGroupChunk;
      if (c >= n_chunks) break;
      KernelArgs ga = a;
      const int32_t* glist = grouped;
      uint64_t g0 = c * kGroupChunk, gend = n_grouped;
      if (MULTI) {
        const uint64_t* pre = jobs.pre + 2 * (jobs.k + 1);
        const int32_t g = job_of(pre, jobs.k, c);
        const GraphDesc d = jobs.descs[g];
        ga = job_args(a, d, g);
        glist = d.grouped;
        g0 = (c - pre[g]) * kGroupChunk;
        gend = d.n_grouped;
      }
      const uint64_t g1 = g0 + kGroupChunk < gend ? g0 + kGroupChunk : gend;
      for (uint64_t x = g0; x < g1; x++) {
        const int32_t u = glist[x];
        acc += wave_pivot<MODE>(ga, u, static_cast<uint32_t>(ga.in_off[u]), static_cast<uint32_t>(ga.in_off[u + 1]),
                                region, wave_words, rl.wave[w]);
      }
    }
  }
  // phase 1 accumulates in thread 0 of each block, phase 2 in lane 0 of each wave
  if (lane == 0 && acc && a.total) atomicAdd(a.total, acc);
}

}  // namespace
}  // namespace tc
