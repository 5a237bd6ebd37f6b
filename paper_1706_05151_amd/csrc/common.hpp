// Shared host/device utilities of the triangle-counting library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <exception>
#include <stdexcept>
#include <string>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;
// Most vertices a graph may have: grid-stride loops over vertices count in
// int32 with strides of at most 2^24, so n + 2^24 must stay below 2^31.
constexpr int32_t kMaxVertices = (1 << 30) + ((1 << 30) - (1 << 25));

// ------------------------------------------------------------ host errors --

struct Failure : std::runtime_error {
  tc_status status;
  Failure(tc_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(tc_status s, const std::string& m) { throw Failure(s, m); }

inline void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  std::string msg = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")";
  (void)hipGetLastError();  // clear the sticky-free error state for the next call
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) throw Failure(TC_E_NOMEM, msg);
  throw Failure(TC_E_DEVICE, msg);
}

#define TC_HIP(x) ::tc::hip_check((x), #x, __FILE__, __LINE__)
#define TC_LAUNCH_CHECK() ::tc::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ------------------------------------------------------- device memory --

// Device memory from the library's per-device block cache (memory.hip).
// dev_alloc: the block is usable by work queued on `s` after the call.
// dev_free: the block may be reused once the work queued on `s` before the
// call is done; work on other streams must be finished by the caller.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
void dev_release_cached();   // returns the current device's idle blocks to the driver
size_t dev_cached_bytes();   // idle bytes held for the current device
size_t dev_reserved_bytes(const void* p);  // bytes of the live block at p (current device), 0 if none
size_t dev_block_bytes(size_t bytes);      // bytes a request of `bytes` reserves

// Scratch buffer released on destruction, ordered after the work queued on its stream.
template <typename T>
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(size_t count, hipStream_t s) { alloc(count, s); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), s_(o.s_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_; n_ = o.n_; s_ = o.s_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  void alloc(size_t count, hipStream_t s) {
    release();
    s_ = s;
    n_ = count;
    if (count == 0) return;
    p_ = static_cast<T*>(dev_alloc(count * sizeof(T), s));
  }
  void release() {
    if (p_) dev_free(p_, s_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  T* detach() { T* p = p_; p_ = nullptr; n_ = 0; return p; }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  hipStream_t s_ = nullptr;
};

// Pinned host words for small device-to-host readbacks on stream s, taken
// from a process-wide pool (memory.hip) and given back on destruction. A copy
// into pinned memory is one asynchronous transfer; into pageable memory the
// runtime stages every copy and waits for it. Values are read only after a
// synchronisation of s that follows the copy; when an exception unwinds past
// the words, s is synchronised first, so no copy still in flight lands in
// words handed to another caller.
constexpr int kHostWords = 16;
uint64_t* host_words_take();
void host_words_give(uint64_t* p);

class HostWords {
 public:
  explicit HostWords(hipStream_t s) : p_(host_words_take()), s_(s), unwinding_(std::uncaught_exceptions()) {}
  ~HostWords() {
    if (std::uncaught_exceptions() > unwinding_) (void)hipStreamSynchronize(s_);
    host_words_give(p_);
  }
  HostWords(const HostWords&) = delete;
  HostWords& operator=(const HostWords&) = delete;
  uint64_t* get() const { return p_; }
  uint64_t operator[](int i) const { return p_[i]; }

 private:
  uint64_t* p_;
  hipStream_t s_;
  int unwinding_;
};

inline int bits_for(uint64_t max_value) {  // bits needed to hold values 0..max_value
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) b++;
  return b < 1 ? 1 : b;
}

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap = 1u << 30) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

// ------------------------------------------------------- device helpers --

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane_id() >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    T y = __shfl_xor(x, d, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// Exclusive scan across a block of BLOCK threads; `smem` holds BLOCK/64 T.
// Returns the exclusive prefix of x and writes the block total to `total`.
template <typename T, int BLOCK>
__device__ __forceinline__ T block_excl_scan(T x, T* smem, T& total) {
  constexpr int NW = BLOCK / kWave;
  const int w = threadIdx.x / kWave;
  T incl = wave_incl_scan(x);
  if (lane_id() == kWave - 1) smem[w] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    T s = smem[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + incl - x;
}

}  // namespace tc
