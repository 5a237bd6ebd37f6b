// Device memory of the library: a per-device cache of freed blocks.
//
// Returning device memory to the driver is slow (the driver clears memory it
// takes back), and the stream-ordered pool of the runtime hands freed memory
// back at synchronisation points. Graph builds and queries allocate the same
// large sizes again and again, so the library keeps freed blocks itself:
//
//  * requests of at most 1 MiB take a block of the next power of two (at least
//    4 KiB) carved from 2 MiB slabs, kept per size class when freed (slabs
//    stay with the library until the process ends), so a small graph does not
//    hold a 2 MiB block per array;
//  * larger sizes are rounded up to 2 MiB; a request takes the smallest cached
//    block that is at least as large and at most 25 % larger;
//  * a freed block gets an event recorded on the freeing stream; the stream
//    that takes the block next waits on that event (stream-ordered reuse, no
//    host synchronisation). An allocation prefers a block freed on its own
//    stream or one whose event has completed, so that work on one stream (a
//    graph build) does not queue behind unrelated work on another (a batch of
//    queries) just because that work freed the last block of the size;
//  * cached bytes are bounded (kCacheLimit); above the bound the largest
//    blocks go back to the driver, and an allocation that fails for lack of
//    memory returns every cached block of its device and tries again.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace tc {
namespace {

constexpr size_t kGranule = size_t(2) << 20;
constexpr size_t kCacheLimit = size_t(96) << 30;
constexpr int kMaxDevices = 64;

constexpr size_t kSmallMin = size_t(4) << 10;  // smallest size class
constexpr size_t kSmallMax = size_t(1) << 20;  // largest size class
constexpr int kClasses = 9;                    // 4 KiB, 8 KiB, ..., 1 MiB

struct Block {
  size_t bytes;
  hipEvent_t ready;             // recorded when the block was freed (null: never used)
  hipStream_t freed_on = nullptr;  // the stream it was freed on
};

// Blocks are looked at this far back from the most recently freed when a
// reusable one is searched for.
constexpr int kReuseScan = 16;

// A block the stream s can take without waiting on another stream's work.
bool free_for(const Block& b, hipStream_t s) {
  if (!b.ready || b.freed_on == s) return true;
  const hipError_t e = hipEventQuery(b.ready);
  if (e == hipSuccess) return true;
  (void)hipGetLastError();  // hipErrorNotReady
  return false;
}

struct DeviceCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<void*, Block>> idle;  // by size
  std::unordered_map<void*, Block> live;
  size_t idle_bytes = 0;
  std::vector<std::pair<void*, Block>> small_free[kClasses];  // freed blocks of each size class
  std::vector<void*> small_fresh[kClasses];                   // blocks of each size class never used
};

int small_class(size_t bytes) {
  int k = 0;
  for (size_t c = kSmallMin; c < bytes; c <<= 1) k++;
  return k;
}

// Never destroyed: the runtime may be gone when static destructors run.
DeviceCache* cache_of(int dev) {
  static DeviceCache* caches = new DeviceCache[kMaxDevices];
  return &caches[dev];
}

int current_device() {
  int dev = 0;
  TC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(TC_E_DEVICE, "device index out of range");
  return dev;
}

// Caller holds c.mu. Returns one idle block to the driver.
void drop_idle(DeviceCache& c, std::multimap<size_t, std::pair<void*, Block>>::iterator it) {
  Block b = it->second.second;
  void* p = it->second.first;
  c.idle.erase(it);
  c.idle_bytes -= b.bytes;
  (void)hipEventSynchronize(b.ready);
  (void)hipEventDestroy(b.ready);
  (void)hipFree(p);
}

// Caller holds c.mu. hipMalloc, returning every idle block first if the device is full.
hipError_t malloc_or_drop(DeviceCache& c, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    while (!c.idle.empty()) drop_idle(c, c.idle.begin());
    e = hipMalloc(p, bytes);
  }
  return e;
}

// Caller holds c.mu. A block of size class k for stream s: the latest freed block if s freed
// it; else the first of the oldest freed blocks whose work is done; else a block never used
// (a new slab is carved when none is left). Freed blocks that are still in use elsewhere are
// passed over, not waited for; they are taken once their work is done.
void* small_alloc(DeviceCache& c, int k, hipStream_t s) {
  const size_t cb = kSmallMin << k;
  auto& fl = c.small_free[k];
  auto take = [&](size_t i) {
    const auto blk = fl[i];
    fl[i] = fl.back();
    fl.pop_back();
    c.live.emplace(blk.first, Block{cb, blk.second.ready, nullptr});
    return blk.first;
  };
  if (!fl.empty() && fl.back().second.freed_on == s) return take(fl.size() - 1);
  for (size_t i = 0; i < fl.size() && i < static_cast<size_t>(kReuseScan); i++)
    if (free_for(fl[i].second, s)) return take(i);
  auto& fresh = c.small_fresh[k];
  if (fresh.empty()) {
    void* slab = nullptr;
    TC_HIP(malloc_or_drop(c, &slab, kGranule));
    for (size_t off = kGranule; off >= cb; off -= cb) fresh.push_back(static_cast<char*>(slab) + off - cb);
  }
  void* p = fresh.back();
  fresh.pop_back();
  c.live.emplace(p, Block{cb, nullptr, nullptr});
  return p;
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  if (bytes <= kSmallMax) return small_alloc(c, small_class(bytes), s);
  const size_t rb = (bytes + kGranule - 1) / kGranule * kGranule;
  auto it = c.idle.lower_bound(rb);
  if (it != c.idle.end() && it->first <= rb + rb / 4) {
    // among the blocks that fit, one that s can take without waiting, else the smallest
    auto pick = it;
    int seen = 0;
    for (auto j = it; j != c.idle.end() && j->first <= rb + rb / 4 && seen < kReuseScan; ++j, ++seen) {
      if (free_for(j->second.second, s)) {
        pick = j;
        break;
      }
    }
    void* p = pick->second.first;
    const Block b = pick->second.second;
    c.idle.erase(pick);
    c.idle_bytes -= b.bytes;
    c.live.emplace(p, Block{b.bytes, b.ready, nullptr});
    if (b.freed_on != s) TC_HIP(hipStreamWaitEvent(s, b.ready, 0));
    return p;
  }
  void* p = nullptr;
  hipError_t e = malloc_or_drop(c, &p, rb);
  TC_HIP(e);
  hipEvent_t ev;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(p);
    TC_HIP(e);
  }
  c.live.emplace(p, Block{rb, ev, nullptr});
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;  // not ours
  Block b = it->second;
  c.live.erase(it);
  if (b.bytes <= kSmallMax) {  // back to its size class, ready once s passes this point
    if (!b.ready && hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);  // no event: the block is free once s has drained
      b.ready = nullptr;
    }
    if (b.ready && hipEventRecord(b.ready, s) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
    }
    b.freed_on = s;
    c.small_free[small_class(b.bytes)].emplace_back(p, b);
    return;
  }
  if (hipEventRecord(b.ready, s) != hipSuccess) {
    // the stream is unusable: wait for the device instead and give the block back
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    (void)hipEventDestroy(b.ready);
    (void)hipFree(p);
    return;
  }
  b.freed_on = s;
  c.idle.emplace(b.bytes, std::make_pair(p, b));
  c.idle_bytes += b.bytes;
  while (c.idle_bytes > kCacheLimit) drop_idle(c, std::prev(c.idle.end()));
}

void dev_release_cached() {
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  while (!c.idle.empty()) drop_idle(c, c.idle.begin());
}

size_t dev_reserved_bytes(const void* p) {
  if (!p) return 0;
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(const_cast<void*>(p));
  return it == c.live.end() ? 0 : it->second.bytes;
}

size_t dev_block_bytes(size_t bytes) {
  if (bytes == 0) return 0;
  if (bytes <= kSmallMax) return kSmallMin << small_class(bytes);
  return (bytes + kGranule - 1) / kGranule * kGranule;
}

size_t dev_cached_bytes() {
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  return c.idle_bytes;
}

// ---- pinned host words: slabs of 64 slots, never returned (a few KiB per
// readback in flight at once); pageable slabs if pinned memory is refused

namespace {
std::mutex g_words_mu;
std::vector<uint64_t*> g_words_free;
}  // namespace

uint64_t* host_words_take() {
  std::lock_guard<std::mutex> lk(g_words_mu);
  if (g_words_free.empty()) {
    constexpr int kSlots = 64;
    const size_t bytes = sizeof(uint64_t) * kHostWords * kSlots;
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      p = new uint64_t[static_cast<size_t>(kHostWords) * kSlots];
    }
    for (int i = 0; i < kSlots; i++) g_words_free.push_back(static_cast<uint64_t*>(p) + static_cast<size_t>(i) * kHostWords);
  }
  uint64_t* w = g_words_free.back();
  g_words_free.pop_back();
  return w;
}

void host_words_give(uint64_t* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_words_mu);
  g_words_free.push_back(p);
}

}  // namespace tc
