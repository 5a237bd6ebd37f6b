// Device memory of the library: a per-device cache of freed blocks.
//
// Returning device memory to the driver is slow (the driver clears memory it
// takes back), and the stream-ordered pool of the runtime hands freed memory
// back at synchronisation points. Graph builds and queries allocate the same
// large sizes again and again, so the library keeps freed blocks itself:
//
//  * sizes are rounded up to 2 MiB; a request takes the smallest cached block
//    that is at least as large and at most 25 % larger;
//  * a freed block gets an event recorded on the freeing stream; the stream
//    that takes the block next waits on that event (stream-ordered reuse, no
//    host synchronisation);
//  * cached bytes are bounded (kCacheLimit); above the bound the largest
//    blocks go back to the driver, and an allocation that fails for lack of
//    memory returns every cached block of its device and tries again.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace tc {
namespace {

constexpr size_t kGranule = size_t(2) << 20;
constexpr size_t kCacheLimit = size_t(96) << 30;
constexpr int kMaxDevices = 64;

struct Block {
  size_t bytes;
  hipEvent_t ready;  // recorded when the block was freed
};

struct DeviceCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<void*, Block>> idle;  // by size
  std::unordered_map<void*, Block> live;
  size_t idle_bytes = 0;
};

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

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  const size_t rb = (bytes + kGranule - 1) / kGranule * kGranule;
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.idle.lower_bound(rb);
  if (it != c.idle.end() && it->first <= rb + rb / 4) {
    void* p = it->second.first;
    const Block b = it->second.second;
    c.idle.erase(it);
    c.idle_bytes -= b.bytes;
    c.live.emplace(p, b);
    TC_HIP(hipStreamWaitEvent(s, b.ready, 0));
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, rb);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    while (!c.idle.empty()) drop_idle(c, c.idle.begin());
    e = hipMalloc(&p, rb);
  }
  TC_HIP(e);
  hipEvent_t ev;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(p);
    TC_HIP(e);
  }
  c.live.emplace(p, Block{rb, ev});
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;  // not ours
  const Block b = it->second;
  c.live.erase(it);
  if (hipEventRecord(b.ready, s) != hipSuccess) {
    // the stream is unusable: wait for the device instead and give the block back
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    (void)hipEventDestroy(b.ready);
    (void)hipFree(p);
    return;
  }
  c.idle.emplace(b.bytes, std::make_pair(p, b));
  c.idle_bytes += b.bytes;
  while (c.idle_bytes > kCacheLimit) drop_idle(c, std::prev(c.idle.end()));
}

void dev_release_cached() {
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  while (!c.idle.empty()) drop_idle(c, c.idle.begin());
}

size_t dev_cached_bytes() {
  DeviceCache& c = *cache_of(current_device());
  std::lock_guard<std::mutex> lk(c.mu);
  return c.idle_bytes;
}

}  // namespace tc
