// Device memory of the library.
//
// Handles (data, plans and their schedules) are created and freed once per
// batch. A HIP allocation maps fresh memory every time (tens to hundreds of
// microseconds per call, during which the GPU waits for the next launch),
// so released handle blocks are kept in a cache keyed by device and size
// class and handed out again to the next request of that class. Handle
// frees synchronise the device before releasing their blocks, as hipFree
// does, so a cached block is idle whichever stream used it.
//
// Scratch that a call allocates and frees in stream order comes from a
// stream-ordered pool per device that keeps its memory between calls.
#include <map>
#include <mutex>
#include <unordered_map>

#include "smart_internal.h"

namespace smart {

namespace {

struct Block {
  size_t bytes;
  int device;
};

struct Cache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void*> free_blocks;  // (device, class) -> block
  std::unordered_map<void*, Block> live;                      // every block handed out
  std::unordered_map<int, size_t> cached_bytes, cap;
  std::unordered_map<int, hipMemPool_t> pools;
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: frees may come from static destructors
  return *c;
}

// Size class: 256-byte minimum, then 8 classes per power of two (a block
// is at most 1/8 larger than its request).
size_t size_class(size_t bytes) {
  size_t b = bytes < 256 ? 256 : bytes;
  int top = 63 - __builtin_clzll((unsigned long long)b);
  const size_t step = top >= 3 ? (size_t)1 << (top - 3) : 1;
  return (b + step - 1) / step * step;
}

size_t cap_of(Cache& c, int dev) {
  auto it = c.cap.find(dev);
  if (it != c.cap.end()) return it->second;
  size_t fr = 0, tot = 0;
  const size_t cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 4 : ((size_t)16 << 30);
  c.cap[dev] = cap;
  return cap;
}

void trim_locked(Cache& c, int dev) {
  for (auto it = c.free_blocks.begin(); it != c.free_blocks.end();) {
    if (it->first.first == dev) {
      (void)hipFree(it->second);
      it = c.free_blocks.erase(it);
    } else {
      ++it;
    }
  }
  c.cached_bytes[dev] = 0;
}

}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = size_class(bytes);
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.free_blocks.find({dev, cls});
  if (it != c.free_blocks.end()) {
    *p = it->second;
    c.free_blocks.erase(it);
    c.cached_bytes[dev] -= cls;
  } else {
    e = hipMalloc(p, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim_locked(c, dev);  // give the cached blocks back and try once more
      e = hipMalloc(p, cls);
      if (e != hipSuccess) {
        *p = nullptr;
        return e;
      }
    }
  }
  c.live[*p] = Block{cls, dev};
  return hipSuccess;
}

void dev_release(void* p) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) {  // not a block of this cache
    (void)hipFree(p);
    return;
  }
  const Block b = it->second;
  c.live.erase(it);
  if (c.cached_bytes[b.device] + b.bytes > cap_of(c, b.device)) {
    (void)hipFree(p);
    return;
  }
  c.free_blocks.insert({{b.device, b.bytes}, p});
  c.cached_bytes[b.device] += b.bytes;
}

void dev_trim(int device) {
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  trim_locked(c, device);
}

hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipMemPool_t pool = nullptr;
  {
    Cache& c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.pools.find(dev);
    if (it != c.pools.end()) {
      pool = it->second;
    } else {
      hipMemPoolProps props{};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      e = hipMemPoolCreate(&pool, &props);
      if (e != hipSuccess) return e;
      uint64_t keep = ~(uint64_t)0;  // keep freed memory in the pool
      e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return e;
      }
      c.pools[dev] = pool;
    }
  }
  return hipMallocFromPoolAsync(p, bytes ? bytes : 1, pool, st);
}

void scratch_free(void* p, hipStream_t st) {
  if (p) (void)hipFreeAsync(p, st);
}

}  // namespace smart
