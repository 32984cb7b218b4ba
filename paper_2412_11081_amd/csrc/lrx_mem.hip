// Device memory cache of the library, one per device, shared by every
// context of the process.
//
// Contexts that come and go (a serving stream) would otherwise hand device
// memory back to the driver and map it again for the next request; memory
// that comes back from the driver must be cleared first, and while it is
// cleared the runtime holds up every thread's allocations and launches.  The
// cache (lrx_cache.h) keeps what it has mapped with hipMalloc until
// lrx_pool_trim.  Callers free a block only once the work that used it has
// finished (a context synchronises its stream first).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "lrx_cache.h"
#include "lrx_internal.h"

namespace lrx {
namespace {

struct HipMapper {
  void* map(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void unmap(void* p) { (void)hipFree(p); }
  void quiesce() { (void)hipDeviceSynchronize(); }
};

struct DeviceCache {
  std::mutex mu;
  BlockCache<HipMapper> cache;
};

std::mutex g_caches_mu;
std::map<int, DeviceCache*> g_caches;   // never destroyed: contexts may be destroyed during static teardown

DeviceCache& cache_of(int device) {
  std::lock_guard<std::mutex> lk(g_caches_mu);
  DeviceCache*& c = g_caches[device];
  if (!c) c = new DeviceCache();
  return *c;
}

}  // namespace

// The caller has made `device` current (hipMalloc maps on the current device).
void* dev_alloc(int device, size_t bytes) {
  DeviceCache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  return C.cache.alloc(bytes);
}

void dev_free(int device, void* p) {
  if (!p) return;
  DeviceCache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  (void)C.cache.free(p);
}

size_t dev_trim(int device, size_t keep) {
  DeviceCache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  return C.cache.trim(keep);
}

void dev_cache_bytes(int device, size_t* mapped, size_t* used) {
  DeviceCache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  if (mapped) *mapped = C.cache.mapped();
  if (used) *used = C.cache.used();
}

}  // namespace lrx
