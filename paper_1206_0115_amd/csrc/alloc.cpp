// Caching device allocator.
//
// Plans are built and released repeatedly (one per charge-position set in a
// serving loop), so device blocks are recycled instead of returned to the HIP
// runtime: sizes are rounded to a size class (multiples of 256 B below 1 MiB,
// otherwise 1/8 steps between powers of two) and kept in per-device free
// lists.  On an allocation failure the cache is emptied and the allocation
// retried once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

#include "fmm_internal.h"

namespace fmm {
namespace {

struct Block {
  size_t size;
  int device;
};

std::mutex g_mu;
std::multimap<std::pair<int, size_t>, void*> g_free;  // (device, size) -> ptr
std::unordered_map<void*, Block> g_live;
size_t g_cached = 0;

size_t size_class(size_t b) {
  if (b == 0) b = 1;
  if (b < (1u << 20)) return (b + 255) & ~size_t(255);
  size_t p = 1;
  while ((p << 1) <= b) p <<= 1;
  size_t step = p / 8;
  return ((b + step - 1) / step) * step;
}

void release_all_locked() {
  for (auto& kv : g_free) hipFree(kv.second);
  g_free.clear();
  g_cached = 0;
}

}  // namespace

void* dev_alloc(size_t bytes) {
  int dev = 0;
  FMM_HIP_CHECK(hipGetDevice(&dev));
  size_t sz = size_class(bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_free.find({dev, sz});
  if (it != g_free.end()) {
    void* p = it->second;
    g_free.erase(it);
    g_cached -= sz;
    g_live[p] = {sz, dev};
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_all_locked();
    e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw FmmError{FMM_ERR_OOM, "device allocation of " + std::to_string(sz) +
                                      " bytes failed: " + hipGetErrorString(e)};
    }
  }
  g_live[p] = {sz, dev};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  g_free.insert({{it->second.device, it->second.size}, p});
  g_cached += it->second.size;
  g_live.erase(it);
}

namespace {
std::mutex g_smu;
std::multimap<int, hipStream_t> g_streams;  // device -> idle side stream
std::multimap<int, hipEvent_t> g_events;    // device -> idle event (no timing)
}  // namespace

hipStream_t side_stream_get(int device) {
  {
    std::lock_guard<std::mutex> lk(g_smu);
    auto it = g_streams.find(device);
    if (it != g_streams.end()) {
      hipStream_t s = it->second;
      g_streams.erase(it);
      return s;
    }
  }
  hipStream_t s = nullptr;
  FMM_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return s;
}

void side_stream_put(int device, hipStream_t s) {
  if (!s) return;
  if (hipStreamSynchronize(s) != hipSuccess) {  // not reused after an error
    (void)hipGetLastError();
    (void)hipStreamDestroy(s);
    return;
  }
  std::lock_guard<std::mutex> lk(g_smu);
  g_streams.insert({device, s});
}

hipEvent_t event_get(int device) {
  {
    std::lock_guard<std::mutex> lk(g_smu);
    auto it = g_events.find(device);
    if (it != g_events.end()) {
      hipEvent_t e = it->second;
      g_events.erase(it);
      return e;
    }
  }
  hipEvent_t e = nullptr;
  FMM_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return e;
}

void event_put(int device, hipEvent_t e) {
  if (!e) return;
  if (hipEventSynchronize(e) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(e);
    return;
  }
  std::lock_guard<std::mutex> lk(g_smu);
  g_events.insert({device, e});
}

// Pinned host staging for the small transfers of plan construction: copies
// between pinned memory and the device skip the driver's pageable staging.
// One buffer per thread, grown on demand and kept for the process.
void* pinned_staging(size_t bytes) {
  thread_local void* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) FMM_HIP_CHECK(hipHostFree(buf));
    buf = nullptr;
    cap = 0;
    size_t want = std::max<size_t>(bytes, size_t(1) << 16);
    FMM_HIP_CHECK(hipHostMalloc(&buf, want, hipHostMallocDefault));
    cap = want;
  }
  return buf;
}

size_t dev_cached_bytes() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_cached;
}

void dev_trim() {
  std::lock_guard<std::mutex> lk(g_mu);
  release_all_locked();
}

}  // namespace fmm
