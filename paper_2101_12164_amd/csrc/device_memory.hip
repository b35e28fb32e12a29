// Stream-ordered device memory and pinned staging of host-to-device copies.
//
// hipMalloc and hipFree wait for the device (hipFree synchronises it), so a
// setup made of many short launches with buffers allocated and freed between
// them would leave the GPU idle at every allocation.  Buffers are instead
// taken from the device's default memory pool in stream order, and metadata
// uploads go through a pinned staging area so the host never waits on them.
#include <cstring>
#include <mutex>

#include "ns_internal.h"

namespace ns {

hipStream_t& alloc_stream() {
  thread_local hipStream_t s = nullptr;
  return s;
}

namespace {

constexpr int MAX_DEVICES = 64;
std::once_flag g_pool_once[MAX_DEVICES];

// Keep freed pool memory for reuse instead of returning it at each synchronisation.
void keep_pool_memory(int dev) {
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
}

// Return the pool's unused memory to the device (before retrying an allocation that failed).
void trim_pool(int dev) {
  hipMemPool_t pool = nullptr;
  (void)hipDeviceSynchronize();
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) (void)hipMemPoolTrimTo(pool, 0);
  (void)hipGetLastError();
}

// Pinned staging area of the calling thread.  Copies from base[0, used) may be in flight; ev is recorded
// after the last of them on stream st.  The area is allocated on first use and kept until the process ends.
struct Staging {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  hipEvent_t ev = nullptr;
  hipStream_t st = nullptr;
  bool pending = false, unavailable = false;
};
thread_local Staging g_stage;
constexpr size_t STAGE_BYTES = size_t(4) << 20;

bool staging_ready(Staging& s) {
  if (s.base) return true;
  if (s.unavailable) return false;
  void* b = nullptr;
  hipEvent_t e = nullptr;
  if (hipHostMalloc(&b, STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    s.unavailable = true;
    return false;
  }
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(b);
    s.unavailable = true;
    return false;
  }
  s.base = static_cast<char*>(b);
  s.cap = STAGE_BYTES;
  s.ev = e;
  return true;
}

}  // namespace

void* dev_alloc(size_t bytes) {
  int dev = 0;
  NS_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < MAX_DEVICES) std::call_once(g_pool_once[dev], keep_pool_memory, dev);
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, alloc_stream());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_pool(dev);
    p = nullptr;
    e = hipMallocAsync(&p, bytes, alloc_stream());
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFreeAsync(p, alloc_stream());
}

void upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  Staging& s = g_stage;
  const size_t need = (bytes + 255) & ~size_t(255);
  if (!staging_ready(s) || need > s.cap) {
    // no staging area, or too large for it: a copy the host waits for
    NS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    NS_HIP(hipStreamSynchronize(st));
    return;
  }
  if (s.pending && (st != s.st || s.used + need > s.cap)) {
    // copies from the area may still read it: wait for the last one (ordered after every earlier one
    // when they share a stream; on a stream switch this wait also covers the previous stream's copies)
    NS_HIP(hipEventSynchronize(s.ev));
    s.used = 0;
    s.pending = false;
  }
  if (s.used + need > s.cap) s.used = 0;
  std::memcpy(s.base + s.used, src, bytes);
  NS_HIP(hipMemcpyAsync(dst, s.base + s.used, bytes, hipMemcpyHostToDevice, st));
  NS_HIP(hipEventRecord(s.ev, st));
  s.used += need;
  s.st = st;
  s.pending = true;
}

void stream_idle(hipStream_t st) {
  Staging& s = g_stage;
  if (s.pending && s.st == st) {
    s.used = 0;
    s.pending = false;
  }
}

}  // namespace ns
