// Device memory cache and pinned staging of host-to-device copies.
//
// hipMalloc and hipFree (and their stream-ordered forms) cost tens to hundreds
// of microseconds per call and hipFree synchronises the device, so a setup
// made of many short launches with buffers allocated and freed between them
// would spend milliseconds in the allocator.  Freed buffers are instead kept
// in a per-device cache and handed out again: a block freed on the calling
// stream is reused at once (stream order protects the work still reading
// it), a block freed on another stream once an event recorded at the free has
// completed.  Metadata uploads go through a pinned staging area so the host
// never waits on them.
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "ns_internal.h"

namespace ns {

hipStream_t& alloc_stream() {
  thread_local hipStream_t s = nullptr;
  return s;
}

namespace {

constexpr int MAX_DEVICES = 64;

struct Block {
  void* p = nullptr;
  size_t size = 0;
  int dev = 0;
  hipStream_t st = nullptr;  // stream of the last free
  hipEvent_t ev = nullptr;   // recorded on st at the last free
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Block> idle[MAX_DEVICES];  // freed blocks by size
  std::unordered_map<void*, Block> live;
};

Cache& cache() {
  static Cache* c = new Cache();  // process lifetime: the blocks are returned when the process ends
  return *c;
}

size_t round_size(size_t b) {
  const size_t small = size_t(1) << 20, big = size_t(2) << 20;
  return b <= small ? (b + 511) & ~size_t(511) : (b + big - 1) / big * big;
}

// Return every idle block of device dev to the driver (before retrying an allocation that failed).
void release_idle(Cache& c, int dev) {
  (void)hipDeviceSynchronize();
  for (auto& kv : c.idle[dev]) {
    (void)hipFree(kv.second.p);
    if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
  }
  c.idle[dev].clear();
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
  if (dev < 0 || dev >= MAX_DEVICES) fail(HIP, "device index out of range");
  const size_t size = round_size(bytes);
  const size_t limit = size + size / 4 + 4096;  // reuse blocks up to a quarter larger
  hipStream_t st = alloc_stream();
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto& idle = c.idle[dev];
  for (auto it = idle.lower_bound(size); it != idle.end() && it->first <= limit; ++it) {
    Block& b = it->second;
    if (b.st == st || hipEventQuery(b.ev) == hipSuccess) {
      Block blk = b;
      idle.erase(it);
      c.live[blk.p] = blk;
      return blk.p;
    }
  }
  (void)hipGetLastError();  // hipEventQuery reports not-ready as an error code
  Block blk;
  blk.size = size;
  blk.dev = dev;
  hipError_t e = hipMalloc(&blk.p, size);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_idle(c, dev);
    blk.p = nullptr;
    e = hipMalloc(&blk.p, size);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c.live[blk.p] = blk;
  return blk.p;
}

void dev_free(void* p) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  Block b = it->second;
  c.live.erase(it);
  b.st = alloc_stream();
  if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) b.ev = nullptr;
  if (!b.ev || hipEventRecord(b.ev, b.st) != hipSuccess) {
    // no event to order a reuse by: keep the block out of the cache
    (void)hipGetLastError();
    (void)hipStreamSynchronize(b.st);
    (void)hipFree(b.p);
    if (b.ev) (void)hipEventDestroy(b.ev);
    return;
  }
  c.idle[b.dev].emplace(b.size, b);
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
