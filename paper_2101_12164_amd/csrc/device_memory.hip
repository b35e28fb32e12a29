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

// Pinned staging areas of the calling thread.  An area serves one stream at a time: copies from
// base[0, used) may be in flight on st, and ev is recorded after the last of them.  An area whose copies
// have completed is handed to whichever stream asks next, so streams that come and go (one per handle)
// share a few areas.  Areas are allocated on first use and kept until the process ends.
struct Staging {
  hipStream_t st = nullptr;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
constexpr int STAGE_AREAS = 8;  // areas per thread
thread_local Staging g_stage[STAGE_AREAS];
thread_local int g_nstage = 0;
thread_local bool g_stage_failed = false;
constexpr size_t STAGE_BYTES = size_t(4) << 20;

// true when every copy from area s has completed
bool area_idle(Staging& s) {
  if (!s.pending) return true;
  const hipError_t e = hipEventQuery(s.ev);
  if (e == hipSuccess) {
    s.pending = false;
    s.used = 0;
    return true;
  }
  (void)hipGetLastError();  // not-ready is reported as an error code
  return false;
}

// An area for `need` bytes of copies on stream st, or nullptr (then the copy waits on the host).
Staging* staging_for(hipStream_t st, size_t need) {
  // the stream's own area while it has room (its copies are ordered on st)
  for (int i = 0; i < g_nstage; ++i) {
    Staging& s = g_stage[i];
    if (s.st != st) continue;
    if (!s.pending) s.used = 0;
    if (s.used + need <= s.cap) return &s;
  }
  // an area whose copies have all completed
  for (int i = 0; i < g_nstage; ++i)
    if (area_idle(g_stage[i])) {
      g_stage[i].st = st;
      return &g_stage[i];
    }
  if (!g_stage_failed && g_nstage < STAGE_AREAS) {
    void* b = nullptr;
    hipEvent_t e = nullptr;
    if (hipHostMalloc(&b, STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      g_stage_failed = true;
      return nullptr;
    }
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(b);
      g_stage_failed = true;
      return nullptr;
    }
    Staging& s = g_stage[g_nstage++];
    s.st = st;
    s.base = static_cast<char*>(b);
    s.cap = STAGE_BYTES;
    s.ev = e;
    return &s;
  }
  if (g_nstage == 0) return nullptr;
  // every area is busy: wait for the stream's own area (or the first one) to drain
  Staging* s = &g_stage[0];
  for (int i = 0; i < g_nstage; ++i)
    if (g_stage[i].st == st) s = &g_stage[i];
  if (s->pending) NS_HIP(hipEventSynchronize(s->ev));
  s->pending = false;
  s->used = 0;
  s->st = st;
  return s;
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
    bool ready = b.st == st;
    if (!ready) {
      // not-ready (and, inside a stream capture, "not permitted") come back as error codes: clear each one
      // here, before a later launch check could report it
      ready = hipEventQuery(b.ev) == hipSuccess;
      if (!ready) (void)hipGetLastError();
    }
    if (ready) {
      Block blk = b;
      idle.erase(it);
      c.live[blk.p] = blk;
      return blk.p;
    }
  }
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
  const size_t need = (bytes + 255) & ~size_t(255);
  Staging* s = need <= STAGE_BYTES ? staging_for(st, need) : nullptr;
  if (!s) {
    // no staging area, or too large for one: a copy the host waits for
    NS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    NS_HIP(hipStreamSynchronize(st));
    return;
  }
  std::memcpy(s->base + s->used, src, bytes);
  NS_HIP(hipMemcpyAsync(dst, s->base + s->used, bytes, hipMemcpyHostToDevice, st));
  NS_HIP(hipEventRecord(s->ev, st));
  s->used += need;
  s->pending = true;
}

void* pinned_scratch(size_t bytes) {
  constexpr size_t CAP = 4096;
  thread_local void* buf = nullptr;
  if (bytes > CAP) fail(INVALID_ARG, "pinned scratch request too large");
  if (!buf) NS_HIP(hipHostMalloc(&buf, CAP, hipHostMallocDefault));
  return buf;
}

void stream_idle(hipStream_t st) {
  for (int i = 0; i < g_nstage; ++i)
    if (g_stage[i].st == st) {
      g_stage[i].used = 0;
      g_stage[i].pending = false;
    }
}

}  // namespace ns
