// Opt-in per-kernel timing with HIP events (for live roofline measurement).
// When enabled, every launch of a timed kernel family is bracketed by two
// events on its stream; totals are resolved lazily when statistics are read.
#include <cstring>
#include <mutex>

#include "../../include/nystrom_schur.h"
#include "ns_internal.h"

namespace ns {
namespace {

const char* kFamilyNames[KF_COUNT] = {"chol_update",        "chol_panel",         "trsm_interior_f64",
                                      "trsm_interior_f32",  "trsm_interface_f64", "trsm_interface_f32",
                                      "schur_epi",          "spmm",               "local_schur_form",
                                      "local_schur_apply_f64", "local_schur_apply_f32",
                                      "interface_inverse_f64", "interface_inverse_f32", "mlp_forward_bf16", "mlp_backward_f32",
                                      "local_schur_apply_bf16", "interface_inverse_bf16", "gram", "block_update",
                                      "small_dense", "gram_narrow", "block_update_narrow",
                                      "local_schur_apply_narrow_f64", "interface_inverse_narrow_f64"};

struct Rec {
  hipEvent_t a, b;
  int fam;
  double bytes, flops;
};

struct KTimer {
  std::mutex mu;
  bool on = false;
  uint32_t mask = 0;  // families timed (bit f = family f)
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[KF_COUNT] = {};
  int64_t count[KF_COUNT] = {};
  double bytes[KF_COUNT] = {};
  double flops[KF_COUNT] = {};
};

KTimer& timer() {
  static KTimer* t = new KTimer();  // process lifetime
  return *t;
}

hipEvent_t get_event(KTimer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  NS_HIP(hipEventCreate(&e));
  return e;
}

void resolve(KTimer& t) {
  for (Rec& r : t.pending) {
    NS_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    NS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    t.total_ms[r.fam] += ms;
    t.count[r.fam] += 1;
    t.bytes[r.fam] += r.bytes;
    t.flops[r.fam] += r.flops;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.pending.clear();
}

}  // namespace

KScope::KScope(int fam_, hipStream_t st_, double bytes_, double flops_)
    : fam(fam_), st(st_), bytes(bytes_), flops(flops_) {
  KTimer& t = timer();
  on = t.on && ((t.mask >> fam_) & 1u);
  if (!on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
    on = false;  // launches recorded into a graph are not timed one by one
    return;
  }
  std::lock_guard<std::mutex> g(t.mu);
  a = get_event(t);
  b = get_event(t);
  NS_HIP(hipEventRecord(a, st));
}

KScope::~KScope() {
  if (!on) return;
  KTimer& t = timer();
  std::lock_guard<std::mutex> g(t.mu);
  if (hipEventRecord(b, st) == hipSuccess) t.pending.push_back(Rec{a, b, fam, bytes, flops});
}

bool kernel_timing_in_loops(bool pcg) {
  KTimer& t = timer();
  std::lock_guard<std::mutex> g(t.mu);
  // families that run only in the setup's factorisation and formation, or in the learned layer; the PCG
  // iterations apply single columns, so the wide Gram products and block updates are not in them
  constexpr uint32_t setup_only = (1u << KF_CHOL_UPDATE) | (1u << KF_CHOL_PANEL) | (1u << KF_LS_FORM) |
                                  (1u << KF_MLP_FWD) | (1u << KF_MLP_BWD);
  const uint32_t outside =
      setup_only | (pcg ? (1u << KF_GRAM) | (1u << KF_BLOCK_UPDATE) | (1u << KF_LS_APPLY64) | (1u << KF_INV64) : 0u);
  return t.on && (t.mask & ~outside) != 0;
}

void kscope_add_work(int fam, double bytes, double flops) {
  KTimer& t = timer();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on || fam < 0 || fam >= KF_COUNT || !((t.mask >> fam) & 1u)) return;
  t.bytes[fam] += bytes;
  t.flops[fam] += flops;
}

}  // namespace ns

extern "C" {

void nystrom_schur_kernel_timing_families(uint32_t mask) {
  ns::KTimer& t = ns::timer();
  std::lock_guard<std::mutex> g(t.mu);
  try {
    ns::resolve(t);
  } catch (...) {
  }
  std::memset(t.total_ms, 0, sizeof(t.total_ms));
  std::memset(t.count, 0, sizeof(t.count));
  std::memset(t.bytes, 0, sizeof(t.bytes));
  std::memset(t.flops, 0, sizeof(t.flops));
  t.mask = mask;
  t.on = mask != 0;
}

void nystrom_schur_kernel_timing(int32_t enable) { nystrom_schur_kernel_timing_families(enable ? ~0u : 0u); }

ns_status nystrom_schur_kernel_stats(const char* family, double* total_ms, int64_t* launches, double* bytes,
                                     double* flops) {
  ns::KTimer& t = ns::timer();
  std::lock_guard<std::mutex> g(t.mu);
  try {
    ns::resolve(t);
  } catch (const ns::Error& e) {
    return ns_status(e.status);
  }
  for (int f = 0; f < ns::KF_COUNT; ++f)
    if (family && std::strcmp(family, ns::kFamilyNames[f]) == 0) {
      if (total_ms) *total_ms = t.total_ms[f];
      if (launches) *launches = t.count[f];
      if (bytes) *bytes = t.bytes[f];
      if (flops) *flops = t.flops[f];
      return NS_OK;
    }
  return NS_ERR_INVALID_ARG;
}

}  // extern "C"
