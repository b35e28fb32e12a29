// Tuned choices of the library's automatic settings, read from a table the autotuner writes
// (paper_2101_12164_amd/autotune.py) and that ships beside the shared library as tuning_<arch>.tsv.
//
// Each line: arch <TAB> kernel <TAB> precision <TAB> size_lo <TAB> size_hi <TAB> value, with precision f64, f32,
// bf16 or * and the size class [size_lo, size_hi] in the unit the kernel's entry names (columns of a block for
// the sweeps and products, interface rows for the iteration graphs).  The first line matching the device's
// architecture, the kernel, the precision and the size wins; with no match the built-in default is used.
// Explicit options (ns_options) always take precedence over the table.
#include <dlfcn.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ns_internal.h"

namespace ns {
namespace {

struct Entry {
  std::string kernel, prec;
  int64_t lo = 0, hi = 0;
  int value = 0;
};

struct Table {
  bool loaded = false;
  std::string arch, path;
  std::vector<Entry> entries;
};

std::mutex g_tune_mu;
Table g_table;
std::vector<std::pair<std::string, int>> g_override;  // process-wide values that take precedence (the tuner)

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string library_dir() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&device_arch), &info) == 0 || !info.dli_fname) return ".";
  std::string p = info.dli_fname;
  const size_t s = p.rfind('/');
  return s == std::string::npos ? "." : p.substr(0, s);
}

void load(Table& t) {
  t.loaded = true;
  t.arch = device_arch();
  if (t.arch.empty()) return;
  t.path = library_dir() + "/tuning_" + t.arch + ".tsv";
  std::ifstream f(t.path);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ss(line);
    std::string arch;
    Entry e;
    if (!(ss >> arch >> e.kernel >> e.prec >> e.lo >> e.hi >> e.value)) continue;
    if (arch != t.arch) continue;
    t.entries.push_back(e);
  }
}

}  // namespace

int tuned(const char* kernel, const char* prec, int64_t size, int fallback) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (!g_table.loaded) load(g_table);
  for (const auto& o : g_override)
    if (o.first == kernel) return o.second;
  for (const Entry& e : g_table.entries)
    if (e.kernel == kernel && (e.prec == "*" || e.prec == prec) && size >= e.lo && size <= e.hi) return e.value;
  return fallback;
}

}  // namespace ns

extern "C" {

// Number of table entries loaded for the current device and the table's path (HOST buffer, may be NULL).
int32_t nystrom_schur_tuning_info(char* path, int32_t cap) {
  std::lock_guard<std::mutex> g(ns::g_tune_mu);
  if (!ns::g_table.loaded) ns::load(ns::g_table);
  if (path && cap > 0) std::snprintf(path, size_t(cap), "%s", ns::g_table.path.c_str());
  return int32_t(ns::g_table.entries.size());
}

// Process-wide value of an automatic setting that takes precedence over the table (value 0 removes it); for
// the autotuner, which times the candidates.  Returns 0, or -1 for a NULL kernel name.
int32_t nystrom_schur_tuning_override(const char* kernel, int32_t value) {
  if (!kernel) return -1;
  std::lock_guard<std::mutex> g(ns::g_tune_mu);
  auto& v = ns::g_override;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].first == kernel) {
      v.erase(v.begin() + i);
      break;
    }
  if (value != 0) v.emplace_back(kernel, value);
  return 0;
}

}  // extern "C"
