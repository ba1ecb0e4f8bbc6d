// Kernel timing with HIP events (opt-in).  When enabled with a name prefix,
// every library launch of a kernel whose name starts with that prefix is
// bracketed by two events recorded on the launch stream; bse_prof_collect()
// waits for them and accumulates the elapsed time per kernel name.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bse_internal.h"

namespace bse {
namespace {
struct Pending {
  int name;
  hipEvent_t a, b;
};
std::mutex mu;
std::string prefix;
bool on = false;
std::vector<std::string> names;
std::map<std::string, int> name_id;
std::vector<double> total_ms;
std::vector<int64_t> launches;
std::vector<Pending> pending;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : stream_(s), idx_(-1) {
  std::lock_guard<std::mutex> g(mu);
  if (!on || std::strncmp(name, prefix.c_str(), prefix.size()) != 0) return;
  auto it = name_id.find(name);
  int id;
  if (it == name_id.end()) {
    id = int(names.size());
    names.push_back(name);
    name_id[name] = id;
    total_ms.push_back(0.0);
    launches.push_back(0);
  } else {
    id = it->second;
  }
  hipEvent_t a = get_event(), b = get_event();
  if (!a || !b) return;
  if (hipEventRecord(a, s) != hipSuccess) return;
  pending.push_back(Pending{id, a, b});
  idx_ = int(pending.size()) - 1;
}

ProfScope::~ProfScope() {
  if (idx_ < 0) return;
  std::lock_guard<std::mutex> g(mu);
  if (idx_ < int(pending.size())) (void)hipEventRecord(pending[idx_].b, stream_);
}

}  // namespace bse

using namespace bse;

extern "C" int32_t bse_prof_enable(const char *pfx) {
  std::lock_guard<std::mutex> g(mu);
  on = pfx && pfx[0];
  prefix = on ? pfx : "";
  return BSE_OK;
}

extern "C" int32_t bse_prof_collect(void) {
  std::lock_guard<std::mutex> g(mu);
  for (Pending &p : pending) {
    if (hipEventSynchronize(p.b) != hipSuccess)
      return fail(BSE_EDEVICE, "hipEventSynchronize failed in bse_prof_collect");
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      total_ms[p.name] += ms;
      launches[p.name] += 1;
    }
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
  return BSE_OK;
}

extern "C" int32_t bse_prof_count(void) {
  std::lock_guard<std::mutex> g(mu);
  return int32_t(names.size());
}

extern "C" int32_t bse_prof_get(int32_t i, char *h_name32, double *h_total_ms, int64_t *h_launches) {
  std::lock_guard<std::mutex> g(mu);
  if (i < 0 || i >= int(names.size())) return fail(BSE_EINVAL, "profile index out of range");
  if (h_name32) {
    std::memset(h_name32, 0, 32);
    std::strncpy(h_name32, names[i].c_str(), 31);
  }
  if (h_total_ms) *h_total_ms = total_ms[i];
  if (h_launches) *h_launches = launches[i];
  return BSE_OK;
}

extern "C" int32_t bse_prof_reset(void) {
  std::lock_guard<std::mutex> g(mu);
  for (size_t i = 0; i < total_ms.size(); ++i) {
    total_ms[i] = 0;
    launches[i] = 0;
  }
  return BSE_OK;
}
