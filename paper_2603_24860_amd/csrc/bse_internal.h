// Internal declarations shared by the library's translation units.
#pragma once
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bse.h"

namespace bse {

// Records a thread-local message for bse_last_error() and returns `st`.
int32_t fail(int32_t st, const char *fmt, ...);

// Point group data built on the host.
struct Group {
  int nops = 0;
  std::vector<int32_t> kmat;    // [nops][9] action on reduced k
  std::vector<double> rcart;    // [nops][9] Cartesian matrix
  struct Irrep {
    std::string name;
    int dim;
    std::vector<double> chi;    // [nops]
  };
  std::vector<Irrep> irreps;
};

// Returns nullptr for an unknown group id.
const Group *get_group(int32_t group);

// Grid helpers (k linear index = (k1 n2 + k2) n3 + k3).
struct Grid {
  int n1, n2, n3;
  int64_t nk() const { return int64_t(n1) * n2 * n3; }
};

// RAII bracket of one kernel launch for the opt-in event profiler.
class ProfScope {
 public:
  ProfScope(const char *name, hipStream_t s);
  ~ProfScope();

 private:
  hipStream_t stream_;
  int idx_;
};

// Launch `kernel` (a __global__ symbol or template instance in parentheses)
// under the profiler name `name`.
#define BSE_LAUNCH(name, kernel, grid, block, lds, stream, ...)               \
  do {                                                                      \
    bse::ProfScope prof_scope_(name, stream);                               \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);      \
  } while (0)

// Split-BF16 form of bse_build (arguments already validated).
int32_t build_bf16x3(const bse_problem *p, void *H, int64_t ldh, void *ws, size_t ws_bytes,
                     bse_stream stream);

// The seed pieces of a plan (bse_seed_plan; filled by bse_build_seed): the
// exchange between k-orbit representatives xs [nkorb nb][ldx], the direct
// blocks of the pair-orbit representatives drep [nporb][nc^2][nv^2], the
// k -> k-orbit and (k, k') -> pair-orbit maps; elements of the plan's
// precision.  For projecting blocks straight from the pieces.
struct SeedPieces {
  bse_problem p;
  int32_t prec;
  int nk;
  const int32_t *porb;
  const void *xs, *drep;
  int64_t ldx;
};
int32_t seed_pieces(int64_t plan, SeedPieces *out);

}  // namespace bse

#define BSE_HIP_CHECK(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return bse::fail(BSE_EDEVICE, "%s failed: %s (%s:%d)", #expr,                \
                       hipGetErrorString(e_), __FILE__, __LINE__);                 \
  } while (0)
