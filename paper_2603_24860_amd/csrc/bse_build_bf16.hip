// Split-BF16 form of the H build (placeholder until the BF16 MFMA kernels land).
#include <hip/hip_runtime.h>

#include "bse_internal.h"

namespace bse {
int32_t build_bf16x3(const bse_problem *, void *, int64_t, void *, size_t, bse_stream) {
  return fail(BSE_EUNSUPPORTED, "split-BF16 build is not implemented yet");
}
}  // namespace bse
