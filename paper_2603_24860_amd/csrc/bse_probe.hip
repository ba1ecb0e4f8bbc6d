// bse_sync_probe: the cost of one global dependency between two steps of the
// batched eigensolver, measured two ways on the caller's stream.
//
// The batched form advances every block by one Householder step per launch,
// so its critical path is one dependent launch per step.  The alternative is
// one persistent (cooperative) launch whose workgroups meet at a grid-wide
// barrier between steps.  Both carry the same work per step here (every
// workgroup reads one value that another workgroup wrote in the previous
// step, so the dependency is real), and the probe times `steps` of them:
//   mode 0  `steps` launches of a grid of `wgs` workgroups, back to back in
//           stream order (each launch depends on the previous one);
//   mode 1  one cooperative launch of `wgs` workgroups that runs `steps`
//           steps separated by grid barriers (cooperative groups).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int QNT = 256;

// step s: workgroup w reads the value workgroup (w + 1) % wgs wrote in step
// s - 1 and writes its own
__device__ __forceinline__ void probe_step(int *buf, int wgs, int s) {
  const int w = blockIdx.x;
  if (threadIdx.x == 0) {
    const int src = (w + 1) % wgs;
    const int v = __hip_atomic_load(buf + (s & 1) * wgs + src, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(buf + ((s + 1) & 1) * wgs + w, v + 1, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(QNT) void k_probe_step(int *buf, int wgs, int s) {
  probe_step(buf, wgs, s);
}

__global__ __launch_bounds__(QNT) void k_probe_persistent(int *buf, int wgs, int steps) {
  cooperative_groups::grid_group g = cooperative_groups::this_grid();
  for (int s = 0; s < steps; ++s) {
    probe_step(buf, wgs, s);
    g.sync();
  }
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" int32_t bse_sync_probe(int32_t mode, int32_t wgs, int32_t steps, int32_t *buf,
                                  double *h_us_per_step, bse_stream stream) {
  if (mode < 0 || mode > 1) return fail(BSE_EINVAL, "mode %d (0 or 1)", mode);
  if (wgs < 1 || wgs > 4096 || steps < 1 || steps > 1000000)
    return fail(BSE_ESHAPE, "wgs 1 .. 4096, steps 1 .. 10^6");
  if (!buf || !h_us_per_step) return fail(BSE_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  if (mode == 1) {  // the cooperative grid must fit on the device at once
    int dev = 0, coop = 0, ncu = 0, per_cu = 0;
    BSE_HIP_CHECK(hipGetDevice(&dev));
    BSE_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    BSE_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BSE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_persistent, QNT, 0));
    if (!coop) return fail(BSE_EUNSUPPORTED, "no cooperative launch on this device");
    if (int64_t(per_cu) * ncu < wgs)
      return fail(BSE_ESHAPE, "%d workgroups do not fit at once (%d x %d)", wgs, ncu, per_cu);
  }
  hipEvent_t e0, e1;
  BSE_HIP_CHECK(hipEventCreate(&e0));
  BSE_HIP_CHECK(hipEventCreate(&e1));
  BSE_HIP_CHECK(hipMemsetAsync(buf, 0, size_t(2) * wgs * sizeof(int32_t), s));
  BSE_HIP_CHECK(hipEventRecord(e0, s));
  if (mode == 0) {
    for (int st = 0; st < steps; ++st)
      hipLaunchKernelGGL(k_probe_step, dim3(wgs), dim3(QNT), 0, s, buf, wgs, st);
  } else {
    void *args[] = {&buf, &wgs, &steps};
    BSE_HIP_CHECK(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_probe_persistent),
                                             dim3(wgs), dim3(QNT), args, 0, s));
  }
  BSE_HIP_CHECK(hipGetLastError());
  BSE_HIP_CHECK(hipEventRecord(e1, s));
  BSE_HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  BSE_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *h_us_per_step = 1e3 * double(ms) / steps;
  return BSE_OK;
}
