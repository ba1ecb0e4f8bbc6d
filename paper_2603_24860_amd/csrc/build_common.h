// Helpers shared by the H build kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace bse {

// Linear index of k - q on the n1 x n2 x n3 grid (both given as linear indices).
__device__ __forceinline__ int kminus(int k, int q, int n1, int n2, int n3) {
  const int k3 = k % n3, k2 = (k / n3) % n2, k1 = k / (n2 * n3);
  const int q3 = q % n3, q2 = (q / n3) % n2, q1 = q / (n2 * n3);
  int a = k1 - q1, b = k2 - q2, c = k3 - q3;
  a += a < 0 ? n1 : 0;
  b += b < 0 ? n2 : 0;
  c += c < 0 ? n3 : 0;
  return (a * n2 + b) * n3 + c;
}

// The direct-term shapes the fused kernels take: Nmb = 64 MI (MI <= 6),
// nv^2 <= 16 and nc^2 <= 48.
__host__ __forceinline__ bool fused_shape(int nmb, int nv, int nc) {
  return nmb % 64 == 0 && nmb <= 384 && nv * nv <= 16 && nc * nc <= 48;
}

}  // namespace bse
