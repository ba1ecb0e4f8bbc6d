// bse_spectrum: absorption spectrum from the optical poles.
//
//   eps2(w) = pref sum_l osc_l [ L(w - pole_l) + L(w + pole_l) ],
//   L(x) = eta / (x^2 + eta^2),
// the imaginary part of Eq. (macro_diel) with the spectral form Eq.
// (reducible_polar) (resonant and antiresonant poles, Lorentzian broadening
// eta); pref = 8 pi / N_k carries the spin factor 2 and V_uc = 1.
// One thread per frequency; the poles stream through LDS in chunks.
#include <hip/hip_runtime.h>

#include "bse_internal.h"

namespace bse {
namespace {
constexpr int SNT = 256;

__global__ __launch_bounds__(SNT) void k_spectrum(int64_t n, const double *__restrict__ pole,
                                                  const double *__restrict__ osc, double pref,
                                                  double eta, int64_t nw,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ eps2) {
  __shared__ double sp[SNT], so[SNT];
  const int64_t j = int64_t(blockIdx.x) * SNT + threadIdx.x;
  const double x = j < nw ? w[j] : 0.0;
  const double e2 = eta * eta;
  double acc = 0.0;
  for (int64_t l0 = 0; l0 < n; l0 += SNT) {
    __syncthreads();
    const int64_t l = l0 + threadIdx.x;
    sp[threadIdx.x] = l < n ? pole[l] : 0.0;
    so[threadIdx.x] = l < n ? osc[l] : 0.0;
    __syncthreads();
    const int m = int(n - l0 < SNT ? n - l0 : SNT);
    for (int i = 0; i < m; ++i) {
      const double a = x - sp[i], b = x + sp[i];
      acc += so[i] * (eta / (a * a + e2) + eta / (b * b + e2));
    }
  }
  if (j < nw) eps2[j] = pref * acc;
}
}  // namespace
}  // namespace bse

using namespace bse;

extern "C" int32_t bse_spectrum(int64_t n, const double *pole, const double *osc, double pref,
                                double eta, int64_t nw, const double *w, double *eps2,
                                bse_stream stream) {
  if (n < 0 || nw < 0) return fail(BSE_ESHAPE, "negative size");
  if (nw == 0) return BSE_OK;
  if ((n > 0 && (!pole || !osc)) || !w || !eps2) return fail(BSE_EINVAL, "NULL pointer");
  if (!(eta > 0)) return fail(BSE_EINVAL, "eta must be > 0");
  BSE_LAUNCH("k_spectrum", k_spectrum, dim3((unsigned)((nw + SNT - 1) / SNT)), dim3(SNT), 0,
                     (hipStream_t)stream, n, pole, osc, pref, eta, nw, w, eps2);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}
