// bse_eels: longitudinal excitons from the optical poles (Sec. III.D.2).
//
// Adding the G = 0 Coulomb term c B B^dag to the block (c = 4 pi / (N_k V_uc)
// times the spin factor of the exchange; the caller passes c) leaves every dark
// direction unchanged and moves each weighted pole p_i (strength w_i > 0, one
// pole per degenerate cluster) to a root of the secular equation Eq. (secular)
//     f(x) = 1 - c sum_i w_i / (x - p_i) = 0.
// f increases on every interval between consecutive weighted poles from -inf
// to +inf, so each interval (p_i, p_{i+1}) holds exactly one root, and one more
// lies in (p_m, p_m + c sum w).  The eigenvector components of Eq.
// (eigenvec_xi), A'_i ~ B_i / (p_i - x), give the strengths of the new poles
//     w'(x) = (B^T A')^2 / |A'|^2 = 1 / (c^2 sum_i w_i / (x - p_i)^2).
//   k_eels_compact  one workgroup: the weighted poles (w > rel * sum w) in order
//   k_eels_roots    one wave per root: a safeguarded rational iteration on its
//                   interval (x = p_lo + t, so no cancellation near the lower
//                   pole; the lanes split the sum over poles), then the
//                   strength; entries past the last root get zero strength.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int CNT = 1024;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ws: p[n], w[n], [0] m (as double), [1] sum w
__global__ __launch_bounds__(CNT) void k_eels_compact(int64_t n, const double *__restrict__ pole,
                                                      const double *__restrict__ osc, double rel,
                                                      double *__restrict__ p,
                                                      double *__restrict__ w,
                                                      double *__restrict__ meta) {
  __shared__ double sh[CNT / 64];
  __shared__ int scan[CNT];
  const int tid = threadIdx.x;
  double s = 0;
  for (int64_t i = tid; i < n; i += CNT) s += osc[i];
  s = wsum(s);
  if ((tid & 63) == 0) sh[tid >> 6] = s;
  __syncthreads();
  double tot = 0;
  for (int i = 0; i < CNT / 64; ++i) tot += sh[i];
  const double thr = rel * tot;
  int64_t base = 0;
  double wtot = 0;
  for (int64_t i0 = 0; i0 < n; i0 += CNT) {
    const int64_t i = i0 + tid;
    const int flag = (i < n && osc[i] > thr) ? 1 : 0;
    scan[tid] = flag;
    __syncthreads();
    for (int o = 1; o < CNT; o <<= 1) {  // inclusive scan (Hillis-Steele)
      const int v = tid >= o ? scan[tid - o] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    if (flag) {
      const int64_t j = base + scan[tid] - 1;
      p[j] = pole[i];
      w[j] = osc[i];
    }
    base += scan[CNT - 1];
    __syncthreads();
  }
  __syncthreads();
  // sum of the kept strengths
  double ws_ = 0;
  for (int64_t j = tid; j < base; j += CNT) ws_ += w[j];
  ws_ = wsum(ws_);
  if ((tid & 63) == 0) sh[tid >> 6] = ws_;
  __syncthreads();
  for (int i = 0; i < CNT / 64; ++i) wtot += sh[i];
  if (tid == 0) {
    meta[0] = double(base);
    meta[1] = wtot;
  }
}

__global__ __launch_bounds__(256) void k_eels_roots(int64_t n, const double *__restrict__ p,
                                                    const double *__restrict__ w,
                                                    const double *__restrict__ meta, double c,
                                                    double *__restrict__ xpole,
                                                    double *__restrict__ xosc) {
  const int lane = threadIdx.x & 63;
  const int64_t xi = int64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (xi >= n) return;
  const int64_t m = int64_t(meta[0]);
  if (xi >= m) {
    if (lane == 0) {
      xpole[xi] = 0.0;
      xosc[xi] = 0.0;
    }
    return;
  }
  const double lo = p[xi];
  const bool top = xi + 1 >= m;
  const double width = top ? c * meta[1] : p[xi + 1] - lo;
  const double hi = top ? 0.0 : p[xi + 1];
  // Safeguarded rational iteration on t = x - lo in (0, width).  At the
  // current t the sum splits into psi (poles at or below lo) and phi (poles
  // above), each replaced by one pole term plus a constant that match its
  // value and slope there:
  //   psi ~ A / t + r1,  phi ~ S / (t - width) + r2,
  // with r1 = sum w (lo - p) / d^2 and r2 = sum w (hi - p) / d^2 formed
  // directly (d = lo - p + t).  The model's root in (0, width) is the
  // positive root of  al t^2 - (al width + cA + cS) t + cA width = 0,
  // al = 1 - c (r1 + r2), taken in the cancellation-free form 2C / (B + sqrt D).
  // A step outside the bracket kept from the signs of f falls back to
  // bisection; the iteration stops when the model no longer moves t.
  double a = 0.0, b = width, t = 0.5 * width;
  double s2 = 0, te = t;
  for (int it = 0; it < 64; ++it) {
    te = t;
    double ps = 0, pd = 0, r1 = 0, fs = 0, fd = 0, r2 = 0;
    for (int64_t j = lane; j < m; j += 64) {
      const double pj = p[j], wj = w[j];
      const double d = (lo - pj) + t;
      const double q = wj / d, q2 = q / d;
      if (j <= xi) {
        ps += q;
        pd += q2;
        r1 += q2 * (lo - pj);
      } else {
        fs += q;
        fd += q2;
        r2 += q2 * (hi - pj);
      }
    }
    ps = wsum(ps);
    pd = wsum(pd);
    r1 = wsum(r1);
    fs = wsum(fs);
    fd = wsum(fd);
    r2 = wsum(r2);
    s2 = pd + fd;
    const double f = 1.0 - c * (ps + fs);
    if (f < 0.0)
      a = t;
    else
      b = t;
    if (f == 0.0 || b - a <= 4.4e-16 * fabs(lo + b)) break;
    const double A = pd * t * t;
    double tn = -1.0;
    if (top) {
      const double al = 1.0 - c * r1;
      if (al > 0.0) tn = c * A / al;
    } else {
      const double dw = t - width;
      const double S = fd * dw * dw;
      const double al = 1.0 - c * (r1 + r2);
      const double Bq = al * width + c * (A + S);
      const double Cq = c * A * width;
      const double D = Bq * Bq - 4.0 * al * Cq;
      if (D >= 0.0) {
        const double den = Bq + sqrt(D);
        if (den > 0.0) tn = 2.0 * Cq / den;
      }
    }
    if (tn > 0.0 && fabs(tn - t) <= 8.9e-16 * fabs(lo + t)) break;
    // the top bracket end c sum w is itself the root when one pole has weight
    t = (tn > a && (tn < b || (top && tn == b))) ? tn : 0.5 * (a + b);
  }
  // te: the last point evaluated; s2 = sum w / d^2 there
  if (lane == 0) {
    xpole[xi] = lo + te;
    xosc[xi] = 1.0 / (c * c * s2);
  }
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" size_t bse_eels_ws(int64_t n) { return n < 1 ? 0 : size_t(2 * n + 2) * 8; }

extern "C" int32_t bse_eels(int64_t n, const double *pole, const double *osc, double c,
                            double *xpole, double *xosc, void *ws, size_t ws_bytes,
                            bse_stream stream) {
  if (n < 1) return fail(BSE_ESHAPE, "n must be >= 1");
  if (!pole || !osc || !xpole || !xosc) return fail(BSE_EINVAL, "NULL pointer");
  if (!(c > 0)) return fail(BSE_EINVAL, "coupling c must be > 0");
  if (!ws || ws_bytes < bse_eels_ws(n)) return fail(BSE_EWORKSPACE, "workspace too small");
  double *p = (double *)ws, *w = p + n, *meta = w + n;
  hipStream_t s = (hipStream_t)stream;
  BSE_LAUNCH("k_eels_compact", k_eels_compact, dim3(1), dim3(CNT), 0, s, n, pole, osc, 1e-14, p,
             w, meta);
  BSE_LAUNCH("k_eels_roots", k_eels_roots, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, p,
             w, meta, c, xpole, xosc);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}
