// bse_haydock: the eps2 of one block without diagonalising it (Lanczos-Haydock,
// which the block-diagonal form of H serves as well as the eigensolver does,
// Sec. III.D.1).
//
// Lanczos on H_mu from v_0 = B_mu / |B_mu| gives a real tridiagonal matrix
// (a_j on the diagonal, b_j beside it); the resolvent element
// v_0^dag (z - H_mu)^-1 v_0 is the continued fraction
//     G(z) = 1 / (z - a_0 - b_1^2 / (z - a_1 - b_2^2 / (...)))
// and, since L_eta(x) = -Im 1 / (x + i eta), Eqs. (macro_diel) and
// (reducible_polar) become
//     eps2(w) = pref |B_mu|^2 (-Im G(w + i eta) - Im G(-w + i eta)).
//
// The recurrence (no reorthogonalisation, the classical form of the method):
//     w = H v_j - b_j v_{j-1},  a_j = Re v_j^dag w,  w -= a_j v_j,
//     b_{j+1} = |w|,  v_{j+1} = w / b_{j+1}.
// Each step is one kernel.  It keeps the residuals unnormalised, P_j = b_j v_j
// (P_0 = B_mu, b_0 = |B_mu|), and Y_j = H P_j; a workgroup owns a few rows.
// Step j first reduces the per-workgroup partial sums of step j-1,
//     b_{j-1}^2 = sum |P_{j-1}|^2,  a_{j-1} = P_{j-1}^dag Y_{j-1} / b_{j-1}^2
//                                          - P_{j-1}^dag P_{j-2} / b_{j-2},
// forms
//     P_j = (Y_{j-1} - a_{j-1} P_{j-1}) / b_{j-1} - (b_{j-1} / b_{j-2}) P_{j-2}
// column chunk by column chunk in LDS, multiplies its rows of H_mu by it
// (FP64 arithmetic on FP32 or FP64 H_mu) and writes its rows of P_j and Y_j
// and its partial sums of |P_j|^2, P_j^dag Y_j and P_j^dag P_{j-1}.  So the
// next vector never makes a round trip through a kernel of its own: one
// dependent launch per step, bound by reading H_mu once (HBM or, for blocks
// that fit, the last-level cache).
//   k_hd_step      one Lanczos step (grid: one workgroup per 4 RPW rows)
//   k_hd_finish    a_{K-1}, b_{K-1} and the last residual norm b_K
//   k_hd_spectrum  one thread per frequency: both continued fractions
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int HNT = 256;           // threads per workgroup (4 waves)
constexpr int HWV = HNT / 64;      // waves per workgroup
constexpr int HCH = 2048;          // columns of the step vector per LDS chunk (32 KB)
constexpr int64_t HD_NMAX = 1 << 20;
constexpr int32_t HD_KMAX = 1 << 20;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums three per-thread values over the workgroup (all threads get the sums).
__device__ __forceinline__ void block_sum3(double &s0, double &s1, double &s2,
                                           double (*red)[HWV]) {
  const int wv = threadIdx.x >> 6;
  s0 = wsum(s0);
  s1 = wsum(s1);
  s2 = wsum(s2);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = s0;
    red[1][wv] = s1;
    red[2][wv] = s2;
  }
  __syncthreads();
  s0 = s1 = s2 = 0.0;
  for (int i = 0; i < HWV; ++i) {
    s0 += red[0][i];
    s1 += red[1][i];
    s2 += red[2][i];
  }
}

// Coefficients of step j >= 1 from the partial sums of step j-1:
// P_j = cy Y_{j-1} + cp P_{j-1} + cq P_{j-2}; also a_{j-1} and b_{j-1}.
// A vanished residual (invariant Krylov space) gives zeros from there on.
struct Coef {
  double cy, cp, cq, alpha, bj1;
};

__device__ Coef hd_coef(int j, int G, const double *__restrict__ pin,
                        const double *__restrict__ b, double (*red)[HWV]) {
  double pp = 0, py = 0, pq = 0;
  for (int g = threadIdx.x; g < G; g += HNT) {
    pp += pin[g];
    py += pin[G + g];
    pq += pin[2 * G + g];
  }
  block_sum3(pp, py, pq, red);
  Coef c{0, 0, 0, 0, 0};
  const double bj2 = j >= 2 ? b[j - 2] : 0.0;
  c.bj1 = sqrt(pp);
  if (pp > 0.0) {
    c.alpha = py / pp - (bj2 > 0.0 ? pq / bj2 : 0.0);
    c.cy = 1.0 / c.bj1;
    c.cp = -c.alpha / c.bj1;
    c.cq = bj2 > 0.0 ? -c.bj1 / bj2 : 0.0;
  }
  return c;
}

__device__ __forceinline__ double2 hd_x(int j, int64_t i, const Coef &c,
                                        const double2 *__restrict__ Bv,
                                        const double2 *__restrict__ Ym1,
                                        const double2 *__restrict__ Pm1,
                                        const double2 *__restrict__ Pm2) {
  if (j == 0) return Bv[i];
  const double2 y = Ym1[i], p = Pm1[i];
  double2 r = make_double2(c.cy * y.x + c.cp * p.x, c.cy * y.y + c.cp * p.y);
  if (j >= 2) {
    const double2 q = Pm2[i];
    r.x += c.cq * q.x;
    r.y += c.cq * q.y;
  }
  return r;
}

template <typename TH>
__device__ __forceinline__ double2 ld_h(const TH *p) {
  const TH h = *p;
  return make_double2(double(h.x), double(h.y));
}

// ws: P[3][n] (ring by j mod 3), Y[2][n], partials[2][3][G] (ring by j mod 2)
// VEC (FP32 H_mu with an even ld and a 16-byte aligned base): each lane
// reads two adjacent columns in one 16-byte load.
template <typename TH, int RPW, bool VEC>
__global__ __launch_bounds__(HNT) void k_hd_step(int64_t n, const TH *__restrict__ H, int64_t ld,
                                                 const double2 *__restrict__ Bv, int j, int G,
                                                 double2 *__restrict__ P, double2 *__restrict__ Y,
                                                 double *__restrict__ part,
                                                 double *__restrict__ a, double *__restrict__ b) {
  static_assert(!VEC || std::is_same<TH, float2>::value, "16-byte pairs of FP32 entries only");
  __shared__ double2 xs[HCH];
  __shared__ double red[3][HWV];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double2 *Pm1 = P + int64_t((j + 2) % 3) * n;
  const double2 *Pm2 = P + int64_t((j + 1) % 3) * n;
  double2 *Pj = P + int64_t(j % 3) * n;
  const double2 *Ym1 = Y + int64_t((j + 1) & 1) * n;
  double2 *Yj = Y + int64_t(j & 1) * n;
  const double *pin = part + int64_t((j + 1) & 1) * 3 * G;
  double *pout = part + int64_t(j & 1) * 3 * G;

  Coef c{0, 0, 0, 0, 0};
  if (j > 0) {
    c = hd_coef(j, G, pin, b, red);
    if (blockIdx.x == 0 && tid == 0) {
      a[j - 1] = c.alpha;
      b[j - 1] = c.bj1;
    }
  }
  const int64_t r0 = (int64_t(blockIdx.x) * HWV + wv) * RPW;
  const TH *hrow[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) hrow[r] = H + (r0 + r < n ? r0 + r : n - 1) * ld;
  double2 acc[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) acc[r] = make_double2(0.0, 0.0);

  for (int64_t c0 = 0; c0 < n; c0 += HCH) {
    const int cn = int(n - c0 < HCH ? n - c0 : HCH);
    __syncthreads();
    for (int t = tid; t < cn; t += HNT) xs[t] = hd_x(j, c0 + t, c, Bv, Ym1, Pm1, Pm2);
    __syncthreads();
    constexpr int U = RPW >= 8 ? 2 : 16 / RPW;  // 16 row loads in flight per lane
    if constexpr (VEC) {
      constexpr int U2 = U / 2;
      int cc = 2 * lane;
      for (; cc + 1 + (U2 - 1) * 128 < cn; cc += U2 * 128) {
        float4 h[RPW][U2];
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
          for (int u = 0; u < U2; ++u)
            h[r][u] = *reinterpret_cast<const float4 *>(hrow[r] + c0 + cc + u * 128);
#pragma unroll
        for (int u = 0; u < U2; ++u) {
          const double2 x0 = xs[cc + u * 128], x1 = xs[cc + 1 + u * 128];
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            const double hr0 = h[r][u].x, hi0 = h[r][u].y, hr1 = h[r][u].z, hi1 = h[r][u].w;
            acc[r].x += hr0 * x0.x - hi0 * x0.y;
            acc[r].y += hr0 * x0.y + hi0 * x0.x;
            acc[r].x += hr1 * x1.x - hi1 * x1.y;
            acc[r].y += hr1 * x1.y + hi1 * x1.x;
          }
        }
      }
      for (; cc < cn; cc += 128) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (cc + e < cn) {
            const double2 x = xs[cc + e];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
              const double2 h = ld_h(hrow[r] + c0 + cc + e);
              acc[r].x += h.x * x.x - h.y * x.y;
              acc[r].y += h.x * x.y + h.y * x.x;
            }
          }
        }
      }
      continue;
    }
    int cc = lane;
    for (; cc + (U - 1) * 64 < cn; cc += U * 64) {
      double2 h[RPW][U];
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) h[r][u] = ld_h(hrow[r] + c0 + cc + u * 64);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 x = xs[cc + u * 64];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          acc[r].x += h[r][u].x * x.x - h[r][u].y * x.y;
          acc[r].y += h[r][u].x * x.y + h[r][u].y * x.x;
        }
      }
    }
    for (; cc < cn; cc += 64) {
      const double2 x = xs[cc];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const double2 h = ld_h(hrow[r] + c0 + cc);
        acc[r].x += h.x * x.x - h.y * x.y;
        acc[r].y += h.x * x.y + h.y * x.x;
      }
    }
  }
  // the stores follow the reduction (a pending store whose registers the
  // reduction reuses would have to complete first)
  double pp = 0, py = 0, pq = 0;
  double2 xo[RPW], yo[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const double yx = wsum(acc[r].x), yy = wsum(acc[r].y);
    const int64_t i = r0 + r;
    xo[r] = yo[r] = make_double2(0.0, 0.0);
    if (lane == 0 && i < n) {
      const double2 x = hd_x(j, i, c, Bv, Ym1, Pm1, Pm2);
      xo[r] = x;
      yo[r] = make_double2(yx, yy);
      pp += x.x * x.x + x.y * x.y;
      py += x.x * yx + x.y * yy;
      if (j > 0) {
        const double2 q = Pm1[i];
        pq += x.x * q.x + x.y * q.y;
      }
    }
  }
  block_sum3(pp, py, pq, red);
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int64_t i = r0 + r;
      if (i < n) {
        Pj[i] = xo[r];
        Yj[i] = yo[r];
      }
    }
  }
  if (tid == 0) {
    pout[blockIdx.x] = pp;
    pout[G + blockIdx.x] = py;
    pout[2 * G + blockIdx.x] = pq;
  }
}

// One workgroup: a_{K-1}, b_{K-1} from the last step's partials, then the norm
// of the last residual P_K into b_K.
__global__ __launch_bounds__(HNT) void k_hd_finish(int64_t n, int K, int G,
                                                   const double2 *__restrict__ P,
                                                   const double2 *__restrict__ Y,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ a,
                                                   double *__restrict__ b) {
  __shared__ double red[3][HWV];
  const int j = K;
  const Coef c = hd_coef(j, G, part + int64_t((j + 1) & 1) * 3 * G, b, red);
  const double2 *Pm1 = P + int64_t((j + 2) % 3) * n;
  const double2 *Pm2 = P + int64_t((j + 1) % 3) * n;
  const double2 *Ym1 = Y + int64_t((j + 1) & 1) * n;
  double s = 0, d1 = 0, d2 = 0;
  for (int64_t i = threadIdx.x; i < n; i += HNT) {
    const double2 x = hd_x(j, i, c, nullptr, Ym1, Pm1, Pm2);
    s += x.x * x.x + x.y * x.y;
  }
  block_sum3(s, d1, d2, red);
  if (threadIdx.x == 0) {
    a[K - 1] = c.alpha;
    b[K - 1] = c.bj1;
    b[K] = sqrt(s);
  }
}

// eps2(w) = pref b_0^2 (-Im G(w + i eta) - Im G(-w + i eta)), the fraction
// evaluated from level K-1 up (the remainder below level K is dropped).
__global__ __launch_bounds__(256) void k_hd_spectrum(int K, const double *__restrict__ a,
                                                     const double *__restrict__ b, double pref,
                                                     double eta, int64_t nw,
                                                     const double *__restrict__ w,
                                                     double *__restrict__ eps2) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nw) return;
  const double om = w[t];
  double g1x = 0, g1y = 0, g2x = 0, g2y = 0;  // G at w + i eta and -w + i eta
  for (int jj = K - 1; jj >= 0; --jj) {
    const double aj = a[jj];
    const double bb = jj + 1 < K ? b[jj + 1] * b[jj + 1] : 0.0;
    // g <- 1 / (z - a_j - bb g)
    double dx = om - aj - bb * g1x, dy = eta - bb * g1y;
    double inv = 1.0 / (dx * dx + dy * dy);
    g1x = dx * inv;
    g1y = -dy * inv;
    dx = -om - aj - bb * g2x;
    dy = eta - bb * g2y;
    inv = 1.0 / (dx * dx + dy * dy);
    g2x = dx * inv;
    g2y = -dy * inv;
  }
  eps2[t] = pref * b[0] * b[0] * (-g1y - g2y);
}

int hd_rpw(int64_t n) { return n <= 8192 ? 2 : n <= 16384 ? 4 : 8; }
int hd_groups(int64_t n) {
  const int64_t rows = int64_t(HWV) * hd_rpw(n);
  return int((n + rows - 1) / rows);
}

template <typename TH, int RPW>
void launch_steps(int64_t n, const TH *H, int64_t ld, const double2 *Bv, int K, int G,
                  double2 *P, double2 *Y, double *part, double *a, double *b, hipStream_t s) {
  if constexpr (std::is_same<TH, float2>::value) {
    if (ld % 2 == 0 && reinterpret_cast<uintptr_t>(H) % 16 == 0) {
      for (int j = 0; j < K; ++j)
        BSE_LAUNCH("k_hd_step", (k_hd_step<TH, RPW, true>), dim3(G), dim3(HNT), 0, s, n, H, ld,
                   Bv, j, G, P, Y, part, a, b);
      return;
    }
  }
  for (int j = 0; j < K; ++j)
    BSE_LAUNCH("k_hd_step", (k_hd_step<TH, RPW, false>), dim3(G), dim3(HNT), 0, s, n, H, ld, Bv, j,
               G, P, Y, part, a, b);
}

template <typename TH>
void run_steps(int64_t n, const TH *H, int64_t ld, const double2 *Bv, int K, int G, double2 *P,
               double2 *Y, double *part, double *a, double *b, hipStream_t s) {
  switch (hd_rpw(n)) {
    case 2: launch_steps<TH, 2>(n, H, ld, Bv, K, G, P, Y, part, a, b, s); break;
    case 4: launch_steps<TH, 4>(n, H, ld, Bv, K, G, P, Y, part, a, b, s); break;
    default: launch_steps<TH, 8>(n, H, ld, Bv, K, G, P, Y, part, a, b, s); break;
  }
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" size_t bse_haydock_ws(int64_t n) {
  if (n < 1 || n > HD_NMAX) return 0;
  return size_t(5 * n) * 16 + size_t(6) * hd_groups(n) * 8;
}

extern "C" int32_t bse_haydock(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64,
                               const void *Bmu, int32_t K, double *a, double *b, void *ws,
                               size_t ws_bytes, bse_stream stream) {
  if (n < 1 || n > HD_NMAX) return fail(BSE_ESHAPE, "n = %lld outside 1 .. %lld", (long long)n,
                                        (long long)HD_NMAX);
  if (ld < n) return fail(BSE_ESHAPE, "ld < n");
  if (K < 1 || K > HD_KMAX) return fail(BSE_EINVAL, "K = %d outside 1 .. %d", K, HD_KMAX);
  if (!Hmu || !Bmu || !a || !b || !ws) return fail(BSE_EINVAL, "NULL pointer");
  if (ws_bytes < bse_haydock_ws(n)) return fail(BSE_EWORKSPACE, "workspace too small");
  const int G = hd_groups(n);
  double2 *P = (double2 *)ws, *Y = P + 3 * n;
  double *part = (double *)(Y + 2 * n);
  hipStream_t s = (hipStream_t)stream;
  const double2 *Bv = (const double2 *)Bmu;
  if (h_fp64)
    run_steps(n, (const double2 *)Hmu, ld, Bv, K, G, P, Y, part, a, b, s);
  else
    run_steps(n, (const float2 *)Hmu, ld, Bv, K, G, P, Y, part, a, b, s);
  BSE_LAUNCH("k_hd_finish", k_hd_finish, dim3(1), dim3(HNT), 0, s, n, K, G, P, Y, part, a, b);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}

extern "C" int32_t bse_haydock_spectrum(int32_t K, const double *a, const double *b, double pref,
                                        double eta, int64_t nw, const double *w, double *eps2,
                                        bse_stream stream) {
  if (K < 1 || K > HD_KMAX) return fail(BSE_EINVAL, "K = %d outside 1 .. %d", K, HD_KMAX);
  if (nw < 0) return fail(BSE_ESHAPE, "negative size");
  if (nw == 0) return BSE_OK;
  if (!a || !b || !w || !eps2) return fail(BSE_EINVAL, "NULL pointer");
  if (!(eta > 0)) return fail(BSE_EINVAL, "eta must be > 0");
  BSE_LAUNCH("k_hd_spectrum", k_hd_spectrum, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0,
             (hipStream_t)stream, K, a, b, pref, eta, nw, w, eps2);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}
