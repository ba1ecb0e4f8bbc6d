// bse_block_eigh: eigenvalues and oscillator strengths of one Hermitian block.
//
// Paper: the block H_mu = U_mu^dag H U_mu is diagonalised on its own
// (Sec. III.D.1); its eigenvalues are the exciton energies Omega_l and the
// oscillator strengths are |B_l|^2 = |A_l^dag B_mu|^2 (Eq. (oscillatorA)).
//
// Method (our design for one GPU):
//  1. A Householder reflection Q0 with Q0^dag B = beta0 e_1 is applied to both
//     sides of a working copy A of H_mu.
//  2. Blocked Householder tridiagonalisation in LAPACK's lower form: column j
//     is annihilated below the subdiagonal by a reflector acting on rows
//     j+1..n-1, so Q e_1 = e_1 stays true.  Within a panel of NBK columns the
//     trailing matrix is updated lazily, A - V W^dag - W V^dag (V, W column
//     major); after the panel the rank-2 NBK update runs on MFMA.
//     Each column costs two kernels, one per global dependency:
//       k_colA: reflector of column j from the reduced partial sums, then
//               y = A22 v (rows split over workgroups, bound by HBM bandwidth)
//               and the partial sums of y^dag v;
//       k_colB: w^dag v follows from y^dag v and the panel dot products
//               (w^dag v = conj(tau) (y^dag v - 2 Re(p^dag q)) with p = V^dag v,
//               q = W^dag v), so the final column of W, the fully updated
//               column j+1 and the partial sums of its norm and of its dot
//               products with V and W come out of one pass.
//     All scalar work is FP64; A is stored in FP64 or (prec FP32) FP32.
//  3. T is real symmetric tridiagonal (the reflectors make the subdiagonal
//     real).  All eigenvalues by 64-way multisection on Sturm counts (one wave
//     per eigenvalue, FP64).  Because Q0 Q maps e_1 to e_1,
//     |B_l|^2 = beta0^2 z_l(0)^2 with z_l the eigenvectors of T, and for a
//     cluster of (numerically) degenerate eigenvalues the summed weight is the
//     residue of G(z) = [(z - T)^-1]_00 = 1 / (z - d_0 - e_0^2 / (z - d_1 - ...))
//     at the cluster, computed by the trapezoidal rule on a circle around the
//     cluster (one wave per cluster, one node per lane); the radius is the
//     geometric mean of the cluster width and the distance to the next
//     eigenvalue, so the error decays like (width / distance)^(M/2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <type_traits>
#include <mutex>
#include <vector>

#include "bse_internal.h"
#include "eigh_geometry.h"
#include "mfma_tile.h"

namespace bse {
namespace {


__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double2 cconj(double2 a) { return double2{a.x, -a.y}; }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return double2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return double2{s * a.x, s * a.y}; }

template <typename T> struct C2T;
template <> struct C2T<float> { typedef float2 t; };
template <> struct C2T<double> { typedef double2 t; };
template <typename C> __device__ __forceinline__ double2 to_d2(C x) {
  return double2{double(x.x), double(x.y)};
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of one double (NTH threads); result valid in all threads.
template <int NTH> __device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < NTH / 64; ++i) s += sh[i];
  return s;
}

// Two sums over the workgroup with one pair of barriers; sh holds 2 NTH / 64.
template <int NTH>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    sh[w] = a;
    sh[NTH / 64 + w] = b;
  }
  __syncthreads();
  double sa = 0, sb = 0;
  for (int i = 0; i < NTH / 64; ++i) {
    sa += sh[i];
    sb += sh[NTH / 64 + i];
  }
  a = sa;
  b = sb;
}

// The same sums for a buffer that the kernel uses only once: one barrier,
// after the partial sums are written (it also publishes earlier LDS stores).
template <int NTH> __device__ __forceinline__ double block_sum_once(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < NTH / 64; ++i) s += sh[i];
  return s;
}
template <int NTH>
__device__ __forceinline__ void block_sum2_once(double &a, double &b, double *sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = a;
    sh[NTH / 64 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  double sa = 0, sb = 0;
  for (int i = 0; i < NTH / 64; ++i) {
    sa += sh[i];
    sb += sh[NTH / 64 + i];
  }
  a = sa;
  b = sb;
}



// Reflector scalars with LAPACK zlarfg semantics:
// (I - tau v v^dag)^dag (alpha, x) = (beta, 0), v = (1, x / (alpha - beta)),
// given alpha and |x|^2.
__device__ __forceinline__ void householder(double2 al, double xn2, double &beta, double2 &tau,
                                            double2 &scale) {
  tau = double2{0, 0};
  scale = double2{0, 0};
  if (xn2 == 0.0 && al.y == 0.0) {
    beta = al.x;
    return;
  }
  const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
  beta = al.x >= 0 ? -nrm : nrm;
  tau = double2{(beta - al.x) / beta, -al.y / beta};
  const double2 den = {al.x - beta, al.y};
  const double dd = den.x * den.x + den.y * den.y;
  scale = double2{den.x / dd, -den.y / dd};
}

// ---------------------------------------------------------------------------
template <typename TH, typename TA>
__device__ __forceinline__ void b_copy_in(int64_t n, const TH *__restrict__ H, int64_t ldh, TA *__restrict__ A,
                          int64_t lda, int64_t r, int64_t xw, int64_t gx) {
  typedef typename C2T<TH>::t CH;
  typedef typename C2T<TA>::t CA;
    for (int64_t c = xw * blockDim.x + threadIdx.x; c < n;
       c += gx * blockDim.x) {
    const CH x = reinterpret_cast<const CH *>(H)[r * ldh + c];
    reinterpret_cast<CA *>(A)[r * lda + c] = CA{TA(x.x), TA(x.y)};
  }
}

// ---------------------------------------------------------------------------
// initial reflection B -> beta0 e_1 (whole matrix, once per solve)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void b_load_b(int64_t n, const double2 *__restrict__ B, double2 *__restrict__ col,
                         double *__restrict__ part3, int wg, int nwgs) {
  __shared__ double sh[ENT / 64];
  double s = 0;
  for (int64_t r = int64_t(wg) * ENT + threadIdx.x; r < n; r += int64_t(nwgs) * ENT) {
    const double2 b = B[r];
    col[r] = b;
    if (r >= 1) s += b.x * b.x + b.y * b.y;
  }
  s = block_sum<ENT>(s, sh);
  if (threadIdx.x == 0) part3[wg] = s;
}

// v from the loaded B (scalars from the norm partials), then y = A v.
template <typename TA>
__device__ __forceinline__ void b_hemv0(int64_t n, int rpw, const TA *__restrict__ A,
                                               int64_t lda, const double2 *__restrict__ col,
                                               const double *__restrict__ part3, int np3,
                                               double *__restrict__ beta0,
                                               double2 *__restrict__ tau,
                                               double2 *__restrict__ vbuf,
                                               double2 *__restrict__ y, int wg) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double s = 0;
  for (int p = threadIdx.x; p < np3; p += ENT) s += part3[p];
  const double xn2 = block_sum<ENT>(s, sh);
  double beta;
  double2 t, sc;
  householder(col[0], xn2, beta, t, sc);
  if (wg == 0 && threadIdx.x == 0) {
    beta0[0] = beta;
    tau[0] = t;
  }
  const int64_t rbase = (int64_t(wg) * (ENT / 64) + wv) * rpw;
  for (int rr = 0; rr < rpw; ++rr) {
    const int64_t r = rbase + rr;
    if (r >= n) break;
    const CA *arow = reinterpret_cast<const CA *>(A) + r * lda;
    double sr = 0, si = 0;
    for (int64_t c = lane; c < n; c += 64) {
      const double2 a = to_d2(arow[c]);
      const double2 v = c == 0 ? double2{1, 0} : cmul(col[c], sc);
      sr += a.x * v.x - a.y * v.y;
      si += a.x * v.y + a.y * v.x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      y[r] = double2{sr, si};
      vbuf[r] = r == 0 ? double2{1, 0} : cmul(col[r], sc);
    }
  }
}

// wraw = tau y and the partial conj(wraw) v
__device__ __forceinline__ void b_w0(int64_t n, const double2 *__restrict__ y,
                                            const double2 *__restrict__ vbuf,
                                            const double2 *__restrict__ tau,
                                            double2 *__restrict__ wraw,
                                            double2 *__restrict__ part2, int wg) {
  __shared__ double sh[ENT / 64];
  const int64_t r = int64_t(wg) * ENT + threadIdx.x;
  double sr = 0, si = 0;
  if (r < n) {
    const double2 w = cmul(tau[0], y[r]);
    wraw[r] = w;
    const double2 c = cmulc(w, vbuf[r]);
    sr = c.x;
    si = c.y;
  }
  sr = block_sum<ENT>(sr, sh);
  si = block_sum<ENT>(si, sh);
  if (threadIdx.x == 0) part2[wg] = double2{sr, si};
}

// A -= v w^dag + w v^dag with w = wraw + alpha v
template <typename TA>
__device__ __forceinline__ void b_rank2(int64_t n, TA *__restrict__ A, int64_t lda,
                                               const double2 *__restrict__ wraw,
                                               const double2 *__restrict__ vbuf,
                                               const double2 *__restrict__ part2, int np2,
                                               const double2 *__restrict__ tau, int64_t r, int64_t xw, int64_t gx) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  double sr = 0, si = 0;
  for (int p = threadIdx.x; p < np2; p += ENT) {
    sr += part2[p].x;
    si += part2[p].y;
  }
  sr = block_sum<ENT>(sr, sh);
  si = block_sum<ENT>(si, sh);
  const double2 t = tau[0];
  const double2 alpha = cmul(double2{-0.5 * t.x, -0.5 * t.y}, double2{sr, si});
    const double2 vr = vbuf[r], wr = cadd(wraw[r], cmul(alpha, vr));
  for (int64_t c = xw * ENT + threadIdx.x; c < n; c += gx * ENT) {
    const double2 vc = vbuf[c], wc = cadd(wraw[c], cmul(alpha, vc));
    CA *p = reinterpret_cast<CA *>(A) + r * lda + c;
    double2 a = to_d2(*p);
    a = csub(a, cmul(vr, cconj(wc)));
    a = csub(a, cmul(wr, cconj(vc)));
    *p = CA{TA(a.x), TA(a.y)};
  }
}

// ---------------------------------------------------------------------------
// panel start: col = A[:, j0] (rows >= j0) and partial |col|^2 over rows >= j0 + 2
// ---------------------------------------------------------------------------
template <typename TA>
__device__ __forceinline__ void b_col0(int64_t n, int64_t j0, const TA *__restrict__ A,
                                              int64_t lda, double2 *__restrict__ col,
                                              double2 *__restrict__ partb, int wg) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  const int64_t r = j0 + int64_t(wg) * ENT + threadIdx.x;
  double s = 0;
  if (r < n) {
    const double2 a = to_d2(reinterpret_cast<const CA *>(A)[r * lda + j0]);
    col[r] = a;
    if (r >= j0 + 2) s = a.x * a.x + a.y * a.y;
  }
  s = block_sum<ENT>(s, sh);
  if (threadIdx.x == 0) partb[int64_t(wg) * PS] = double2{s, 0};
}

// ---------------------------------------------------------------------------
// k_colA: reflector of column jn from its final entries col[jn..n) and the
// partial sums S1 = sum_{r >= jn+2} |col|^2 of k_colB (or k_col0 at a panel
// start): beta, tau and v = (1, scale col[jn+2..]) on rows m0 = jn+1 .. n-1,
// then y = A22 v.  The row sums do not wait for the scalars:
//   y[r] = A[r][m0] + scale * sum_{c > m0} A[r][c] col[c],
// so the loads of A overlap the reduction of S1.  A row is split over WPR
// waves (contiguous column ranges, combined in LDS), each streaming its range
// with a two-stage software pipeline of HU loads per lane.  Every workgroup
// leaves its partial sum of conj(y) v.
// ---------------------------------------------------------------------------
constexpr int HU = 4;

// Workgroups 0..3 of k_colA also reduce the panel dot products that the
// previous k_colB left in its np records (slots 1 .. 2 NBK: BV_l, BW_l):
// workgroup w sums slots 16 w .. 16 w + 15, thread t slot t % 16 over the
// records t / 16, t / 16 + 16, ...; k_colB then reads 2 NBK sums instead of
// every record.
constexpr int BQ = 2;  // record loads per thread issued with the other loads
__device__ __forceinline__ void bred_load(double2 (&q)[BQ], const double2 *__restrict__ partb,
                                          int np, int wg, bool on) {
  const int s = threadIdx.x % 16, g = threadIdx.x / 16;
#pragma unroll
  for (int u = 0; u < BQ; ++u)
    q[u] = on ? partb[int64_t(std::min(g + 16 * u, np - 1)) * PS + 1 + 16 * wg + s]
              : double2{0, 0};
}
__device__ __forceinline__ double2 bred_part(const double2 (&q)[BQ],
                                             const double2 *__restrict__ partb, int np, int wg) {
  const int s = threadIdx.x % 16, g = threadIdx.x / 16;
  double2 acc = {0, 0};
#pragma unroll
  for (int u = 0; u < BQ; ++u)
    if (g + 16 * u < np) acc = cadd(acc, q[u]);
  for (int p0 = g + 16 * BQ; p0 < np; p0 += 16 * BQ) {  // batches issued together
    double2 q2[BQ];
#pragma unroll
    for (int u = 0; u < BQ; ++u)
      q2[u] = partb[int64_t(std::min(p0 + 16 * u, np - 1)) * PS + 1 + 16 * wg + s];
#pragma unroll
    for (int u = 0; u < BQ; ++u)
      if (p0 + 16 * u < np) acc = cadd(acc, q2[u]);
  }
  return acc;
}

template <typename TA, int WPR>
__device__ __forceinline__ void b_colA(int64_t n, int64_t jn, int ir,
                                              const TA *__restrict__ A, int64_t lda,
                                              double2 *__restrict__ V, int64_t ldv,
                                              const double2 *__restrict__ col,
                                              const double2 *__restrict__ partb, int np,
                                              double2 *__restrict__ tau,
                                              double2 *__restrict__ scl, double *__restrict__ d,
                                              double *__restrict__ e, double2 *__restrict__ y,
                                              double2 *__restrict__ parta,
                                              double2 *__restrict__ bred, int wg) {
  typedef typename C2T<TA>::t CA;
  constexpr int RT = (ENT / 64) / WPR;  // rows per workgroup
  __shared__ double sh[ENT / 64];
  __shared__ double sh2[2 * (ENT / 64)];
  __shared__ double2 srow[ENT / 64];
  __shared__ double2 bsh[ENT / 16][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = jn + 1;
  const int64_t r = m0 + int64_t(wg) * RT + wv / WPR;
  const int part = wv % WPR;
  // ---- independent loads: every global load is issued from a clamped,
  // in-bounds index before any value is used, so none waits for another ----
  const bool last = m0 >= n;
  const int64_t rc = std::min<int64_t>(r, n - 1), mc = std::min<int64_t>(m0, n - 1);
  double2 px[PMAX / ENT];  // np <= PMAX = 4 ENT records
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u) px[u] = partb[int64_t(std::min(tid + ENT * u, np - 1)) * PS];
  const bool red_on = wg < 4 && ir > 0 && !last;
  double2 bq[BQ];
  bred_load(bq, partb, np, wg, red_on);
  const double2 cjn = col[jn], cm0 = col[mc], cr = col[rc];
  const double2 a0 = to_d2(reinterpret_cast<const CA *>(A)[rc * lda + mc]);
  const bool lead = lane == 0 && part == 0 && r < n;
  // ---- row sums over this wave's column range ----
  double sr = 0, si = 0;
  if (r < n) {
    const int64_t len = n - (m0 + 1);
    const int64_t per = ((len + WPR - 1) / WPR + 63) / 64 * 64;
    const int64_t cs = m0 + 1 + part * per, ce = std::min<int64_t>(n, cs + per);
    const CA *arow = reinterpret_cast<const CA *>(A) + r * lda;
    CA an[HU];
    double2 cn[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int64_t c = std::min<int64_t>(cs + lane + 64 * u, n - 1);
      an[u] = arow[c];
      cn[u] = col[c];
    }
    for (int64_t c0 = cs; c0 < ce; c0 += 64 * HU) {
      CA ac[HU];
      double2 cc[HU];
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        ac[u] = an[u];
        cc[u] = cn[u];
      }
      const int64_t c1 = c0 + 64 * HU;  // next pass, loaded while this one is summed
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        const int64_t c = std::min<int64_t>(c1 + lane + 64 * u, n - 1);
        an[u] = arow[c];
        cn[u] = col[c];
      }
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        const bool ok = c0 + lane + 64 * u < ce;
        const double2 a = ok ? to_d2(ac[u]) : double2{0, 0};
        sr += a.x * cc[u].x - a.y * cc[u].y;
        si += a.x * cc[u].y + a.y * cc[u].x;
      }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
  }
  double s1 = 0;
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u)
    if (tid + ENT * u < np) s1 += px[u].x;
  if (lane == 0) srow[wv] = double2{sr, si};
  // ---- reflector scalars (every workgroup) ----
  const double S1 = block_sum_once<ENT>(s1, sh);  // also publishes srow
  if (last) {
    if (wg == 0 && tid == 0) d[jn] = cjn.x;
    return;
  }
  double beta;
  double2 tj, sc;
  householder(cm0, S1, beta, tj, sc);
  // the stores follow the reduction: a store whose data registers are
  // reused by the reduction would have to complete first
  double2 yv = {0, 0}, yo = {0, 0}, vo = {0, 0};
  if (lead) {
    double2 rs = srow[wv];
#pragma unroll
    for (int k = 1; k < WPR; ++k) rs = cadd(rs, srow[wv + k]);
    yo = cadd(a0, cmul(sc, rs));
    vo = r == m0 ? double2{1, 0} : cmul(sc, cr);  // lead: r < n, so rc = r
    yv = cmulc(yo, vo);
  }
  if (red_on) bsh[tid / 16][tid % 16] = bred_part(bq, partb, np, wg);
  double yr = yv.x, yi = yv.y;
  block_sum2_once<ENT>(yr, yi, sh2);  // also publishes bsh
  if (red_on && tid < 16) {
    double2 b = bsh[0][tid];
#pragma unroll
    for (int g = 1; g < ENT / 16; ++g) b = cadd(b, bsh[g][tid]);
    bred[16 * wg + tid] = b;
  }
  if (lead) {
    y[r] = yo;
    V[int64_t(ir) * ldv + r] = vo;
  }
  if (tid == 0) {
    parta[wg] = double2{yr, yi};
    if (wg == 0) {
      d[jn] = cjn.x;
      e[jn] = beta;
      tau[m0] = tj;
      scl[m0] = sc;
    }
  }
}

// k_colA for large trailing blocks: LDS_RW rows per wave, 4 LDS_RW rows per
// workgroup.  The current column is staged in LDS in chunks of CCH entries,
// so each workgroup reads it from L2 once for all its rows instead of once
// per row (FP64 column entries are twice the bytes of FP32 A entries); every
// lane keeps LDS_RW x U row loads in flight.  Same results as b_colA.
template <typename TA>
__device__ __forceinline__ void b_colA_lds(int64_t n, int64_t jn, int ir,
                                           const TA *__restrict__ A, int64_t lda,
                                           double2 *__restrict__ V, int64_t ldv,
                                           const double2 *__restrict__ col,
                                           const double2 *__restrict__ partb, int np,
                                           double2 *__restrict__ tau, double2 *__restrict__ scl,
                                           double *__restrict__ d, double *__restrict__ e,
                                           double2 *__restrict__ y, double2 *__restrict__ parta,
                                           double2 *__restrict__ bred, int wg) {
  typedef typename C2T<TA>::t CA;
  constexpr int RW = LDS_RW, RWG = (ENT / 64) * RW;
  constexpr int CCH = 2048;     // column entries per LDS chunk (32 KB)
  constexpr int U = 16 / RW;    // columns per lane per pass: RW U = 16 loads in flight
  __shared__ double sh[ENT / 64];
  __shared__ double sh2[2 * (ENT / 64)];
  __shared__ double2 xs[CCH];
  __shared__ double2 bsh[ENT / 16][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = jn + 1;
  const bool last = m0 >= n;
  const int64_t mc = std::min<int64_t>(m0, n - 1);
  const int64_t rbase = m0 + int64_t(wg) * RWG + int64_t(wv) * RW;
  double2 px[PMAX / ENT];
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u) px[u] = partb[int64_t(std::min(tid + ENT * u, np - 1)) * PS];
  const bool red_on = wg < 4 && ir > 0 && !last;
  double2 bq[BQ];
  bred_load(bq, partb, np, wg, red_on);
  const double2 cjn = col[jn], cm0 = col[mc];
  const CA *arow[RW];
  double2 a0[RW], cr[RW];
  double sr[RW], si[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    const int64_t rk = std::min<int64_t>(rbase + k, n - 1);
    arow[k] = reinterpret_cast<const CA *>(A) + rk * lda;
    a0[k] = to_d2(arow[k][mc]);
    cr[k] = col[rk];
    sr[k] = si[k] = 0.0;
  }
  for (int64_t c0 = m0 + 1; c0 < n; c0 += CCH) {
    const int cn = int(std::min<int64_t>(CCH, n - c0));
    __syncthreads();
    for (int t = tid; t < cn; t += ENT) xs[t] = col[c0 + t];
    __syncthreads();
    if constexpr (sizeof(TA) == 4) {
      // FP32 working copy: two adjacent columns per lane in one 16-byte load
      // (rows start at multiples of 16 entries, so an even column is aligned)
      const int first = int(c0 & 1);
      if (first && lane == 0) {
        const double2 x = xs[0];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
          const double2 av = to_d2(arow[k][c0]);
          sr[k] += av.x * x.x - av.y * x.y;
          si[k] += av.x * x.y + av.y * x.x;
        }
      }
      constexpr int U2 = U / 2;
      int cc = first + 2 * lane;
      for (; cc + 1 + (U2 - 1) * 128 < cn; cc += U2 * 128) {
        float4 a[RW][U2];
#pragma unroll
        for (int k = 0; k < RW; ++k)
#pragma unroll
          for (int u = 0; u < U2; ++u)
            a[k][u] = *reinterpret_cast<const float4 *>(arow[k] + c0 + cc + 128 * u);
#pragma unroll
        for (int u = 0; u < U2; ++u) {
          const double2 x0 = xs[cc + 128 * u], x1 = xs[cc + 1 + 128 * u];
#pragma unroll
          for (int k = 0; k < RW; ++k) {
            const double ar = a[k][u].x, ai = a[k][u].y, br = a[k][u].z, bi = a[k][u].w;
            sr[k] += ar * x0.x - ai * x0.y;
            si[k] += ar * x0.y + ai * x0.x;
            sr[k] += br * x1.x - bi * x1.y;
            si[k] += br * x1.y + bi * x1.x;
          }
        }
      }
      for (; cc < cn; cc += 128) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (cc + h < cn) {
            const double2 x = xs[cc + h];
#pragma unroll
            for (int k = 0; k < RW; ++k) {
              const double2 av = to_d2(arow[k][c0 + cc + h]);
              sr[k] += av.x * x.x - av.y * x.y;
              si[k] += av.x * x.y + av.y * x.x;
            }
          }
        }
      }
      continue;
    }
    int cc = lane;
    for (; cc + (U - 1) * 64 < cn; cc += U * 64) {
      CA a[RW][U];
#pragma unroll
      for (int k = 0; k < RW; ++k)
#pragma unroll
        for (int u = 0; u < U; ++u) a[k][u] = arow[k][c0 + cc + 64 * u];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 x = xs[cc + 64 * u];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
          const double2 av = to_d2(a[k][u]);
          sr[k] += av.x * x.x - av.y * x.y;
          si[k] += av.x * x.y + av.y * x.x;
        }
      }
    }
    for (; cc < cn; cc += 64) {
      const double2 x = xs[cc];
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        const double2 av = to_d2(arow[k][c0 + cc]);
        sr[k] += av.x * x.x - av.y * x.y;
        si[k] += av.x * x.y + av.y * x.x;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    sr[k] = wave_sum(sr[k]);
    si[k] = wave_sum(si[k]);
  }
  double s1 = 0;
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u)
    if (tid + ENT * u < np) s1 += px[u].x;
  const double S1 = block_sum_once<ENT>(s1, sh);
  if (last) {
    if (wg == 0 && tid == 0) d[jn] = cjn.x;
    return;
  }
  double beta;
  double2 tj, sc;
  householder(cm0, S1, beta, tj, sc);
  double2 yv = {0, 0}, yo[RW], vo[RW];  // stores after the reduction, as in b_colA
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    const int64_t r = rbase + k;
    yo[k] = cadd(a0[k], cmul(sc, double2{sr[k], si[k]}));
    vo[k] = r == m0 ? double2{1, 0} : cmul(sc, cr[k]);
    if (lane == 0 && r < n) yv = cadd(yv, cmulc(yo[k], vo[k]));
  }
  if (red_on) bsh[tid / 16][tid % 16] = bred_part(bq, partb, np, wg);
  double yr = yv.x, yi = yv.y;
  block_sum2_once<ENT>(yr, yi, sh2);  // also publishes bsh
  if (red_on && tid < 16) {
    double2 b = bsh[0][tid];
#pragma unroll
    for (int g = 1; g < ENT / 16; ++g) b = cadd(b, bsh[g][tid]);
    bred[16 * wg + tid] = b;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      const int64_t r = rbase + k;
      if (r < n) {
        y[r] = yo[k];
        V[int64_t(ir) * ldv + r] = vo[k];
      }
    }
  }
  if (tid == 0) {
    parta[wg] = double2{yr, yi};
    if (wg == 0) {
      d[jn] = cjn.x;
      e[jn] = beta;
      tau[m0] = tj;
      scl[m0] = sc;
    }
  }
}

// Sums of RG values (complex) over the 64 lanes of a wave in one butterfly:
// each exchange halves the values a lane keeps, so lane l ends with the full
// sum of value l / (64 / RG) after RG - 1 + 6 - log2(RG) complex shuffles
// (instead of 6 RG).
template <int RG, int L>
__device__ __forceinline__ void wave_fold(double2 (&v)[RG], int lane) {
  if constexpr (L > 1) {
    constexpr int o = 32 * L / RG;  // 32 for the first exchange
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
      const double2 keep = hi ? v[i + L / 2] : v[i], send = hi ? v[i] : v[i + L / 2];
      v[i] = double2{keep.x + __shfl_xor(send.x, o, 64), keep.y + __shfl_xor(send.y, o, 64)};
    }
    wave_fold<RG, L / 2>(v, lane);
  }
}
template <int RG>
__device__ __forceinline__ double2 wave_sums(double2 (&v)[RG], int lane) {
  wave_fold<RG, RG>(v, lane);
  double2 x = v[0];
#pragma unroll
  for (int o = 32 / RG; o > 0; o >>= 1) {
    x.x += __shfl_xor(x.x, o, 64);
    x.y += __shfl_xor(x.y, o, 64);
  }
  return x;
}

// k_colA, tile forms (more than TILE_M trailing rows):
// the same reflector, V column, scalars and panel-product reduction as
// b_colA_lds, with the HEMV y = A22 v taken from the lower tiles of the
// trailing block.  Workgroup wg takes tile (bi, bj), bi >= bj, of the grid
// of T x T tiles starting at g_tbase(m0).  A diagonal tile multiplies its
// whole square (both triangles); a tile below the diagonal also stands for
// its mirror above the diagonal: its row sums go to slot bj of its rows, the
// sums conj(A[r][c]) v[r] over its rows to slot bi of its columns.  The partial
// sums of y^dag v come per tile in the same way.  The entries v[m0] = 1 and
// v[c] = scale col[c] (c > m0) enter as col[c] with the scale applied to the
// finished sums, the column m0 separately (as in b_colA_lds).
template <typename TA, int T>
__device__ __forceinline__ void b_colA_tile(int64_t n, int64_t jn, int ir,
                                            const TA *__restrict__ A, int64_t lda,
                                            double2 *__restrict__ V, int64_t ldv,
                                            const double2 *__restrict__ col,
                                            const double2 *__restrict__ partb, int np,
                                            double2 *__restrict__ tau, double2 *__restrict__ scl,
                                            double *__restrict__ d, double *__restrict__ e,
                                            double2 *__restrict__ ys, int64_t ldys,
                                            double2 *__restrict__ parta,
                                            double2 *__restrict__ bred, int wg) {
  static_assert(T == 64 || T == 128 || T == 256, "tile sizes");
  typedef typename C2T<TA>::t CA;
  constexpr bool F32 = sizeof(TA) == 4;
  constexpr int CPL = T / 64;                            // complex entries per lane and row
  constexpr int RPW = T / (ENT / 64);                    // rows per wave
  // rows in flight per wave (16-byte loads: 16 per lane for FP32, 8 for FP64)
  constexpr int RG = F32 ? (T == 64 ? 16 : (T == 128 ? 8 : 4)) : (T == 64 ? 8 : 4);
  static_assert(RPW % RG == 0, "row groups");
  __shared__ double sh[ENT / 64];
  __shared__ double sh2[2 * (ENT / 64)];
  __shared__ double2 xr[T], xc[T];     // col[] at the tile's rows / columns (0 unless m0 < . < n)
  __shared__ double2 cpart[ENT / 64][T];
  __shared__ double2 rpart[T];
  __shared__ double2 bsh[ENT / 16][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = jn + 1, base = g_tbase(m0);
  int bi = int((sqrt(8.0 * double(wg) + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= wg) ++bi;
  while (bi > 0 && bi * (bi + 1) / 2 > wg) --bi;
  const int bj = wg - bi * (bi + 1) / 2;
  const bool diag = bi == bj;
  const int64_t r0 = base + int64_t(bi) * T, c0 = base + int64_t(bj) * T;
  // ---- loads that do not depend on the tile's products ----
  double2 px[PMAX / ENT];
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u) px[u] = partb[int64_t(std::min(tid + ENT * u, np - 1)) * PS];
  const bool red_on = wg < 4 && ir > 0;
  double2 bq[BQ];
  bred_load(bq, partb, np, wg, red_on);
  const double2 cjn = col[jn], cm0 = col[m0];
  // thread t < T: row r0 + t and column c0 + t of the tile
  const int64_t rt = r0 + tid, ct = c0 + tid;
  double2 a0 = {0, 0};
  if (tid < T) {
    xr[tid] = (rt > m0 && rt < n) ? col[rt] : double2{0, 0};
    xc[tid] = (ct > m0 && ct < n) ? col[ct] : double2{0, 0};
    if (bj == 0) a0 = to_d2(reinterpret_cast<const CA *>(A)[std::min<int64_t>(std::max<int64_t>(rt, m0), n - 1) * lda + m0]);
  }
  __syncthreads();
  // this lane's columns: FP32 with CPL > 1: c0 + 2 lane + 128 (u / 2) + (u & 1)
  // (pairs of columns in one 16-byte load); otherwise c0 + lane + 64 u
  auto lcol = [&](int u) { return (F32 && CPL > 1) ? 2 * lane + 128 * (u / 2) + (u & 1) : lane + 64 * u; };
  double2 xl[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) xl[u] = xc[lcol(u)];
  double2 cacc[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) cacc[u] = double2{0, 0};
  const TA *arow0 = A;
  // Columns at or past n: the loads stay inside the row (padding to lda), and
  // the values are replaced by zero, since the padding holds no data (its x
  // entries are zero, but 0 times NaN is not).
  bool cok[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) cok[u] = c0 + lcol(u) < n;
  for (int g = 0; g < RPW / RG; ++g) {
    const int rl0 = wv * RPW + g * RG;
    double2 acc[RG];
    if constexpr (F32 && CPL == 1) {
      float2 a[RG];
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const int64_t rr = std::min<int64_t>(std::max<int64_t>(r0 + rl0 + q, m0), n - 1);
        const int64_t cc = std::min<int64_t>(c0 + lane, lda - 1);
        a[q] = reinterpret_cast<const float2 *>(arow0)[rr * lda + cc];
      }
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const double2 av = cok[0] ? to_d2(a[q]) : double2{0, 0};
        acc[q] = cmul(av, xl[0]);
        if (!diag) cacc[0] = cadd(cacc[0], cmulc(av, xr[rl0 + q]));
      }
    } else if constexpr (!F32) {
      CA a[RG][CPL];
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const int64_t rr = std::min<int64_t>(std::max<int64_t>(r0 + rl0 + q, m0), n - 1);
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const int64_t cc = std::min<int64_t>(c0 + lane + 64 * u, lda - 1);
          a[q][u] = reinterpret_cast<const CA *>(arow0)[rr * lda + cc];
        }
      }
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const double2 xq = xr[rl0 + q];
        double2 sacc = {0, 0};
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const double2 av = cok[u] ? to_d2(a[q][u]) : double2{0, 0};
          sacc = cadd(sacc, cmul(av, xl[u]));
          if (!diag) cacc[u] = cadd(cacc[u], cmulc(av, xq));
        }
        acc[q] = sacc;
      }
    } else {
      float4 a[RG][CPL / 2];
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const int64_t rr = std::min<int64_t>(std::max<int64_t>(r0 + rl0 + q, m0), n - 1);
#pragma unroll
        for (int u = 0; u < CPL / 2; ++u) {
          const int64_t cc = std::min<int64_t>(c0 + 2 * lane + 128 * u, lda - 2);
          a[q][u] = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(arow0) + 2 * (rr * lda + cc));
        }
      }
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const double2 xq = xr[rl0 + q];
        double2 sacc = {0, 0};
#pragma unroll
        for (int u = 0; u < CPL / 2; ++u) {
          const double2 av = cok[2 * u] ? double2{double(a[q][u].x), double(a[q][u].y)} : double2{0, 0};
          const double2 bv = cok[2 * u + 1] ? double2{double(a[q][u].z), double(a[q][u].w)} : double2{0, 0};
          sacc = cadd(sacc, cadd(cmul(av, xl[2 * u]), cmul(bv, xl[2 * u + 1])));
          if (!diag) {
            cacc[2 * u] = cadd(cacc[2 * u], cmulc(av, xq));
            cacc[2 * u + 1] = cadd(cacc[2 * u + 1], cmulc(bv, xq));
          }
        }
        acc[q] = sacc;
      }
    }
    const double2 rs = wave_sums<RG>(acc, lane);
    if (lane % (64 / RG) == 0) rpart[rl0 + lane / (64 / RG)] = rs;
  }
  if (!diag) {
#pragma unroll
    for (int u = 0; u < CPL; ++u) cpart[wv][lcol(u)] = cacc[u];
  }
  double s1 = 0;
#pragma unroll
  for (int u = 0; u < PMAX / ENT; ++u)
    if (tid + ENT * u < np) s1 += px[u].x;
  const double S1 = block_sum_once<ENT>(s1, sh);  // also publishes rpart, cpart
  double beta;
  double2 tj, sc;
  householder(cm0, S1, beta, tj, sc);
  double2 qf = {0, 0};
  if (tid < T) {
    if (rt >= m0 && rt < n) {
      const double2 yr = cadd(cmul(sc, rpart[tid]), a0);
      const double2 vr = rt == m0 ? double2{1, 0} : cmul(sc, xr[tid]);
      qf = cmulc(yr, vr);
      ys[int64_t(bj) * ldys + rt] = yr;
      if (diag) V[int64_t(ir) * ldv + rt] = vr;
    }
    if (!diag && ct >= m0 && ct < n) {
      double2 cs = cpart[0][tid];
#pragma unroll
      for (int w = 1; w < ENT / 64; ++w) cs = cadd(cs, cpart[w][tid]);
      const double2 yc = cmul(sc, cs);
      const double2 vc = ct == m0 ? double2{1, 0} : cmul(sc, xc[tid]);
      qf = cadd(qf, cmulc(yc, vc));
      ys[int64_t(bi) * ldys + ct] = yc;
    }
  }
  if (red_on) bsh[tid / 16][tid % 16] = bred_part(bq, partb, np, wg);
  double qr = qf.x, qi = qf.y;
  block_sum2_once<ENT>(qr, qi, sh2);  // also publishes bsh
  if (red_on && tid < 16) {
    double2 b = bsh[0][tid];
#pragma unroll
    for (int gq = 1; gq < ENT / 16; ++gq) b = cadd(b, bsh[gq][tid]);
    bred[16 * wg + tid] = b;
  }
  if (tid == 0) {
    parta[wg] = double2{qr, qi};
    if (wg == 0) {
      d[jn] = cjn.x;
      e[jn] = beta;
      tau[m0] = tj;
      scl[m0] = sc;
    }
  }
}

// sum of part[0..np) with eight loads in flight per thread
__device__ __forceinline__ double2 gather_sum(const double2 *__restrict__ part, int np, int tid) {
  double2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int p = tid + ENT * u;
    acc[u] = p < np ? part[p] : double2{0, 0};
  }
  for (int p = tid + 8 * ENT; p < np; p += ENT) acc[0] = cadd(acc[0], part[p]);
#pragma unroll
  for (int u = 1; u < 8; ++u) acc[0] = cadd(acc[0], acc[u]);
  return acc[0];
}

// ---------------------------------------------------------------------------
// k_colB: column jn (panel index ir), rows r >= jx = jn + 1, RB rows per
// workgroup.  With the panel dot products of the new reflector
//   p_l = V_l^dag v = conj(V_l[jx]) + scale BV_l,  q_l = W_l^dag v = conj(W_l[jx]) + scale BW_l
// (l < ir, from the partial sums BV, BW of the previous column, which k_colA
// has summed over the records into bred) and
//   w^dag v = conj(tau) (y^dag v - 2 Re(p^dag q)),  alpha = -tau (w^dag v) / 2:
//   W_ir[r] = tau (y[r] - sum_{l<ir} (V_l[r] q_l + W_l[r] p_l)) + alpha v[r]
// and, if column jx is in the panel, its entries with every update
//   col[r] = A[r][jx] - sum_{l<=ir} (V_l[r] conj(W_l[jx]) + W_l[r] conj(V_l[jx]))
// together with the partial sums over rows >= jx + 2 that the next column needs.
// Record of one workgroup: [0] (S1, 0), [1 + l] BV_l, [1 + NBK + l] BW_l.
// The workgroup's rows of V_0..V_ir, W_0..W_ir are staged in LDS once; four
// threads share a row (sums over l) or a column (sums over rows).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 shfl_sum4(double2 x) {
  x.x += __shfl_xor(x.x, 1, 64);
  x.y += __shfl_xor(x.y, 1, 64);
  x.x += __shfl_xor(x.x, 2, 64);
  x.y += __shfl_xor(x.y, 2, 64);
  return x;
}

template <typename TA>
__device__ __forceinline__ void b_colB(int64_t n, int64_t jn, int ir, int more,
                                              const TA *__restrict__ A, int64_t lda,
                                              const double2 *__restrict__ V,
                                              double2 *__restrict__ W, int64_t ldv,
                                              const double2 *__restrict__ y,
                                              const double2 *__restrict__ ys, int64_t ldys,
                                              int nbt,
                                              const double2 *__restrict__ parta, int npa,
                                              const double2 *__restrict__ bred,
                                              const double2 *__restrict__ tau,
                                              const double2 *__restrict__ scl,
                                              double2 *__restrict__ col,
                                              double2 *__restrict__ pout, int wg) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  __shared__ double sh2[2 * (ENT / 64)];
  __shared__ double2 tile[2 * NBK * TP];  // [V_0..V_{NBK-1} | W_0..W_{NBK-1}] x rows
  __shared__ double2 spq[ENT / 64][2 * NBK], shd[2 * NBK];  // p | q per wave, head V_l[jx] | W_l[jx]
  __shared__ double2 sy[RB], sa[RB], sv[RB], sw[RB], sc_[RB];
  __shared__ double2 syj[ENT / 64];  // tile forms: partial sums of y[jx] per wave
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t jx = jn + 1;
  const int64_t rb = jx + int64_t(wg) * RB;
  // ---- loads: every global load is issued from a clamped, in-bounds index
  // before any value is consumed, so none waits for another ----
  constexpr int NT = 2 * NBK * RB / ENT;  // tile entries per thread
  const int i = tid % RB, k0 = tid / RB;
  const int64_t r0 = rb + i, rcl = std::min<int64_t>(r0, n - 1);
  // panel dot products of the previous column's records, reduced by k_colA
  const double2 bvx = bred[lane % NBK], bwx = bred[NBK + lane % NBK];
  double2 tx[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int k = k0 + (ENT / RB) * u, l = k % NBK;  // uniform over the wave
    tx[u] = l < ir ? (k < NBK ? V : W)[int64_t(l) * ldv + rcl] : double2{0, 0};
  }
  const double2 hx = (tid < NBK ? V : W)[int64_t(tid % NBK) * ldv + jx];
  // y of row rcl, or (tile forms) of row ry: four lanes per row, each summing
  // the slots kk, kk + 4, ... of it, and y[jx] from slots tid, tid + ENT, ...
  static_assert(RB == 16 * (ENT / 64), "tile forms: 16 rows per wave");
  const int ryl = wv * 16 + (lane >> 2), kk = lane & 3;
  const int64_t ry = rb + ryl;
  double2 yx = {0, 0}, yj = {0, 0};
  if (nbt == 0) {
    yx = y[rcl];
  } else {
    const int64_t ryc = std::min<int64_t>(ry, n - 1);
    // the first 16 slots of each lane in flight together (clamped, masked),
    // any further ones in a loop
    constexpr int YQ = 16;
    double2 yq[YQ];
#pragma unroll
    for (int u = 0; u < YQ; ++u) yq[u] = ys[int64_t(std::min(kk + 4 * u, nbt - 1)) * ldys + ryc];
    for (int k = tid; k < nbt; k += ENT) yj = cadd(yj, ys[int64_t(k) * ldys + jx]);
#pragma unroll
    for (int u = 0; u < YQ; ++u)
      if (kk + 4 * u < nbt) yx = cadd(yx, yq[u]);
    for (int k = kk + 4 * YQ; k < nbt; k += 4) yx = cadd(yx, ys[int64_t(k) * ldys + ryc]);
  }
  const double2 vx = V[int64_t(ir) * ldv + rcl];
  const double2 ax = to_d2(reinterpret_cast<const CA *>(A)[rcl * lda + jx]);
  // The partial sums of k_colA come in a few fixed sizes chosen by a uniform
  // branch on their count, so that no duplicate (clamped) entry is fetched
  // more than the size class needs.
  constexpr int NG = 16;  // partial sums of k_colA held in registers per thread
  double2 gx[NG];
  auto load_gx = [&](auto cnt) {
    constexpr int C = decltype(cnt)::value;
#pragma unroll
    for (int u = 0; u < NG; ++u) gx[u] = u < C ? parta[std::min(tid + ENT * u, npa - 1)] : double2{0, 0};
  };
  if (npa <= ENT) load_gx(std::integral_constant<int, 1>());
  else if (npa <= 2 * ENT) load_gx(std::integral_constant<int, 2>());
  else if (npa <= 4 * ENT) load_gx(std::integral_constant<int, 4>());
  else load_gx(std::integral_constant<int, NG>());
  const double2 t = tau[jx], sc = scl[jx];
  double2 yjx = nbt == 0 ? y[jx] : double2{0, 0};
  // ---- consume ----
  if (tid < 2 * NBK) shd[tid] = tid % NBK < ir ? hx : double2{0, 0};
#pragma unroll
  for (int u = 0; u < NT; ++u) tile[(k0 + (ENT / RB) * u) * TP + i] = r0 < n ? tx[u] : double2{0, 0};
  if (nbt > 0) {
    yx.x += __shfl_xor(yx.x, 1, 64);
    yx.y += __shfl_xor(yx.y, 1, 64);
    yx.x += __shfl_xor(yx.x, 2, 64);
    yx.y += __shfl_xor(yx.y, 2, 64);
    if (kk == 0) sy[ryl] = ry < n ? yx : double2{0, 0};
    yj.x = wave_sum(yj.x);
    yj.y = wave_sum(yj.y);
    if (lane == 0) syj[wv] = yj;
  }
  if (tid < RB) {
    if (nbt == 0) sy[i] = r0 < n ? yx : double2{0, 0};
    sv[i] = r0 < n ? vx : double2{0, 0};
    sa[i] = (more && r0 < n) ? ax : double2{0, 0};
  }
  double2 ypart = {0, 0};
#pragma unroll
  for (int u = 0; u < NG; ++u)
    if (tid + ENT * u < npa) ypart = cadd(ypart, gx[u]);
  for (int p = tid + NG * ENT; p < npa; p += ENT) ypart = cadd(ypart, parta[p]);
  double yr = ypart.x, yi = ypart.y;
  block_sum2_once<ENT>(yr, yi, sh2);  // also publishes the LDS stores above
  if (nbt > 0) {
    yjx = syj[0];
#pragma unroll
    for (int w = 1; w < ENT / 64; ++w) yjx = cadd(yjx, syj[w]);
  }
  // every wave, lane l < NBK: p_l, q_l, Re(conj(p_l) q_l) and the head term
  // V_l[jx] q_l + W_l[jx] p_l, summed over l in one pass; each wave keeps its
  // own copy of p and q in LDS, so no barrier is needed before the rows
  double pq_re, hr, hi;
  {
    double2 pl = {0, 0}, ql = {0, 0}, hl = {0, 0};
    if (lane < ir) {
      const int lw = NBK + lane;
      pl = cadd(cconj(shd[lane]), cmul(sc, bvx));
      ql = cadd(cconj(shd[lw]), cmul(sc, bwx));
      hl = cadd(cmul(shd[lane], ql), cmul(shd[lw], pl));
    }
    if (lane < NBK) {
      spq[wv][lane] = pl;
      spq[wv][NBK + lane] = ql;
    }
    pq_re = wave_sum(pl.x * ql.x + pl.y * ql.y);  // Re(p^dag q)
    hr = wave_sum(hl.x);
    hi = wave_sum(hl.y);
  }
  const double2 wdv = cmulc(t, double2{yr - 2.0 * pq_re, yi});
  const double2 alpha = cmul(double2{-0.5 * t.x, -0.5 * t.y}, wdv);
  // head entry W_ir[jx] (v[jx] = 1)
  const double2 wh = more ? cadd(cmul(t, csub(yjx, double2{hr, hi})), alpha) : double2{0, 0};
  // ---- rows: four threads per row, panel columns l = part, part + 4, ... ----
  const int row = tid >> 2, part = tid & 3;
  const int64_t r = rb + row;
  double2 hw = {0, 0}, hc = {0, 0};
#pragma unroll
  for (int l0 = 0; l0 < NBK; l0 += 4) {
    const int l = l0 + part;
    if (l < ir) {
      const double2 vl = tile[l * TP + row], wl = tile[(NBK + l) * TP + row];
      hw = cadd(hw, cadd(cmul(vl, spq[wv][NBK + l]), cmul(wl, spq[wv][l])));
      hc = cadd(hc, cadd(cmul(vl, cconj(shd[NBK + l])), cmul(wl, cconj(shd[l]))));
    }
  }
  hw = shfl_sum4(hw);
  hc = shfl_sum4(hc);
  const double2 v = sv[row];
  const double2 w = cadd(cmul(t, csub(sy[row], hw)), cmul(alpha, v));
  double2 c = {0, 0};
  if (more) c = csub(csub(csub(sa[row], hc), cmul(v, cconj(wh))), w);  // conj(V_ir[jx]) = 1
  if (part == 0) {
    if (r < n) {
      W[int64_t(ir) * ldv + r] = w;
      if (more) col[r] = c;
    }
    sw[row] = r < n ? w : double2{0, 0};
    sc_[row] = (r < n && r >= jx + 2) ? c : double2{0, 0};
  }
  if (!more) return;
  double s1 = (part == 0 && r < n && r >= jx + 2) ? c.x * c.x + c.y * c.y : 0.0;
  s1 = block_sum_once<ENT>(s1, sh);  // also publishes sw, sc_
  double2 *pr = pout + int64_t(wg) * PS;
  if (tid == 0) pr[0] = double2{s1, 0};
  // ---- BV_l, BW_l (l <= ir): four threads per panel column ----
  const int k = tid >> 2, l = k % NBK;
  const bool isw = k >= NBK;
  if (l <= ir) {
    double2 acc = {0, 0};
#pragma unroll 4
    for (int i = part; i < RB; i += 4) {
      const double2 m = l < ir ? tile[k * TP + i] : (isw ? sw[i] : sv[i]);
      acc = cadd(acc, cmulc(m, sc_[i]));
    }
    acc = shfl_sum4(acc);  // the four lanes of a column are active together
    if (part == 0) pr[1 + k] = acc;
  }
}

// Trailing update on MFMA: A[r][c] -= sum_l V_l[r] conj(W_l[c]) + W_l[r] conj(V_l[c])
// for r, c >= c0; real GEMM with K = 4 nbk (x conj(y) interleave, see bse_build).

template <typename T, int S>
__device__ __forceinline__ void b_her2k(int64_t n, int64_t c0, int nbk,
                                               const double2 *__restrict__ V,
                                               const double2 *__restrict__ W, int64_t ldv,
                                               T *__restrict__ A, int64_t lda, int64_t bx, int64_t by,
                                               bool mirror) {
  constexpr int BM = HerTile<T, S>::BM, BN = HerTile<T, S>::BN, BK = HerTile<T, S>::BK;
  constexpr int P = Pitch<T, BK>::value, MI = BM / 32, NI = BN / 32, KC = BK / 2;
  constexpr int NA = (BM / 2) * KC / ENT, NB = BN * KC / ENT;
  static_assert(BM == 2 * BN, "square tiles in complex entries");
  typedef typename C2T<T>::t C2;
  constexpr int UP = BN + 1;  // LDS pitch of the staged update
  constexpr size_t SLAB = sizeof(T) * (BM + BN) * P, STAGE = sizeof(C2) * BN * UP;
  __shared__ __attribute__((aligned(16))) char smem[SLAB > STAGE ? SLAB : STAGE];
  T *As = reinterpret_cast<T *>(smem), *Bs = As + BM * P;
  C2 *Us = reinterpret_cast<C2 *>(smem);  // after the slabs: [a][b] update of the tile
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t a0 = c0 + by * (BM / 2), b0 = c0 + bx * BN;
  if (a0 >= n || b0 >= n) return;
  typename Mfma<T>::acc_t acc[MI][NI];
  acc_zero<T, MI, NI>(acc);
  const int wm0 = (wv >> 1) * (BM / 2), wn0 = (wv & 1) * (BN / 2);
  const int K2 = 2 * nbk;  // complex reduction length: [V | W] against [W | V]
  for (int i0 = 0; i0 < K2; i0 += KC) {
    // every load from an in-bounds address (rows clamped to n - 1, panel
    // columns to K2 - 1), all issued before any is used; out-of-range
    // entries are zeroed by selects, so no load sits behind a branch
    double2 xa[NA], xb[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u) {  // consecutive threads: consecutive rows (column major V, W)
      const int it = tid + ENT * u, r = it % (BM / 2), ii = it / (BM / 2);
      const int I = std::min(i0 + ii, K2 - 1);
      const int64_t ac = std::min<int64_t>(a0 + r, n - 1);
      xa[u] = (I < nbk ? V + int64_t(I) * ldv : W + int64_t(I - nbk) * ldv)[ac];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + ENT * u, r = it % BN, ii = it / BN;
      const int I = std::min(i0 + ii, K2 - 1);
      const int64_t bc = std::min<int64_t>(b0 + r, n - 1);
      xb[u] = (I < nbk ? W + int64_t(I) * ldv : V + int64_t(I - nbk) * ldv)[bc];
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + ENT * u, r = it % (BM / 2), ii = it / (BM / 2);
      const bool ok = a0 + r < n && i0 + ii < K2;
      const double2 x = {ok ? xa[u].x : 0.0, ok ? xa[u].y : 0.0};
      *reinterpret_cast<C2 *>(As + (2 * r) * P + 2 * ii) = C2{T(x.x), T(x.y)};
      *reinterpret_cast<C2 *>(As + (2 * r + 1) * P + 2 * ii) = C2{T(x.y), T(-x.x)};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + ENT * u, r = it % BN, ii = it / BN;
      const bool ok = b0 + r < n && i0 + ii < K2;
      const double2 x = {ok ? xb[u].x : 0.0, ok ? xb[u].y : 0.0};
      *reinterpret_cast<C2 *>(Bs + r * P + 2 * ii) = C2{T(x.x), T(x.y)};
    }
    __syncthreads();
    mfma_slab<T, MI, NI, BK>(acc, As, Bs, wm0, wn0, lane);
    __syncthreads();
  }
  const int r16 = lane & 15, g = lane >> 4;
  // read-modify-write of the tile: every read first (clamped addresses),
  // then the predicated writes, so no read waits behind a write
  C2 old[MI][NI][2];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int64_t b = std::min<int64_t>(b0 + wn0 + 16 * ni + r16, n - 1);
      const int64_t a = a0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        old[mi][ni][h] = reinterpret_cast<const C2 *>(A)[std::min<int64_t>(a + h, n - 1) * lda + b];
    }
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int64_t b = b0 + wn0 + 16 * ni + r16;
      const int64_t a = a0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        C2 x = old[mi][ni][h];
        x.x -= acc[mi][ni][2 * h];
        x.y -= acc[mi][ni][2 * h + 1];
        if (a + h < n && b < n) reinterpret_cast<C2 *>(A)[(a + h) * lda + b] = x;
      }
    }
  if (!mirror || bx == by) return;  // a diagonal tile holds both triangles itself
  // mirror tile: A[b][a] -= conj(U[a][b])
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int al = (wm0 + 16 * mi + 4 * g) / 2 + h, bl = wn0 + 16 * ni + r16;
        Us[al * UP + bl] = C2{acc[mi][ni][2 * h], acc[mi][ni][2 * h + 1]};
      }
  __syncthreads();  // (the last slab ended with a barrier: smem is free)
  const int il = tid % BN;
  constexpr int JM = BN / (ENT / BN);  // mirror entries per thread
  C2 mold[JM];
  const int64_t ac = std::min<int64_t>(a0 + il, n - 1);
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int jl = tid / BN + (ENT / BN) * q;
    mold[q] = reinterpret_cast<const C2 *>(A)[std::min<int64_t>(b0 + jl, n - 1) * lda + ac];
  }
#pragma unroll
  for (int q = 0; q < JM; ++q) {
    const int jl = tid / BN + (ENT / BN) * q;
    const int64_t b = b0 + jl, a = a0 + il;
    const C2 u = Us[il * UP + jl];
    C2 x = mold[q];
    x.x -= u.x;
    x.y += u.y;
    if (b < n && a < n) reinterpret_cast<C2 *>(A)[b * lda + a] = x;
  }
}

#include "eigh_band.h"

// ---------------------------------------------------------------------------
// tridiagonal eigenvalues (multisection) and cluster weights
// ---------------------------------------------------------------------------
// 1 / x to full double precision: hardware estimate plus two Newton steps
// (arguments are kept away from zero and denormals by the pivot guard).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// scalars: [0] Gershgorin low, [1] high, [2] |T| (max row sum), [3] pivmin,
// [4] cluster gap tolerance
__device__ __forceinline__ void b_tri_prep(int64_t n, const double *__restrict__ d,
                                                  const double *__restrict__ e, double ctol_rel,
                                                  double *__restrict__ e2,
                                                  double *__restrict__ sc,
                                                  int32_t *__restrict__ status) {
  if (threadIdx.x < 4) status[threadIdx.x] = 0;  // counters of this solve
  __shared__ double s_lo[RNT / 64], s_hi[RNT / 64], s_tn[RNT / 64];
  double lo = 1e300, hi = -1e300, tn = 0;
  for (int64_t k = threadIdx.x; k < n; k += RNT) {
    const double el = k > 0 ? fabs(e[k - 1]) : 0.0, er = k + 1 < n ? fabs(e[k]) : 0.0;
    lo = fmin(lo, d[k] - el - er);
    hi = fmax(hi, d[k] + el + er);
    tn = fmax(tn, fabs(d[k]) + el + er);
    if (k + 1 < n) e2[k] = e[k] * e[k];
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    tn = fmax(tn, __shfl_xor(tn, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[w] = lo;
    s_hi[w] = hi;
    s_tn[w] = tn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < RNT / 64; ++i) {
      lo = fmin(lo, s_lo[i]);
      hi = fmax(hi, s_hi[i]);
      tn = fmax(tn, s_tn[i]);
    }
    const double pivmin = 1e-100 * fmax(1.0, tn);
    const double pad = 4.4e-16 * fmax(1.0, tn) * double(n) + pivmin;
    sc[0] = lo - pad;
    sc[1] = hi + pad;
    sc[2] = tn;
    sc[3] = pivmin;
    sc[4] = ctol_rel * fmax(1.0, tn);
  }
}

// number of eigenvalues of T below x (LDL^T Sturm sequence with pivot guard).
// d and e2 are the same for every lane.  Whole blocks of SU steps read their
// inputs one block ahead (contiguous uniform loads), so the dependent chain of
// the recurrence does not wait for a load at every step; the last partial
// block loads as it goes.
constexpr int SU = 8;
__device__ __forceinline__ int sturm_count(const double *__restrict__ d,
                                           const double *__restrict__ e2, int64_t n, double x,
                                           double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  auto step = [&](double dk, double ek) {
    q = dk - x - ek * rcp64(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  };
  int64_t k = 1;
  if (k + SU <= n) {
    double dn[SU], en[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      dn[u] = d[k + u];
      en[u] = e2[k - 1 + u];
    }
    for (; k + SU <= n; k += SU) {
      double dc[SU], ec[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        dc[u] = dn[u];
        ec[u] = en[u];
      }
      if (k + 2 * SU <= n) {
        const double *dp = d + k + SU, *ep = e2 + k + SU - 1;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          dn[u] = dp[u];
          en[u] = ep[u];
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) step(dc[u], ec[u]);
    }
  }
  for (; k < n; ++k) step(d[k], e2[k - 1]);
  return cnt;
}

// x_g, g = 0 .. NGRID - 1: the interior points of a uniform grid over the
// Gershgorin interval [sc[0], sc[1]] (the same expression wherever it is used)
__device__ __forceinline__ double grid_x(const double *__restrict__ sc, int g) {
  return sc[0] + (sc[1] - sc[0]) * double(g + 1) / double(NGRID + 1);
}

// Shared first step of the bisection: Sturm counts at the NGRID grid points,
// one thread per point (NGRID / ENT workgroups).
__device__ __forceinline__ void b_bisect_grid(int64_t n, const double *__restrict__ d,
                                              const double *__restrict__ e2,
                                              const double *__restrict__ sc,
                                              int *__restrict__ grid, int wg) {
  const int g = wg * ENT + int(threadIdx.x);
  grid[g] = sturm_count(d, e2, n, grid_x(sc, g), sc[3]);
}

// One wave per eigenvalue index: each pass evaluates 64 Sturm counts at the
// interior points of the current interval (lane l at a + (l+1)(b-a)/65) and
// keeps the sub-interval holding eigenvalue i; ~9 passes reach FP64 resolution
// from the Gershgorin interval.  With grid (the counts of b_bisect_grid) the
// start is the grid cell holding eigenvalue i, found in two ballots over
// 64-entry segments, which saves two passes.
__device__ __forceinline__ void b_bisect(int64_t n, const double *__restrict__ d,
                                                const double *__restrict__ e2,
                                                const double *__restrict__ sc,
                                                const int *__restrict__ grid,
                                                double *__restrict__ omega,
                                                int32_t *__restrict__ status, int wg) {
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(wg) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  double a = sc[0], b = sc[1];
  const double pivmin = sc[3];
  if (grid) {
    // count(x) = eigenvalues below x; the first g with count(x_g) > i gives
    // x_{g-1} <= lambda_i < x_g
    const unsigned long long m1 = __ballot(grid[64 * lane + 63] > i);
    if (m1) {
      const int seg = __builtin_ctzll(m1);
      const unsigned long long m2 = __ballot(grid[64 * seg + lane] > i);
      const int g = 64 * seg + __builtin_ctzll(m2);  // m2 != 0: the segment's last entry is > i
      b = grid_x(sc, g);
      if (g > 0) a = grid_x(sc, g - 1);
    } else {
      a = grid_x(sc, NGRID - 1);
    }
  }
  for (int pass = 0; pass < 24; ++pass) {
    if (b - a <= 2.3e-16 * fmax(fabs(a), fabs(b)) + pivmin) break;
    const double x = a + (b - a) * double(lane + 1) / 65.0;
    const int cnt = sturm_count(d, e2, n, x, pivmin);
    // first lane whose point has more than i eigenvalues below it
    const unsigned long long m = __ballot(cnt > i);
    const int f = m ? __builtin_ctzll(m) : 64;
    const double na = f == 0 ? a : a + (b - a) * double(f) / 65.0;
    const double nb = f == 64 ? b : a + (b - a) * double(f + 1) / 65.0;
    if (!(na > a || nb < b)) break;  // no progress at this resolution
    a = na;
    b = nb;
  }
  const double x = 0.5 * (a + b);
  if (lane == 0) {
    omega[i] = x;
    if (!isfinite(x)) atomicAdd(status + 1, 1);  // no finite eigenvalue (non-finite T)
  }
}

// Weights: a cluster is a maximal run of eigenvalues whose consecutive gaps
// are <= sc[4]; its head (first index) gets the cluster centre as pole and
// beta0^2 times the residue of G(z) = [(z - T)^-1]_00 as strength, the other
// members get zero strength.  One wave per index; lanes are contour nodes.
// The contour is a circle about the centre c of radius sqrt(half g) (half:
// half-width of the cluster, g: distance from c to the nearest eigenvalue
// outside it), which holds the members at a ratio sqrt(half / g) of its
// radius and the neighbours at the same ratio beyond it.  A run whose
// half-width exceeds g / 4 (a dense spectrum, where the gaps of FP32 working
// storage's tolerance chain many distinct eigenvalues) cannot be held apart
// that way; it is split into its runs of gaps within the FP64 resolution,
// each with a contour of its own.
constexpr int NCONT = 64;  // trapezoidal nodes on the circle (32 in the upper half)
__device__ __forceinline__ void b_weights(int64_t n, const double *__restrict__ d,
                                                 const double *__restrict__ e2,
                                                 const double *__restrict__ sc,
                                                 const double *__restrict__ beta0,
                                                 const double *__restrict__ omega,
                                                 double *__restrict__ pole,
                                                 double *__restrict__ osc,
                                                 int32_t *__restrict__ clo, int wg) {
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(wg) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double ctol = sc[4];
  const double li = omega[i];
  // the run of i: consecutive gaps <= ctol, 64 gaps examined per step
  int64_t i0 = i, j = i;
  while (i0 > 0) {
    const int64_t k = i0 - 1 - lane, kc = k < 0 ? 0 : k;  // gap omega[k] .. omega[k + 1]
    const bool brk = k < 0 || omega[kc + 1] - omega[kc] > ctol;
    const unsigned long long m = __ballot(brk);
    if (m) {
      i0 -= __builtin_ctzll(m);
      break;
    }
    i0 -= 64;
  }
  while (j + 1 < n) {
    const int64_t k = j + lane, kc = k + 1 < n ? k : n - 2;
    const bool brk = k + 1 >= n || omega[kc + 1] - omega[kc] > ctol;
    const unsigned long long m = __ballot(brk);
    if (m) {
      j += __builtin_ctzll(m);
      break;
    }
    j += 64;
  }
  double c, half, g;
  auto geometry = [&](int64_t a, int64_t b) {
    c = 0.5 * (omega[a] + omega[b]);
    half = 0.5 * (omega[b] - omega[a]);
    g = 1e300;
    if (a > 0) g = fmin(g, c - omega[a - 1]);
    if (b + 1 < n) g = fmin(g, omega[b + 1] - c);
    if (g > 1e299) g = fmax(1.0, sc[2]);
  };
  geometry(i0, j);
  if (half > 0.25 * g) {
    const double dtol = 8.0 * 2.2e-16 * sqrt(double(n)) * fmax(1.0, sc[2]);
    int64_t a = i, b = i;
    while (a > i0 && omega[a] - omega[a - 1] <= dtol) --a;
    while (b < j && omega[b + 1] - omega[b] <= dtol) ++b;
    i0 = a;
    j = b;
    geometry(i0, j);
  }
  if (clo && lane == 0) clo[i] = int32_t(i0);  // the cluster, for the refinement
  if (i != i0) {
    if (lane == 0) {
      pole[i] = li;
      osc[i] = 0.0;
    }
    return;
  }
  const double rad = sqrt(fmax(half, 1e-6 * g) * g);
  double wsum = 0.0;
  if (lane < NCONT / 2) {
    const double th = 6.283185307179586 * (lane + 0.5) / NCONT;
    const double ct = cos(th), st = sin(th);
    const double zx = c + rad * ct, zy = rad * st;
    // h = z - d_{n-1}; h = z - d_k - e_k^2 / h, k = n-2 .. 0; G = 1 / h
    // (whole blocks of SU steps read their inputs one block ahead, as in
    // sturm_count)
    double hx = zx - d[n - 1], hy = zy;
    auto step = [&](double dk, double ek) {
      const double inv = ek * rcp64(hx * hx + hy * hy);
      hx = zx - dk - hx * inv;
      hy = zy + hy * inv;
    };
    int64_t k = n - 2;
    if (k - SU + 1 >= 0) {
      double dn[SU], en[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        dn[u] = d[k - u];
        en[u] = e2[k - u];
      }
      for (; k - SU + 1 >= 0; k -= SU) {
        double dc[SU], ec[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          dc[u] = dn[u];
          ec[u] = en[u];
        }
        if (k - 2 * SU + 1 >= 0) {
          const double *dp = d + (k - SU), *ep = e2 + (k - SU);
#pragma unroll
          for (int u = 0; u < SU; ++u) {
            dn[u] = dp[-u];
            en[u] = ep[-u];
          }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) step(dc[u], ec[u]);
      }
    }
    for (; k >= 0; --k) step(d[k], e2[k]);
    const double den = rcp64(hx * hx + hy * hy);
    const double gx = hx * den, gy = -hy * den;
    wsum = gx * rad * ct - gy * rad * st;  // Re[G (z - c)]
  }
  wsum = wave_sum(wsum);
  if (lane == 0) {
    pole[i] = c;
    osc[i] = beta0[0] * beta0[0] * wsum * 2.0 / NCONT;
  }
}

static_assert(RB == RB_ROWS, "k_colB rows per workgroup");

// ---------------------------------------------------------------------------
// kernels: single block (descriptor by value, grid = the block's workgroups)
// and batched (descriptor array sorted by n descending; pre[b] is the first
// workgroup of block b in this launch, the active blocks are 0 .. nact-1)
// ---------------------------------------------------------------------------
#define BSE_FIND_BLOCK                                                                    \
  __shared__ int spre[NBMAX + 1];                                                         \
  for (int i_ = threadIdx.x; i_ <= nact; i_ += blockDim.x) spre[i_] = pre[i_];            \
  __syncthreads();                                                                        \
  int lo_ = 0, hi_ = nact;                                                                \
  while (hi_ - lo_ > 1) {                                                                 \
    const int mid_ = (lo_ + hi_) >> 1;                                                    \
    if (spre[mid_] <= int(blockIdx.x)) lo_ = mid_; else hi_ = mid_;                       \
  }                                                                                       \
  const Desc &D = Ds[lo_];                                                                \
  const int wg = int(blockIdx.x) - spre[lo_];

#define BSE_PAIR(NAME, ARGS, ...)                                                         \
  template <typename TH, typename TA, int WPR>                                            \
  __global__ __launch_bounds__(ENT) void k_##NAME(Desc D, ARGS) {                         \
    const int wg = int(blockIdx.x);                                                       \
    __VA_ARGS__                                                                           \
  }                                                                                       \
  template <typename TH, typename TA, int WPR>                                            \
  __global__ __launch_bounds__(ENT) void k_##NAME##_b(const Desc *__restrict__ Ds,        \
                                                      const int *__restrict__ pre,        \
                                                      int nact, ARGS) {                   \
    BSE_FIND_BLOCK                                                                        \
    __VA_ARGS__                                                                           \
  }

#define BSE_COMMA ,
BSE_PAIR(copy_in, int unused_, {
  (void)unused_;
  const int64_t gx = g_copy_gx(D.n);
  b_copy_in<TH, TA>(D.n, (const TH *)D.H, D.ld, (TA *)D.A, D.lda, wg / gx, wg % gx, gx);
})
BSE_PAIR(load_b, int unused_, {
  (void)unused_;
  b_load_b(D.n, D.B, D.col, D.part3, wg, (int)g_nwg(D.n));
})
BSE_PAIR(hemv0, int unused_, {
  (void)unused_;
  b_hemv0<TA>(D.n, g_rpw(D.n), (const TA *)D.A, D.lda, D.col, D.part3, (int)g_nwg(D.n),
              D.beta0, D.tau, D.vbuf, D.y, wg);
})
BSE_PAIR(w0, int unused_, {
  (void)unused_;
  b_w0(D.n, D.y, D.vbuf, D.tau, D.wraw, D.part2, wg);
})
BSE_PAIR(rank2, int unused_, {
  (void)unused_;
  const int64_t gx = g_rank2_gx(D.n);
  b_rank2<TA>(D.n, (TA *)D.A, D.lda, D.wraw, D.vbuf, D.part2, (int)g_nwg(D.n), D.tau, wg / gx,
              wg % gx, gx);
})
BSE_PAIR(col0, int64_t j0 BSE_COMMA int cur, {
  b_col0<TA>(D.n, j0, (const TA *)D.A, D.lda, D.col, cur ? D.partb1 : D.partb0, wg);
})
BSE_PAIR(colA, int64_t jn BSE_COMMA int cur, {
  if constexpr (WPR < 0) {
      b_colA_tile<TA, tile_of(WPR)>(D.n, jn, int(jn % NBK), (const TA *)D.A, D.lda, D.V, D.ldv,
                                D.col, cur ? D.partb1 : D.partb0, g_np_in(D.n, jn), D.tau, D.scl,
                                D.d, D.e, D.ys, D.ldys, D.parta, D.bred, wg);
  } else if constexpr (WPR == 0)
    b_colA_lds<TA>(D.n, jn, int(jn % NBK), (const TA *)D.A, D.lda, D.V, D.ldv, D.col,
                   cur ? D.partb1 : D.partb0, g_np_in(D.n, jn), D.tau, D.scl, D.d, D.e, D.y,
                   D.parta, D.bred, wg);
  else
    b_colA<TA, WPR>(D.n, jn, int(jn % NBK), (const TA *)D.A, D.lda, D.V, D.ldv, D.col,
                    cur ? D.partb1 : D.partb0, g_np_in(D.n, jn), D.tau, D.scl, D.d, D.e, D.y,
                    D.parta, D.bred, wg);
})
BSE_PAIR(colB, int64_t jn BSE_COMMA int cur, {
  const int64_t m = D.n - jn - 1;
  int npa, nbt = 0;  // partial sums of y^dag v; slots of y (tile forms)
  if constexpr (WPR < 0) {
    npa = (int)g_tiles(D.n, jn + 1, tile_of(WPR));
    nbt = (int)g_tblocks(D.n, jn + 1, tile_of(WPR));
  } else {
    npa = g_colA_wgs(m, WPR);
  }
  b_colB<TA>(D.n, jn, int(jn % NBK), g_more(D.n, jn), (const TA *)D.A, D.lda, D.V, D.W, D.ldv,
             D.y, D.ys, D.ldys, nbt, D.parta, npa, D.bred, D.tau, D.scl, D.col,
             cur ? D.partb0 : D.partb1, wg);
})
// trailing update of one workgroup: tile S; every tile below HER_TRI_M
// trailing rows, else the lower ones row by row: wg = by (by + 1) / 2 + bx
template <typename TA, int S>
__device__ __forceinline__ void her2k_wg(const Desc &D, int64_t j0, int wg) {
  constexpr int BN = HerTile<TA, S>::BN;
  const int nbk = g_nbk(D.n, j0);
  const int64_t c0 = j0 + nbk, t = cdiv(D.n - c0, BN);
  if (!her_tri(t, BN)) {
    b_her2k<TA, S>(D.n, c0, nbk, D.V, D.W, D.ldv, (TA *)D.A, D.lda, wg % t, wg / t, false);
  } else {
    int64_t by = int64_t((sqrt(8.0 * double(wg) + 1.0) - 1.0) * 0.5);
    while (by * (by + 1) / 2 > wg) --by;
    while ((by + 1) * (by + 2) / 2 <= wg) ++by;
    const int64_t bx = wg - by * (by + 1) / 2;
    b_her2k<TA, S>(D.n, c0, nbk, D.V, D.W, D.ldv, (TA *)D.A, D.lda, bx, by, true);
  }
}
template <typename TH, typename TA, int S>
__global__ __launch_bounds__(ENT) void k_her2k(Desc D, int64_t j0) {
  her2k_wg<TA, S>(D, j0, int(blockIdx.x));
}
template <typename TH, typename TA, int S>
__global__ __launch_bounds__(ENT) void k_her2k_b(const Desc *__restrict__ Ds,
                                                 const int *__restrict__ pre, int nact,
                                                 int64_t j0) {
  BSE_FIND_BLOCK
  her2k_wg<TA, S>(D, j0, wg);
}
BSE_PAIR(bisect_grid, int unused_, {
  (void)unused_;
  b_bisect_grid(D.n, D.d, D.e2, D.tsc, D.bgrid, wg);
})
BSE_PAIR(bisect, int use_grid, {
  b_bisect(D.n, D.d, D.e2, D.tsc, use_grid ? D.bgrid : nullptr, D.omega, D.status, wg);
})
BSE_PAIR(weights, int unused_, {
  (void)unused_;
  b_weights(D.n, D.d, D.e2, D.tsc, D.beta0, D.omega, D.pole, D.osc, D.K > 0 ? D.clo : nullptr, wg);
})
#undef BSE_PAIR

// ---------------------------------------------------------------------------
// k_tail: the last columns of the reduction in one workgroup.  From a panel
// boundary j0 with at most MT trailing rows (all earlier updates applied),
// the trailing block is held in LDS in FP64 and reduced by unblocked
// Householder steps (LAPACK zhetd2, lower form): reflector of column j from
// |x|^2, w = tau A22 v, alpha = -tau (w^dag v) / 2, w += alpha v,
// A22 -= v w^dag + w v^dag.  Same reflector convention and outputs (d, e,
// tau, scl and, with refinement, every reflector) as the blocked columns, so
// the result is the same tridiagonal up to rounding; each column costs a few
// workgroup barriers instead of two dependent kernel launches.
// ---------------------------------------------------------------------------
template <typename TA>
__device__ __forceinline__ void b_tail(const Desc &D, int64_t j0, int keep) {
  typedef typename C2T<TA>::t CA;
  constexpr int NWT = TNT / 64;
  __shared__ double2 As[MT * MT];
  __shared__ double2 part[NWT * MT];  // partial A22 v of each wave's column chunk
  __shared__ double2 wv_[MT];         // w of the current step
  __shared__ double2 dpart[NWT];      // per wave: sum_r conj(partial y_r) v_r
  __shared__ double npart[NWT];       // per wave: |x|^2 of the next column
  __shared__ double red[TNT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = D.n, lda = D.lda, ldv = D.ldv;
  const int mt = int(n - j0);  // 1 <= mt <= MT: j0 = g_tail0(n)
  const CA *A = reinterpret_cast<const CA *>(D.A);
  for (int q = tid; q < mt * mt; q += TNT) {
    const int r = q / mt, c = q % mt;
    As[r * MT + c] = to_d2(A[(j0 + r) * lda + j0 + c]);
  }
  __syncthreads();
  double x2 = 0;  // |x|^2 of the current column below its subdiagonal entry
  for (int r = 2 + tid; r < mt; r += TNT) {
    const double2 a = As[r * MT];
    x2 += a.x * a.x + a.y * a.y;
  }
  x2 = block_sum<TNT>(x2, red);
  // Three barriers per column.  v is never stored: v[c] = 1 at c = j + 1 and
  // scale A[c][j] below, read from column j, which the later steps leave
  // unchanged.  Thread j keeps the scalars of column j; nothing goes to
  // global memory inside the loop (a barrier would wait for such a store).
  double my_d = 0, my_e = 0;
  double2 my_tau = {0, 0}, my_sc = {0, 0};
  for (int j = 0; j < mt; ++j) {
    if (tid == j) my_d = As[j * MT + j].x;
    if (j == mt - 1) break;
    double beta;
    double2 tj, sc;
    householder(As[(j + 1) * MT + j], x2, beta, tj, sc);
    if (tid == j) {
      my_e = beta;
      my_tau = tj;
      my_sc = sc;
    }
    auto vof = [&](int c) { return c == j + 1 ? double2{1, 0} : cmul(sc, As[c * MT + j]); };
    // y = A22 v.  A22 is Hermitian, y[r] = sum_c conj(A[c][r]) v[c]: wave w
    // sums its chunk of columns c for every row (lane: rows r0 and r0 + 64,
    // contiguous in LDS; A[c][j] read as a broadcast), and its share of
    // y^dag v; the partials are added below in a fixed order.
    {
      const int cs = (mt - j - 1 + NWT - 1) / NWT;
      const int cb = j + 1 + wv * cs, ce = std::min(cb + cs, mt);
      const int r0 = j + 1 + lane, r1 = r0 + 64;
      double2 p0 = {0, 0}, p1 = {0, 0};
      for (int c = cb; c < ce; ++c) {
        const double2 v = vof(c);
        if (r0 < mt) p0 = cadd(p0, cmulc(As[c * MT + r0], v));
        if (r1 < mt) p1 = cadd(p1, cmulc(As[c * MT + r1], v));
      }
      double dr = 0, di = 0;
      if (r0 < mt) {
        part[wv * MT + r0] = p0;
        const double2 t = cmulc(p0, vof(r0));
        dr += t.x;
        di += t.y;
      }
      if (r1 < mt) {
        part[wv * MT + r1] = p1;
        const double2 t = cmulc(p1, vof(r1));
        dr += t.x;
        di += t.y;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      if (lane == 0) dpart[wv] = double2{dr, di};
    }
    __syncthreads();
    // w = tau y + alpha v, alpha = -tau (w_raw^dag v) / 2, w_raw^dag v = conj(tau) y^dag v
    double2 ydv = {0, 0};
#pragma unroll
    for (int q = 0; q < NWT; ++q) ydv = cadd(ydv, dpart[q]);
    const double2 alpha = cmul(double2{-0.5 * tj.x, -0.5 * tj.y}, cmulc(tj, ydv));
    for (int r = j + 1 + tid; r < mt; r += TNT) {
      double2 y = {0, 0};
#pragma unroll
      for (int q = 0; q < NWT; ++q) y = cadd(y, part[q * MT + r]);
      wv_[r] = cadd(cmul(tj, y), cmul(alpha, vof(r)));
    }
    __syncthreads();
    // A22 -= v w^dag + w v^dag: one wave per row, each lane owning columns c0
    // and c0 + 64; lane 0 owns column j + 1 and sums |x|^2 of the next step
    const int c0 = j + 1 + lane, c1 = c0 + 64;
    const double2 vc0 = c0 < mt ? vof(c0) : double2{0, 0};
    const double2 vc1 = c1 < mt ? vof(c1) : double2{0, 0};
    const double2 wc0 = c0 < mt ? wv_[c0] : double2{0, 0};
    const double2 wc1 = c1 < mt ? wv_[c1] : double2{0, 0};
    double xn = 0;
    for (int r = j + 1 + wv; r < mt; r += NWT) {
      const double2 vr = vof(r), wr = wv_[r];
      if (c0 < mt) {
        const double2 a =
            csub(As[r * MT + c0], cadd(cmul(vr, cconj(wc0)), cmul(wr, cconj(vc0))));
        As[r * MT + c0] = a;
        if (lane == 0 && r >= j + 3) xn += a.x * a.x + a.y * a.y;
      }
      if (c1 < mt)
        As[r * MT + c1] = csub(As[r * MT + c1], cadd(cmul(vr, cconj(wc1)), cmul(wr, cconj(vc1))));
    }
    if (lane == 0) npart[wv] = xn;
    __syncthreads();
    x2 = 0;
#pragma unroll
    for (int q = 0; q < NWT; ++q) x2 += npart[q];
  }
  // outputs of column tid (indices of the whole block)
  const int64_t jn = j0 + tid;
  if (tid < mt) D.d[jn] = my_d;
  if (tid < mt - 1) {
    D.e[jn] = my_e;
    D.tau[jn + 1] = my_tau;
    D.scl[jn + 1] = my_sc;
    if (keep)
      for (int r = tid + 1; r < mt; ++r)
        D.Vall[jn * ldv + j0 + r] = r == tid + 1 ? double2{1, 0} : cmul(my_sc, As[r * MT + tid]);
  }
}

template <typename TA>
__global__ __launch_bounds__(TNT) void k_tail(Desc D, int64_t j0, int keep) {
  b_tail<TA>(D, j0, keep);
}
// batched: one workgroup per block of Ds[b0 ..), each from its own tail start
template <typename TA>
__global__ __launch_bounds__(TNT) void k_tail_b(const Desc *__restrict__ Ds, int b0, int64_t unused_) {
  (void)unused_;
  const Desc &D = Ds[b0 + int(blockIdx.x)];
  b_tail<TA>(D, g_tail0(D.n), 0);
}

// the tridiagonal preparation runs one RNT-thread workgroup per block
template <typename TA>
__global__ __launch_bounds__(RNT) void k_tri_prep(Desc D, double ctol) {
  b_tri_prep(D.n, D.d, D.e, ctol, D.e2, D.tsc, D.status);
}
template <typename TA>
__global__ __launch_bounds__(RNT) void k_tri_prep_b(const Desc *__restrict__ Ds,
                                                   const int *__restrict__ pre, int nact,
                                                   int unused_) {
  (void)unused_;
  BSE_FIND_BLOCK
  (void)wg;
  b_tri_prep(D.n, D.d, D.e, ctol_rel(D.n, sizeof(TA) == 8), D.e2, D.tsc, D.status);
}


// ---------------------------------------------------------------------------
// refinement of the lowest K eigenvalues against the stored H_mu (FP64)
//   k_invit   eigenvectors z of T by inverse iteration (3 steps) for each of
//             the lowest K eigenvalues; the members of a cluster of
//             (numerically) degenerate eigenvalues start from distinct
//             vectors and are orthogonalised in order, so a cluster gets an
//             orthonormal basis of its invariant subspace
//   k_backxf  x = Q0 H(0) H(1) ... H(n-2) z, applying the stored reflectors
//             a panel at a time (block form below)
//   k_hx_part partial sums of x^dag H_mu x and |x|^2 (HXR rows, HXV vectors)
//   k_rq_fin  theta = Re(x^dag H_mu x) / |x|^2 replaces omega[l]; the pole of
//             a cluster inside the refined range becomes the mean of its members
// The Rayleigh quotient of an approximate eigenvector with error delta is
// exact to O(delta^2 |H_mu|), so rounding of the eigensolver itself (FP32
// storage of the working copy) is removed; errors of H_mu are not.
// ---------------------------------------------------------------------------
// (T - sigma) x = rhs for symmetric tridiagonal T (diag d, off-diag e) by
// Gaussian elimination with partial pivoting (rows i and i + 1), one thread.
// The running diagonal and superdiagonal entries are carried in registers and
// the read-only inputs are fetched TCH entries ahead of their use, so the
// serial chain waits on arithmetic rather than on memory.  Stored factors:
// ddi[i] = 1 / pivot_i, du[i], du2[i] (second superdiagonal from an
// interchange), dl[i] (multiplier), piv[i] = 1 if rows i, i + 1 were swapped.
constexpr int TCH = 16;
__device__ void tri_solve(int64_t n, const double *__restrict__ d, const double *__restrict__ e,
                          double sigma, double tiny, double *__restrict__ ddi,
                          double *__restrict__ du, double *__restrict__ du2,
                          double *__restrict__ dl, double *__restrict__ piv) {
  double cd = d[0] - sigma;         // current diagonal entry of row i
  double cu = n > 1 ? e[0] : 0.0;   // current superdiagonal entry of row i
  for (int64_t i0 = 0; i0 + 1 < n; i0 += TCH) {
    double dn[TCH], en[TCH], eu[TCH];
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 + k;
      const int64_t i1 = std::min<int64_t>(i + 1, n - 1), i0c = std::min<int64_t>(i, n - 2);
      const int64_t i2 = std::min<int64_t>(i + 1, n - 2);
      dn[k] = d[i1] - sigma;
      en[k] = e[i0c];
      eu[k] = i + 2 < n ? e[i2] : 0.0;  // select on a loaded value
    }
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 + k;
      if (i + 1 >= n) break;
      const double bl = en[k];
      if (fabs(cd) >= fabs(bl)) {
        const double pv = fabs(cd) < tiny ? (cd < 0 ? -tiny : tiny) : cd;
        const double ip = 1.0 / pv, f = bl * ip;
        ddi[i] = ip;
        dl[i] = f;
        du[i] = cu;
        du2[i] = 0.0;
        piv[i] = 0.0;
        cd = dn[k] - f * cu;
        cu = eu[k];
      } else {
        const double ib = 1.0 / bl, f = cd * ib;
        ddi[i] = ib;
        dl[i] = f;
        du[i] = dn[k];
        du2[i] = eu[k];
        piv[i] = 1.0;
        cd = cu - f * dn[k];
        cu = -f * eu[k];
      }
    }
  }
  if (fabs(cd) < tiny) cd = cd < 0 ? -tiny : tiny;
  ddi[n - 1] = 1.0 / cd;
}

// solves with the factors of tri_solve; b holds the right-hand side on entry
// and the solution on exit
__device__ void tri_apply(int64_t n, const double *__restrict__ ddi,
                          const double *__restrict__ du, const double *__restrict__ du2,
                          const double *__restrict__ dl, const double *__restrict__ piv,
                          double *__restrict__ b) {
  double cb = b[0];
  for (int64_t i0 = 0; i0 + 1 < n; i0 += TCH) {
    double bn[TCH], l[TCH], pv[TCH];
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 + k;
      const int64_t i1 = std::min<int64_t>(i + 1, n - 1), ic = std::min<int64_t>(i, n - 2);
      bn[k] = b[i1];
      l[k] = dl[ic];
      pv[k] = piv[ic];
    }
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 + k;
      if (i + 1 >= n) break;
      if (pv[k] == 0.0) {
        b[i] = cb;
        cb = bn[k] - l[k] * cb;
      } else {
        b[i] = bn[k];
        cb = cb - l[k] * bn[k];
      }
    }
  }
  double x1 = cb * ddi[n - 1];  // b[n - 1]
  b[n - 1] = x1;
  if (n < 2) return;
  double x0 = (b[n - 2] - du[n - 2] * x1) * ddi[n - 2];
  b[n - 2] = x0;
  for (int64_t i0 = n - 3; i0 >= 0; i0 -= TCH) {
    double bb[TCH], u1[TCH], u2[TCH], q[TCH];
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 - k;
      const int64_t ic = i >= 0 ? i : 0;
      bb[k] = b[ic];
      u1[k] = du[ic];
      u2[k] = du2[ic];
      q[k] = ddi[ic];
    }
#pragma unroll
    for (int k = 0; k < TCH; ++k) {
      const int64_t i = i0 - k;
      if (i < 0) break;
      const double xi = (bb[k] - u1[k] * x0 - u2[k] * x1) * q[k];
      b[i] = xi;
      x1 = x0;
      x0 = xi;
    }
  }
}

// The members of a cluster are iterated together: each inverse-iteration
// step solves every member's system at once (one serial solver per wave,
// each with its own shift), then orthonormalises the members in order
// (Gram-Schmidt over the cluster).  Workgroup l returns member m = l - head.
constexpr int INV_IT = 3;  // inverse-iteration steps
__global__ __launch_bounds__(ENT) void k_invit(Desc D) {
  __shared__ double sh[ENT / 64];
  const int64_t n = D.n, l = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double tn = D.tsc[2];
  const double *om = D.omega;
  const int64_t i = D.clo[l];  // l's cluster as the weights formed it
  const int64_t m = l - i;     // member index of l in its cluster
  double *scr = D.scr + size_t(l) * (6 * CMAX) * n;
  double *mem = scr + 5 * CMAX * n;  // [CMAX][n] member vectors
  double *z = D.Z + size_t(l) * n;
  if (m >= CMAX) {  // cluster too large to refine: mark, omega[l] stays
    for (int64_t k = tid; k < n; k += ENT) z[k] = __builtin_nan("");
    return;
  }
  const double tiny = 2.2e-16 * fmax(1.0, tn);
  auto fac = [&](int64_t q, int f) { return scr + (5 * q + f) * n; };  // ddi du du2 dl piv
  for (int64_t q = wv; q <= m; q += ENT / 64)
    if (lane == 0) tri_solve(n, D.d, D.e, om[i + q], tiny, fac(q, 0), fac(q, 1), fac(q, 2), fac(q, 3),
                             fac(q, 4));
  for (int64_t q = 0; q <= m; ++q) {
    double *v = mem + q * n;
    for (int64_t k = tid; k < n; k += ENT) v[k] = 1.0 + 0.5 * sin(0.7 * double(k + 1) * double(q + 1));
  }
  __syncthreads();
  for (int it = 0; it < INV_IT; ++it) {
    for (int64_t q = wv; q <= m; q += ENT / 64)
      if (lane == 0) tri_apply(n, fac(q, 0), fac(q, 1), fac(q, 2), fac(q, 3), fac(q, 4), mem + q * n);
    __syncthreads();
    for (int64_t q = 0; q <= m; ++q) {  // modified Gram-Schmidt over the members, in order
      double *v = mem + q * n;
      for (int64_t p = 0; p < q; ++p) {
        const double *u = mem + p * n;
        double dot = 0;
        for (int64_t k = tid; k < n; k += ENT) dot += u[k] * v[k];
        dot = block_sum<ENT>(dot, sh);
        for (int64_t k = tid; k < n; k += ENT) v[k] -= dot * u[k];
        __syncthreads();
      }
      double s2 = 0;
      for (int64_t k = tid; k < n; k += ENT) s2 += v[k] * v[k];
      s2 = block_sum<ENT>(s2, sh);
      const double inv = s2 > 0 ? 1.0 / sqrt(s2) : 0.0;
      for (int64_t k = tid; k < n; k += ENT) v[k] *= inv;
      __syncthreads();
    }
  }
  const double *v = mem + m * n;
  for (int64_t k = tid; k < n; k += ENT) z[k] = v[k];
}

// Block form of the back-transformation.  The reflectors of columns
// j0 .. j0 + b - 1 (one panel, b <= NBK) multiply as
//     H(j0) H(j0 + 1) ... H(j0 + b - 1) = I - V T V^dag
// with T upper triangular: T[i][i] = tau_i and
//     T[0:i, i] = -tau_i T[0:i, 0:i] (V[:, 0:i]^dag v_i)
// (the forward, column-wise accumulation of the compact WY form).
//   k_bx_tmat     one workgroup per panel: the Gram products v_k^dag v_i
//                 (k < i) over LDS-staged row chunks, then T
//   k_backxf      one workgroup per vector, panels from the last to the
//                 first: w = V^dag x (one block reduction per panel), t = T w,
//                 x -= V t; then the initial reflection.  Each thread owns
//                 the rows tid + ENT q of x throughout.
constexpr int BXR = 128;  // rows of a panel staged per chunk in k_bx_tmat

__global__ __launch_bounds__(ENT) void k_bx_tmat(Desc D) {
  constexpr int NP = NBK * (NBK - 1) / 2;  // pairs k < i
  __shared__ double2 vs[BXR][NBK];
  __shared__ double2 gs[NBK][NBK];
  __shared__ double2 ts[NBK][NBK];
  __shared__ unsigned char pk[NP], pi[NP];
  const int64_t n = D.n, ldv = D.ldv;
  const int tid = threadIdx.x;
  const int64_t j0 = int64_t(blockIdx.x) * NBK;
  const int bp = int(std::min<int64_t>(NBK, n - 1 - j0));
  for (int q = tid; q < NP; q += ENT) {
    int i = 1;
    while ((i + 1) * i / 2 <= q) ++i;
    pi[q] = (unsigned char)i;
    pk[q] = (unsigned char)(q - i * (i - 1) / 2);
  }
  for (int q = tid; q < NBK * NBK; q += ENT) ts[q / NBK][q % NBK] = double2{0, 0};
  __syncthreads();
  double2 acc[(NP + ENT - 1) / ENT];
#pragma unroll
  for (int u = 0; u < (NP + ENT - 1) / ENT; ++u) acc[u] = double2{0, 0};
  for (int64_t r0 = j0 + 1; r0 < n; r0 += BXR) {
    __syncthreads();
    for (int q = tid; q < BXR * NBK; q += ENT) {
      const int rr = q % BXR, c = q / BXR;
      const int64_t row = r0 + rr;
      vs[rr][c] = (c < bp && row < n && row >= j0 + c + 1) ? D.Vall[(j0 + c) * ldv + row]
                                                           : double2{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (NP + ENT - 1) / ENT; ++u) {
      const int q = tid + ENT * u;
      if (q < NP) {
        const int k = pk[q], i = pi[q];
        double2 a = acc[u];
        for (int rr = 0; rr < BXR; ++rr) a = cadd(a, cmulc(vs[rr][k], vs[rr][i]));
        acc[u] = a;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < (NP + ENT - 1) / ENT; ++u) {
    const int q = tid + ENT * u;
    if (q < NP) gs[pk[q]][pi[q]] = acc[u];
  }
  __syncthreads();
  for (int i = 0; i < bp; ++i) {
    const double2 ti = D.tau[j0 + i + 1];
    if (tid < i) {
      double2 sacc = {0, 0};
      for (int m = tid; m < i; ++m) sacc = cadd(sacc, cmul(ts[tid][m], gs[m][i]));
      ts[tid][i] = cmul(double2{-ti.x, -ti.y}, sacc);
    }
    if (tid == i) ts[i][i] = ti;
    __syncthreads();
  }
  double2 *T = D.Tm + size_t(blockIdx.x) * NBK * NBK;
  for (int q = tid; q < NBK * NBK; q += ENT) T[q] = ts[q / NBK][q % NBK];
}

__global__ __launch_bounds__(ENT) void k_backxf(Desc D) {
  __shared__ double sh[ENT / 64];
  __shared__ double2 sw[ENT / 64][NBK];
  __shared__ double2 st[NBK];
  const int64_t n = D.n, ldv = D.ldv, l = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double *z = D.Z + size_t(l) * n;
  double2 *x = D.X + size_t(l) * n;
  for (int64_t k = tid; k < n; k += ENT) x[k] = double2{z[k], 0.0};
  const int64_t npan = n >= 2 ? cdiv(n - 1, NBK) : 0;
  for (int64_t p = npan - 1; p >= 0; --p) {
    const int64_t j0 = p * NBK;
    const int bp = int(std::min<int64_t>(NBK, n - 1 - j0));
    const double2 *V = D.Vall + j0 * ldv;
    const double2 *T = D.Tm + size_t(p) * NBK * NBK;
    // w = V^dag x over the panel's rows (v_c is zero above row j0 + c + 1)
    double2 w[NBK];
#pragma unroll
    for (int c = 0; c < NBK; ++c) w[c] = double2{0, 0};
    // every load is unconditional (column index clamped in bounds) and the
    // support mask is applied to the value, so the loads of a row overlap
    for (int64_t r = (j0 + 1) / ENT * ENT + tid; r < n; r += ENT) {
      if (r < j0 + 1) continue;
      const double2 xr = x[r];
      double2 vr[NBK];
#pragma unroll
      for (int c = 0; c < NBK; ++c) vr[c] = V[std::min(c, bp - 1) * ldv + r];
#pragma unroll
      for (int c = 0; c < NBK; ++c) {
        const double2 t = cmulc(vr[c], xr);
        const bool ok = c < bp && r >= j0 + c + 1;
        w[c].x += ok ? t.x : 0.0;
        w[c].y += ok ? t.y : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < NBK; ++c) {
      w[c].x = wave_sum(w[c].x);
      w[c].y = wave_sum(w[c].y);
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < NBK; ++c) sw[wv][c] = w[c];
    }
    __syncthreads();
    if (tid < bp) {  // t = T w (T upper triangular)
      double2 tc = {0, 0};
      for (int m = tid; m < bp; ++m) {
        double2 wm = sw[0][m];
        for (int q = 1; q < ENT / 64; ++q) wm = cadd(wm, sw[q][m]);
        tc = cadd(tc, cmul(T[tid * NBK + m], wm));
      }
      st[tid] = tc;
    }
    __syncthreads();
    double2 tc[NBK];
#pragma unroll
    for (int c = 0; c < NBK; ++c) tc[c] = st[c];
    for (int64_t r = (j0 + 1) / ENT * ENT + tid; r < n; r += ENT) {
      if (r < j0 + 1) continue;
      double2 xr = x[r];
      double2 vr[NBK];
#pragma unroll
      for (int c = 0; c < NBK; ++c) vr[c] = V[std::min(c, bp - 1) * ldv + r];
#pragma unroll
      for (int c = 0; c < NBK; ++c) {
        const double2 t = cmul(vr[c], tc[c]);
        const bool ok = c < bp && r >= j0 + c + 1;
        xr.x -= ok ? t.x : 0.0;
        xr.y -= ok ? t.y : 0.0;
      }
      x[r] = xr;
    }
    __syncthreads();
  }
  {  // the initial reflection (rows 0 ..)
    const double2 *v = D.vbuf;
    const double2 t = D.tau[0];
    double sr = 0, si = 0;
    for (int64_t r = tid; r < n; r += ENT) {
      const double2 c = cmulc(v[r], x[r]);
      sr += c.x;
      si += c.y;
    }
    sr = block_sum<ENT>(sr, sh);
    si = block_sum<ENT>(si, sh);
    const double2 f = cmul(t, double2{sr, si});
    for (int64_t r = tid; r < n; r += ENT) x[r] = csub(x[r], cmul(f, v[r]));
  }
}

// Back-transformation through the stage-1 panels of the two-stage reduction
// (refinement): x -= V T (V^dag x) for the panels from the last to the first,
// then the initial reflection.  Per panel two launches over (row blocks of
// BPR rows) x (groups of BPV vectors), so every compute unit takes part and
// the panel's reflectors are read once per launch for BPV vectors:
//   k_bp_part   partial w = V^dag x over the block's rows (the block's x
//               staged in LDS; thread (c, g): column c, rows g, g + 8, ...;
//               the eight row groups of a column summed by xor shuffles)
//   k_bp_apply  w summed over the blocks, s = T w, x -= V s over the block's
//               rows (one row per thread at a time)
// The panel's reflector c is stored with its zeros and unit entry over the
// panel's m rows (column c of [SBW][m]), and T is upper triangular.
__global__ __launch_bounds__(ENT) void k_bp_part(Desc D, int64_t p) {
  static_assert(ENT == SBW * 8, "k_bp_part: eight row groups per column");
  constexpr int U = 8;  // rows of a thread with their loads in flight together
  static_assert(BPR % (8 * U) == 0, "k_bp_part: whole rounds of rows");
  __shared__ double2 xs[BPV][BPR];  // the block's rows of the group's vectors
  const int64_t n = D.n, K = D.K, j0 = p * SBW, p0 = j0 + SBW, m = n - p0;
  const int64_t rb = int64_t(blockIdx.x) * BPR, l0 = int64_t(blockIdx.y) * BPV;
  const int64_t rend = std::min<int64_t>(rb + BPR, m);
  const int tid = threadIdx.x, c = tid / 8, g = tid % 8;
  // rows past the block (or past m) are staged as zeros and read from its last row
#pragma unroll
  for (int u = 0; u < BPV * BPR / ENT; ++u) {
    const int e = tid + ENT * u, v = e / BPR, rr = e % BPR;
    const double2 *x = D.X + size_t(std::min<int64_t>(l0 + v, K - 1)) * n + p0;
    const double2 xv = x[std::min<int64_t>(rb + rr, rend - 1)];
    xs[v][rr] = csel(rb + rr < rend, xv, double2{0, 0});
  }
  __syncthreads();
  const double2 *V = D.vrow + g_sb_voff(n, p) * SBW + c * m;
  double2 w[BPV];
#pragma unroll
  for (int v = 0; v < BPV; ++v) w[v] = double2{0, 0};
  for (int r0 = g; r0 < BPR; r0 += 8 * U) {
    double2 vr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) vr[u] = V[std::min<int64_t>(rb + r0 + 8 * u, rend - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < BPV; ++v) w[v] = cadd(w[v], cmulc(vr[u], xs[v][r0 + 8 * u]));
  }
#pragma unroll
  for (int v = 0; v < BPV; ++v)
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      w[v].x += __shfl_xor(w[v].x, o, 64);
      w[v].y += __shfl_xor(w[v].y, o, 64);
    }
  if (g == 0) {
#pragma unroll
    for (int v = 0; v < BPV; ++v)
      if (l0 + v < K) D.bxw[(size_t(blockIdx.x) * K + l0 + v) * SBW + c] = w[v];
  }
}

constexpr int BPT = 512;  // threads of k_bp_apply: one block row each
__global__ __launch_bounds__(BPT) void k_bp_apply(Desc D, int64_t p) {
  __shared__ double2 ws_[BPV][SBW], ss[SBW][BPV], Ts[SBW][SBW + 1];
  const int64_t n = D.n, K = D.K, j0 = p * SBW, p0 = j0 + SBW, m = n - p0;
  const int64_t rb = int64_t(blockIdx.x) * BPR, l0 = int64_t(blockIdx.y) * BPV;
  const int64_t nb = cdiv(m, BPR);
  const int tid = threadIdx.x;
  {  // the panel's T into LDS, its loads in flight with the partial sums below
    const double2 *T = D.Tm + size_t(p) * SBW * SBW;
#pragma unroll
    for (int u = 0; u < SBW * SBW / BPT; ++u) {
      const int e = tid + BPT * u;
      Ts[e / SBW][e % SBW] = T[e];
    }
  }
  if (tid < BPV * SBW) {  // w of vector v, entry c: the sum over the row blocks
    const int v = tid / SBW, c = tid % SBW;
    const int64_t l = std::min<int64_t>(l0 + v, K - 1);
    double2 a = {0, 0};
    for (int64_t b0 = 0; b0 < nb; b0 += 8) {  // eight loads in flight
      double2 t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        t[u] = D.bxw[(size_t(std::min<int64_t>(b0 + u, nb - 1)) * K + l) * SBW + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) a = cadd(a, csel(b0 + u < nb, t[u], double2{0, 0}));
    }
    ws_[v][c] = a;
  }
  __syncthreads();
  if (tid < BPV * SBW) {  // s = T w (T upper triangular)
    const int v = tid / SBW, c = tid % SBW;
    double2 a = {0, 0};
    for (int e = c; e < SBW; ++e) a = cadd(a, cmul(Ts[c][e], ws_[v][e]));
    ss[c][v] = a;
  }
  __syncthreads();
  const double2 *V = D.vrow + g_sb_voff(n, p) * SBW;
  double2 *x[BPV];
#pragma unroll
  for (int v = 0; v < BPV; ++v) x[v] = D.X + size_t(std::min<int64_t>(l0 + v, K - 1)) * n + p0;
  const int64_t rend = std::min<int64_t>(rb + BPR, m);
  for (int64_t r = rb + tid; r < rend; r += BPT) {
    double2 a[BPV];
#pragma unroll
    for (int v = 0; v < BPV; ++v) a[v] = double2{0, 0};
#pragma unroll 8
    for (int c = 0; c < SBW; ++c) {
      const double2 vr = V[c * m + r];
#pragma unroll
      for (int v = 0; v < BPV; ++v) a[v] = cadd(a[v], cmul(vr, ss[c][v]));
    }
#pragma unroll
    for (int v = 0; v < BPV; ++v)
      if (l0 + v < K) x[v][r] = csub(x[v][r], a[v]);
  }
}

// the initial reflection of each back-transformed vector (one workgroup per vector)
__global__ __launch_bounds__(ENT) void k_bx_q0(Desc D) {
  __shared__ double sh[ENT / 64];
  const int64_t n = D.n, l = blockIdx.x;
  const int tid = threadIdx.x;
  double2 *x = D.X + size_t(l) * n;
  const double2 *v = D.vbuf;
  const double2 t = D.tau[0];
  double sr = 0, si = 0;
  for (int64_t r = tid; r < n; r += ENT) {
    const double2 c = cmulc(v[r], x[r]);
    sr += c.x;
    si += c.y;
  }
  sr = block_sum<ENT>(sr, sh);
  si = block_sum<ENT>(si, sh);
  const double2 f = cmul(t, double2{sr, si});
  for (int64_t r = tid; r < n; r += ENT) x[r] = csub(x[r], cmul(f, v[r]));
}

// partial sums of x^dag H_mu x and |x|^2 over HXR rows for HXV vectors per
// workgroup: grid (cdiv(n, HXR), cdiv(K, HXV)).  Wave w takes rows
// HXR bx + 4 w .. + 3; each H_mu entry read serves HXV vectors and each x
// entry four rows, so H_mu is read K / HXV times instead of K times.  Rows
// past n and vectors past K read row n - 1 and vector K - 1 and are dropped.
template <typename TH>
__global__ __launch_bounds__(ENT) void k_hx_part(Desc D) {
  typedef typename C2T<TH>::t CH;
  constexpr int RW = HXR / (ENT / 64);  // rows per wave
  static_assert(RW * (ENT / 64) == HXR, "k_hx_part: rows split evenly over the waves");
  __shared__ double sh[ENT / 64][HXV][2];
  const int64_t n = D.n, K = D.K, l0 = int64_t(blockIdx.y) * HXV;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = int64_t(blockIdx.x) * HXR + RW * wv;
  const CH *h[RW];
  const double2 *x[HXV];
#pragma unroll
  for (int q = 0; q < RW; ++q)
    h[q] = reinterpret_cast<const CH *>(D.H) + std::min<int64_t>(r0 + q, n - 1) * D.ld;
#pragma unroll
  for (int v = 0; v < HXV; ++v) x[v] = D.X + size_t(std::min<int64_t>(l0 + v, K - 1)) * n;
  double yr[RW][HXV], yi[RW][HXV];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int v = 0; v < HXV; ++v) yr[q][v] = yi[q][v] = 0;
  constexpr int CU = 4;  // columns per lane with their loads in flight together
  for (int64_t c0 = lane; c0 < n; c0 += 64 * CU) {
    double2 a[CU][RW], b[CU][HXV];
#pragma unroll
    for (int u = 0; u < CU; ++u) {  // columns past n read column n - 1 and are dropped
      const int64_t c = std::min<int64_t>(c0 + 64 * u, n - 1);
#pragma unroll
      for (int q = 0; q < RW; ++q) a[u][q] = to_d2(h[q][c]);
#pragma unroll
      for (int v = 0; v < HXV; ++v) b[u][v] = x[v][c];
    }
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const double f = c0 + 64 * u < n ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const double ax = f * a[u][q].x, ay = f * a[u][q].y;
#pragma unroll
        for (int v = 0; v < HXV; ++v) {
          yr[q][v] += ax * b[u][v].x - ay * b[u][v].y;
          yi[q][v] += ax * b[u][v].y + ay * b[u][v].x;
        }
      }
    }
  }
  // Re(conj(x_r) y_r) and |x_r|^2 over this wave's rows, on every lane
  double num[HXV], den[HXV];
#pragma unroll
  for (int v = 0; v < HXV; ++v) num[v] = den[v] = 0;
#pragma unroll
  for (int q = 0; q < RW; ++q) {
    const bool in = r0 + q < n;
    const int64_t rc = std::min<int64_t>(r0 + q, n - 1);
#pragma unroll
    for (int v = 0; v < HXV; ++v) {
      const double sr = wave_sum(yr[q][v]), si = wave_sum(yi[q][v]);
      const double2 xr = x[v][rc];
      num[v] += in ? xr.x * sr + xr.y * si : 0.0;
      den[v] += in ? xr.x * xr.x + xr.y * xr.y : 0.0;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < HXV; ++v) {
      sh[wv][v][0] = num[v];
      sh[wv][v][1] = den[v];
    }
  }
  __syncthreads();
  if (tid < 2 * HXV) {
    const int v = tid >> 1, f = tid & 1;
    double t = 0;
#pragma unroll
    for (int w = 0; w < ENT / 64; ++w) t += sh[w][v][f];
    if (l0 + v < K) D.rqp[(size_t(l0 + v) * size_t(cdiv(n, HXR)) + blockIdx.x) * 2 + f] = t;
  }
}

// one workgroup: reduce the partial quotients, write the refined values in
// ascending order and re-centre the poles of refined clusters
__global__ __launch_bounds__(ENT) void k_rq_fin(Desc D) {
  __shared__ double sh[ENT / 64];
  __shared__ double th[KMAX];
  const int64_t n = D.n, K = D.K, nw = cdiv(n, HXR);
  const int tid = threadIdx.x;
  for (int64_t l = 0; l < K; ++l) {
    double num = 0, den = 0;
    for (int64_t p = tid; p < nw; p += ENT) {
      num += D.rqp[(size_t(l) * nw + p) * 2];
      den += D.rqp[(size_t(l) * nw + p) * 2 + 1];
    }
    num = block_sum<ENT>(num, sh);
    den = block_sum<ENT>(den, sh);
    if (tid == 0) {
      const bool ok = den > 0 && num == num;
      th[l] = ok ? num / den : D.omega[l];
      if (!ok) D.status[0] += 1;  // left unrefined (cluster beyond CMAX members)
    }
  }
  __syncthreads();
  if (tid == 0) {
    for (int64_t a = 1; a < K; ++a) {  // insertion sort (K <= KMAX)
      const double v = th[a];
      int64_t b = a - 1;
      while (b >= 0 && th[b] > v) {
        th[b + 1] = th[b];
        --b;
      }
      th[b + 1] = v;
    }
    // the clusters of the weights (runs of equal clo): heads carry the pole
    int64_t i = 0;
    while (i < K) {
      int64_t j = i;
      while (j + 1 < n && D.clo[j + 1] == i) ++j;
      if (j < K) {
        double s = 0;
        for (int64_t q = i; q <= j; ++q) s += th[q];
        D.pole[i] = s / double(j - i + 1);
        for (int64_t q = i + 1; q <= j; ++q) D.pole[q] = th[q];
      } else {
        D.status[2] += 1;  // cluster straddling K: its pole stays unrefined
      }
      i = j + 1;
    }
    for (int64_t l = 0; l < K; ++l) {
      D.wref[l] = th[l];
      D.omega[l] = th[l];
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// single block
// ---------------------------------------------------------------------------
template <typename TH, typename TA>
int32_t eigh_run(int64_t n, const void *Hmu, int64_t ld, const void *Bmu, double *omega,
                 double *pole, double *osc, void *ws, hipStream_t s, int64_t K) {
  Desc D;
  ws_layout(n, sizeof(TA) == 8, &D, (char *)ws, K);
  D.H = Hmu;
  D.ld = ld;
  D.B = (const double2 *)Bmu;
  D.omega = omega;
  D.pole = pole;
  D.osc = osc;
  auto grid = [&](int kind, int64_t j, int wpr) {
    return dim3((unsigned)kind_wgs<TA>(kind, n, j, wpr));
  };
  BSE_LAUNCH("k_copy_in", (k_copy_in<TH, TA, 4>), grid(K_COPY, 0, 4), dim3(ENT), 0, s, D, 0);
  // ---- initial reflection: B -> beta0 e_1, A <- Q0^dag A Q0 ----
  BSE_LAUNCH("k_load_b", (k_load_b<TH, TA, 4>), grid(K_LOADB, 0, 4), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_hemv0", (k_hemv0<TH, TA, 4>), grid(K_HEMV0, 0, 4), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_w0", (k_w0<TH, TA, 4>), grid(K_W0, 0, 4), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_rank2", (k_rank2<TH, TA, 4>), grid(K_RANK2, 0, 4), dim3(ENT), 0, s, D, 0);
  BSE_HIP_CHECK(hipGetLastError());
  // ---- blocked tridiagonalisation, two kernels per column ----
  int cur = 0;  // partial-sum record buffer written last
  const Desc D0 = D;
  for (int64_t j0 = 0; j0 < n; j0 += NBK) {
    if (j0 == g_tail0(n)) {  // the rest in one workgroup, in LDS
      BSE_LAUNCH("k_tail", k_tail<TA>, dim3(1), dim3(TNT), 0, s, D0, j0, int(K > 0));
      break;
    }
    const int nbk = g_nbk(n, j0);
    if (K > 0) D.V = D0.Vall + j0 * D0.ldv;  // keep every reflector for the back-transform
    BSE_LAUNCH("k_col0", (k_col0<TH, TA, 4>), grid(K_COL0, j0, 4), dim3(ENT), 0, s, D, j0, cur);
    for (int i = 0; i < nbk; ++i) {
      const int64_t jn = j0 + i, m = n - jn - 1;
      const int wpr = single_wpr(m);
#define BSE_COLA(W)                                                                         \
  BSE_LAUNCH("k_colA", (k_colA<TH, TA, W>), grid(K_COLA, jn, W), dim3(ENT), 0, s, D, jn, cur); \
  if (m > 0)                                                                                \
    BSE_LAUNCH("k_colB", (k_colB<TH, TA, W>), grid(K_COLB, jn, W), dim3(ENT), 0, s, D, jn, cur);
      if (wpr == 4) {
        BSE_COLA(4)
      } else if (wpr == 2) {
        BSE_COLA(2)
      } else if (wpr == 1) {
        BSE_COLA(1)
      } else {
        if (m > TILE_M) {  // lower tiles of the working copy
          const int tw = tile_wpr(m);
          if (tw == -1) {
            BSE_COLA(-1)
          } else if (tw == -2) {
            BSE_COLA(-2)
          } else {
            BSE_COLA(-3)
          }
        } else {
          BSE_COLA(0)
        }
      }
#undef BSE_COLA
      if (m <= 0) break;  // last diagonal element recorded; nothing below it
      cur ^= 1;
    }
    BSE_HIP_CHECK(hipGetLastError());
    if (kind_wgs<TA>(K_HER2K, n, j0, 4) > 0)
      BSE_LAUNCH("k_her2k", (k_her2k<TH, TA, 0>), grid(K_HER2K, j0, 4), dim3(ENT), 0, s, D, j0);
    BSE_HIP_CHECK(hipGetLastError());
  }
  // ---- tridiagonal eigenvalues and optical weights ----
  BSE_LAUNCH("k_tri_prep", k_tri_prep<TA>, dim3(1), dim3(RNT), 0, s, D,
             ctol_rel(n, sizeof(TA) == 8));
  BSE_LAUNCH("k_bisect_grid", (k_bisect_grid<TH, TA, 4>), dim3(NGRID / ENT), dim3(ENT), 0, s, D,
             0);
  BSE_LAUNCH("k_bisect", (k_bisect<TH, TA, 4>), grid(K_BISECT, 0, 4), dim3(ENT), 0, s, D, 1);
  BSE_LAUNCH("k_weights", (k_weights<TH, TA, 4>), grid(K_WEIGHTS, 0, 4), dim3(ENT), 0, s, D, 0);
  BSE_HIP_CHECK(hipGetLastError());
  if (K > 0) {
    D = D0;
    BSE_LAUNCH("k_invit", k_invit, dim3((unsigned)K), dim3(ENT), 0, s, D);
    if (n >= 2)
      BSE_LAUNCH("k_bx_tmat", k_bx_tmat, dim3((unsigned)cdiv(n - 1, NBK)), dim3(ENT), 0, s, D);
    BSE_LAUNCH("k_backxf", k_backxf, dim3((unsigned)K), dim3(ENT), 0, s, D);
    BSE_LAUNCH("k_hx_part", k_hx_part<TH>, dim3((unsigned)cdiv(n, HXR), (unsigned)cdiv(K, HXV)),
               dim3(ENT), 0,
               s, D);
    BSE_LAUNCH("k_rq_fin", k_rq_fin, dim3(1), dim3(ENT), 0, s, D);
    BSE_HIP_CHECK(hipGetLastError());
  }
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// single block, two-stage reduction; with refinement (K > 0) every reflector
// of both stages is kept and the eigenvectors of T are carried back through
// the chase (k_bx_chase), then through the stage-1 panels (k_bp_part,
// k_bp_apply) and the initial reflection (k_bx_q0)
// ---------------------------------------------------------------------------
template <typename TH, typename TA>
int32_t eigh_run_2s(int64_t n, const void *Hmu, int64_t ld, const void *Bmu, double *omega,
                    double *pole, double *osc, void *ws, hipStream_t s, int64_t K) {
  Desc D;
  ws_layout(n, sizeof(TA) == 8, &D, (char *)ws, K, true);
  D.H = Hmu;
  D.ld = ld;
  D.B = (const double2 *)Bmu;
  D.omega = omega;
  D.pole = pole;
  D.osc = osc;
  auto grid = [&](int kind) { return dim3((unsigned)kind_wgs<TA>(kind, n, 0, 4)); };
  BSE_LAUNCH("k_copy_in", (k_copy_in<TH, TA, 4>), grid(K_COPY), dim3(ENT), 0, s, D, 0);
  // ---- initial reflection: B -> beta0 e_1, A <- Q0^dag A Q0 ----
  BSE_LAUNCH("k_load_b", (k_load_b<TH, TA, 4>), grid(K_LOADB), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_hemv0", (k_hemv0<TH, TA, 4>), grid(K_HEMV0), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_w0", (k_w0<TH, TA, 4>), grid(K_W0), dim3(ENT), 0, s, D, 0);
  BSE_LAUNCH("k_rank2", (k_rank2<TH, TA, 4>), grid(K_RANK2), dim3(ENT), 0, s, D, 0);
  BSE_HIP_CHECK(hipGetLastError());
  // ---- stage 1: full -> band, one panel of SBW columns at a time ----
  int64_t j0 = 0;
  for (; j0 + SBW < n; j0 += SBW) {
    const int64_t p0 = j0 + SBW, m = n - p0;
    const int nw = (int)g_sb_nw(m), nref = (int)std::min<int64_t>(SBW, m);
    const dim3 rows((unsigned)cdiv(m, 64));  // k_sb_u, k_sb_w: 64 panel rows per workgroup
    BSE_LAUNCH("k_sb_pstart", k_sb_pstart<TA>, dim3(nw), dim3(ENT), 0, s, D, j0);
    for (int c = 0; c < nref; ++c)
      BSE_LAUNCH("k_sb_pcol", k_sb_pcol, dim3(nw), dim3(PCT), 0, s, D, j0, c, nw);
    BSE_LAUNCH("k_sb_tmat", k_sb_tmat<TA>, dim3(1), dim3(RNT), 0, s, D, j0, nw);
    BSE_LAUNCH("k_sb_u", k_sb_u<TA>, rows, dim3(ENT), 0, s, D, j0);
    BSE_LAUNCH("k_sb_hemm", k_sb_hemm<TA>, dim3((unsigned)g_sb_hemm_wgs(m)), dim3(ENT), 0, s, D,
               j0);
    const int nx = (int)g_sb_nx(m);
    BSE_LAUNCH("k_sb_xred", k_sb_xred, dim3(nx), dim3(ENT), 0, s, D, j0);
    BSE_LAUNCH("k_sb_z", k_sb_z, dim3(1), dim3(RNT), 0, s, D, nx);
    BSE_LAUNCH("k_sb_w", k_sb_w, rows, dim3(ENT), 0, s, D, j0);
    BSE_LAUNCH("k_her2k", k_sb_her2k<TA>, dim3((unsigned)sb_her2k_wgs<TA>(n, p0)), dim3(ENT), 0,
               s, D, p0);
    BSE_HIP_CHECK(hipGetLastError());
  }
  BSE_LAUNCH("k_sb_bandtail", k_sb_bandtail<TA>, dim3(1), dim3(ENT), 0, s, D, j0);
  // ---- stage 2: band -> tridiagonal, launch t runs the tasks 2 i + k = t ----
  for (int64_t t = 0; t <= g_bc_tmax(n); ++t) {
    const int64_t lo = g_bc_ilo(n, t), hi = g_bc_ihi(n, t);
    if (lo > hi) continue;
    if (K > 0)
      BSE_LAUNCH("k_sb_chase", k_sb_chase<true>, dim3((unsigned)(hi - lo + 1)), dim3(BCT), 0, s,
                 D, t, hi);
    else
      BSE_LAUNCH("k_sb_chase", k_sb_chase<false>, dim3((unsigned)(hi - lo + 1)), dim3(BCT), 0, s,
                 D, t, hi);
  }
  BSE_LAUNCH("k_sb_diag", k_sb_diag, dim3((unsigned)cdiv(n, ENT)), dim3(ENT), 0, s, D);
  BSE_HIP_CHECK(hipGetLastError());
  // ---- tridiagonal eigenvalues and optical weights ----
  BSE_LAUNCH("k_tri_prep", k_tri_prep<TA>, dim3(1), dim3(RNT), 0, s, D,
             ctol_rel(n, sizeof(TA) == 8));
  BSE_LAUNCH("k_bisect_grid", (k_bisect_grid<TH, TA, 4>), dim3(NGRID / ENT), dim3(ENT), 0, s, D,
             0);
  BSE_LAUNCH("k_bisect", (k_bisect<TH, TA, 4>), grid(K_BISECT), dim3(ENT), 0, s, D, 1);
  BSE_LAUNCH("k_weights", (k_weights<TH, TA, 4>), grid(K_WEIGHTS), dim3(ENT), 0, s, D, 0);
  BSE_HIP_CHECK(hipGetLastError());
  if (K > 0) {
    BSE_LAUNCH("k_invit", k_invit, dim3((unsigned)K), dim3(ENT), 0, s, D);
    if (n <= BXL - SBW)
      BSE_LAUNCH("k_bx_chase", k_bx_chase_lds, dim3((unsigned)K), dim3(BXT), 0, s, D);
    else
      BSE_LAUNCH("k_bx_chase", k_bx_chase, dim3((unsigned)K), dim3(BXC), 0, s, D);
    for (int64_t p = g_sb_npan(n) - 1; p >= 0; --p) {
      const dim3 g((unsigned)cdiv(n - SBW * (p + 1), BPR), (unsigned)cdiv(K, BPV));
      BSE_LAUNCH("k_bp_part", k_bp_part, g, dim3(ENT), 0, s, D, p);
      BSE_LAUNCH("k_bp_apply", k_bp_apply, g, dim3(BPT), 0, s, D, p);
    }
    BSE_LAUNCH("k_bx_q0", k_bx_q0, dim3((unsigned)K), dim3(ENT), 0, s, D);
    BSE_LAUNCH("k_hx_part", k_hx_part<TH>, dim3((unsigned)cdiv(n, HXR), (unsigned)cdiv(K, HXV)),
               dim3(ENT), 0,
               s, D);
    BSE_LAUNCH("k_rq_fin", k_rq_fin, dim3(1), dim3(ENT), 0, s, D);
    BSE_HIP_CHECK(hipGetLastError());
  }
  return BSE_OK;
}

// Smallest block that takes the two-stage reduction; process-wide, set by
// bse_block_eigh_set_two_stage.
std::atomic<int64_t> g_two_stage_min{4096};
inline bool takes_two_stage(int64_t n, int64_t) { return n >= g_two_stage_min.load(); }

// ---------------------------------------------------------------------------
// batched: every active block advances one step per launch
// ---------------------------------------------------------------------------
struct BatchLaunch {
  int kind;
  int64_t j;
  int cur;
  int nact;
  int total;
  size_t pre_off;  // ints into the prefix table
};

struct BatchPlan {
  int nb = 0, h_fp64 = 0, prec = 0, wpr = 4, htile = 0;
  char *ws = nullptr;
  Desc *d_desc = nullptr;
  int *d_pre = nullptr;
  std::vector<int64_t> n;  // sorted, descending
  std::vector<BatchLaunch> launches;
};

// Launch sequence and prefix tables of a batch (host side).
template <typename TA>
void plan_launches(BatchPlan &P, std::vector<int> &pre) {
  P.launches.clear();
  pre.clear();
  const int nb = P.nb;
  auto add = [&](int kind, int64_t j, int cur) {
    BatchLaunch L{kind, j, cur, 0, 0, pre.size()};
    int64_t tot = 0;
    pre.push_back(0);
    for (int b = 0; b < nb; ++b) {
      const int64_t w = kind_wgs<TA>(kind, P.n[b], j, P.wpr, P.htile);
      if (w == 0) break;  // sorted descending: the rest are inactive too
      tot += w;
      pre.push_back((int)tot);
      ++L.nact;
    }
    L.total = (int)tot;
    if (L.nact == 0) {
      pre.pop_back();
      return;
    }
    P.launches.push_back(L);
  };
  const int64_t nmax = P.n[0];
  add(K_COPY, 0, 0);
  add(K_LOADB, 0, 0);
  add(K_HEMV0, 0, 0);
  add(K_W0, 0, 0);
  add(K_RANK2, 0, 0);
  int cur = 0;
  for (int64_t j0 = 0; j0 < nmax; j0 += NBK) {
    add(K_COL0, j0, cur);
    for (int i = 0; i < NBK && j0 + i < nmax; ++i) {
      const int64_t jn = j0 + i;
      add(K_COLA, jn, cur);
      add(K_COLB, jn, cur);
      cur ^= 1;
    }
    add(K_HER2K, j0, cur);
  }
  // every block's tail in one launch: a block's working copy is not touched
  // after its last panel, so the tails need not sit in the lockstep chain
  P.launches.push_back(BatchLaunch{K_TAIL, 0, 0, nb, nb, 0});
  add(K_TRI, 0, 0);
  add(K_BGRID, 0, 0);
  add(K_BISECT, 0, 0);
  add(K_WEIGHTS, 0, 0);
}

template <typename TH, typename TA, int W>
int32_t batch_launch(const BatchPlan &P, const BatchLaunch &L, hipStream_t s) {
  const dim3 g((unsigned)L.total), b(ENT);
  const int *pre = P.d_pre + L.pre_off;
  const Desc *Ds = P.d_desc;
  switch (L.kind) {
    case K_COPY: BSE_LAUNCH("k_copy_in", (k_copy_in_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_LOADB: BSE_LAUNCH("k_load_b", (k_load_b_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_HEMV0: BSE_LAUNCH("k_hemv0", (k_hemv0_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_W0: BSE_LAUNCH("k_w0", (k_w0_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_RANK2: BSE_LAUNCH("k_rank2", (k_rank2_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_COL0: BSE_LAUNCH("k_col0", (k_col0_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, L.j, L.cur); break;
    case K_COLA: BSE_LAUNCH("k_colA", (k_colA_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, L.j, L.cur); break;
    case K_COLB: BSE_LAUNCH("k_colB", (k_colB_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, L.j, L.cur); break;
    case K_HER2K:
      if (P.htile)
        BSE_LAUNCH("k_her2k", (k_her2k_b<TH, TA, 1>), g, b, 0, s, Ds, pre, L.nact, L.j);
      else
        BSE_LAUNCH("k_her2k", (k_her2k_b<TH, TA, 0>), g, b, 0, s, Ds, pre, L.nact, L.j);
      break;
    case K_TRI: BSE_LAUNCH("k_tri_prep", k_tri_prep_b<TA>, g, dim3(RNT), 0, s, Ds, pre, L.nact, 0); break;
    case K_TAIL: BSE_LAUNCH("k_tail", k_tail_b<TA>, g, dim3(TNT), 0, s, Ds, L.cur, L.j); break;
    case K_BGRID: BSE_LAUNCH("k_bisect_grid", (k_bisect_grid_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
    case K_BISECT: BSE_LAUNCH("k_bisect", (k_bisect_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 1); break;
    default: BSE_LAUNCH("k_weights", (k_weights_b<TH, TA, W>), g, b, 0, s, Ds, pre, L.nact, 0); break;
  }
  return BSE_OK;
}

template <typename TH, typename TA>
int32_t batch_run(const BatchPlan &P, hipStream_t s) {
  for (const BatchLaunch &L : P.launches) {
    int32_t st = P.wpr == 4   ? batch_launch<TH, TA, 4>(P, L, s)
                 : P.wpr == 2 ? batch_launch<TH, TA, 2>(P, L, s)
                              : batch_launch<TH, TA, 1>(P, L, s);
    if (st) return st;
  }
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}

std::mutex g_plan_mu;
std::map<int64_t, BatchPlan> g_plans;
int64_t g_next_plan = 1;

size_t batch_ws_bytes(int32_t nb, const int64_t *h_n, bool a_fp64, std::vector<size_t> *offs,
                      size_t *desc_off, size_t *pre_off, size_t pre_ints) {
  size_t off = 0;
  for (int b = 0; b < nb; ++b) {
    if (offs) offs->push_back(off);
    off += ws_layout(h_n[b], a_fp64, nullptr, nullptr);
  }
  if (desc_off) *desc_off = off;
  off += align256(size_t(nb) * sizeof(Desc));
  if (pre_off) *pre_off = off;
  off += align256(pre_ints * sizeof(int));
  return off;
}

// upper bound of the prefix-table size: launches x (active blocks + 1)
size_t pre_bound(int32_t nb, const int64_t *h_n) {
  int64_t nmax = 0;
  for (int b = 0; b < nb; ++b) nmax = std::max(nmax, h_n[b]);
  const size_t launches = 9 + size_t(cdiv(nmax, NBK)) * (2 * NBK + 2);  // 9 one-off kinds
  return launches * size_t(nb + 1);
}

}  // namespace bse

using namespace bse;

extern "C" size_t bse_block_eigh_ws(int64_t n, int32_t h_fp64, int32_t prec, int32_t nrefine) {
  (void)h_fp64;
  if (n < 1 || nrefine < 0 || nrefine > KMAX) return 0;
  const int64_t K = std::min<int64_t>(nrefine, n);
  return ws_layout(n, prec == BSE_FP64, nullptr, nullptr, K, takes_two_stage(n, K));
}

extern "C" int64_t bse_block_eigh_set_two_stage(int64_t nmin) {
  if (nmin < 0) return g_two_stage_min.load();
  return g_two_stage_min.exchange(std::max<int64_t>(nmin, 2));
}

extern "C" int32_t bse_block_eigh(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64,
                                  const void *Bmu, int32_t prec, int32_t nrefine, double *omega,
                                  double *pole, double *osc, void *ws, size_t ws_bytes,
                                  bse_stream stream) {
  if (n < 1) return fail(BSE_ESHAPE, "n must be >= 1");
  if (n > 64 * 1024) return fail(BSE_ESHAPE, "n too large");
  if (!Hmu || !Bmu || !omega || !pole || !osc) return fail(BSE_EINVAL, "NULL pointer");
  if (ld < n) return fail(BSE_ESHAPE, "ld < n");
  if (prec != BSE_FP64 && prec != BSE_FP32) return fail(BSE_EINVAL, "unsupported precision");
  if (nrefine < 0 || nrefine > KMAX)
    return fail(BSE_EINVAL, "nrefine = %d outside 0 .. %d", nrefine, KMAX);
  const int64_t K = std::min<int64_t>(nrefine, n);
  const bool two = takes_two_stage(n, K);
  const size_t need = ws_layout(n, prec == BSE_FP64, nullptr, nullptr, K, two);
  if (!ws || ws_bytes < need)
    return fail(BSE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  if (two) {
    if (prec == BSE_FP64)
      return h_fp64 ? eigh_run_2s<double, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                    : eigh_run_2s<float, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
    return h_fp64 ? eigh_run_2s<double, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                  : eigh_run_2s<float, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
  }
  if (prec == BSE_FP64)
    return h_fp64 ? eigh_run<double, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                  : eigh_run<float, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
  return h_fp64 ? eigh_run<double, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                : eigh_run<float, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
}

// ---------------------------------------------------------------------------
// allocation-free single block: the workspace is a file-scope device array
// ---------------------------------------------------------------------------
// Every GPU the library runs on holds one copy until the process ends.  In
// host code `scratch` names a host-side stand-in, not the device array: its
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and only that address is passed to kernels.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEV] = {};

// Device address of this device's scratch array (looked up on first use).
int32_t scratch_of(hipStream_t s, void **out) {
  int dev = -1;
  BSE_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return fail(BSE_EDEVICE, "device %d out of range", dev);
  if (s) {
    int sdev = -1;
    BSE_HIP_CHECK(hipStreamGetDevice(s, &sdev));
    if (sdev != dev)
      return fail(BSE_EINVAL, "stream of device %d, but device %d is current", sdev, dev);
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    BSE_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(BSE_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BSE_OK;
}
}  // namespace

extern "C" size_t bse_block_eigh_noalloc_max(void) { return SCRATCH_BYTES; }

extern "C" int32_t bse_block_eigh_noalloc(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64,
                                          const void *Bmu, int32_t prec, int32_t nrefine,
                                          double *omega, double *pole, double *osc,
                                          bse_stream stream) {
  if (n < 1) return fail(BSE_ESHAPE, "n must be >= 1");
  if (n > 64 * 1024) return fail(BSE_ESHAPE, "n too large");
  if (!Hmu || !Bmu || !omega || !pole || !osc) return fail(BSE_EINVAL, "NULL pointer");
  if (ld < n) return fail(BSE_ESHAPE, "ld < n");
  if (prec != BSE_FP64 && prec != BSE_FP32) return fail(BSE_EINVAL, "unsupported precision");
  if (nrefine < 0 || nrefine > KMAX)
    return fail(BSE_EINVAL, "nrefine = %d outside 0 .. %d", nrefine, KMAX);
  const int64_t K = std::min<int64_t>(nrefine, n);
  const size_t need = ws_layout(n, prec == BSE_FP64, nullptr, nullptr, K);
  if (need > SCRATCH_BYTES)
    return fail(BSE_EWORKSPACE,
                "n = %lld needs %zu bytes of workspace; the static scratch holds %zu",
                (long long)n, need, SCRATCH_BYTES);
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  const int32_t st = scratch_of(s, &ws);
  if (st != BSE_OK) return st;
  if (prec == BSE_FP64)
    return h_fp64 ? eigh_run<double, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                  : eigh_run<float, double>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
  return h_fp64 ? eigh_run<double, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K)
                : eigh_run<float, float>(n, Hmu, ld, Bmu, omega, pole, osc, ws, s, K);
}

extern "C" int32_t bse_block_eigh_status(int64_t n, int32_t prec, int32_t nrefine,
                                         const void *ws, int32_t *h_status, bse_stream stream) {
  if (n < 1 || n > 64 * 1024) return fail(BSE_ESHAPE, "n outside 1 .. 65536");
  if (!h_status) return fail(BSE_EINVAL, "NULL pointer");
  if (prec != BSE_FP64 && prec != BSE_FP32) return fail(BSE_EINVAL, "unsupported precision");
  if (nrefine < 0 || nrefine > KMAX)
    return fail(BSE_EINVAL, "nrefine = %d outside 0 .. %d", nrefine, KMAX);
  hipStream_t s = (hipStream_t)stream;
  const void *base = ws;
  if (!base) {  // the static workspace of bse_block_eigh_noalloc on this device
    void *p = nullptr;
    const int32_t st = scratch_of(s, &p);
    if (st != BSE_OK) return st;
    base = p;
  }
  Desc D;
  ws_layout(n, prec == BSE_FP64, &D, (char *)base, std::min<int64_t>(nrefine, n));
  int32_t h[4] = {0, 0, 0, 0};
  BSE_HIP_CHECK(hipMemcpyAsync(h, D.status, sizeof(h), hipMemcpyDeviceToHost, s));
  BSE_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < 4; ++i) h_status[i] = h[i];
  if (h[0] > 0 || h[1] > 0)
    return fail(BSE_ENOCONV, "%d of the lowest %d eigenvalues left unrefined, %d non-finite",
                h[0], nrefine, h[1]);
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// batched block eigensolver
// ---------------------------------------------------------------------------
namespace {
int32_t check_batch(int32_t nb, const int64_t *h_n, int32_t prec) {
  if (nb < 1 || nb > NBMAX) return fail(BSE_ESHAPE, "batch of %d blocks (1 .. %d)", nb, NBMAX);
  if (!h_n) return fail(BSE_EINVAL, "NULL block sizes");
  for (int b = 0; b < nb; ++b)
    if (h_n[b] < 1 || h_n[b] > 16384)
      return fail(BSE_ESHAPE, "block %d: n = %lld outside 1 .. 16384", b, (long long)h_n[b]);
  if (prec != BSE_FP64 && prec != BSE_FP32) return fail(BSE_EINVAL, "unsupported precision");
  return BSE_OK;
}

// Recomputes the launch sequence for P.wpr and uploads the prefix table.
int32_t upload_tables(BatchPlan &P, hipStream_t s) {
  std::vector<int> pre;
  if (P.prec == BSE_FP64)
    plan_launches<double>(P, pre);
  else
    plan_launches<float>(P, pre);
  BSE_HIP_CHECK(hipMemcpyAsync(P.d_pre, pre.data(), pre.size() * sizeof(int),
                               hipMemcpyHostToDevice, s));
  BSE_HIP_CHECK(hipStreamSynchronize(s));
  return BSE_OK;
}

int32_t run_plan(const BatchPlan &P, hipStream_t s) {
  if (P.prec == BSE_FP64)
    return P.h_fp64 ? batch_run<double, double>(P, s) : batch_run<float, double>(P, s);
  return P.h_fp64 ? batch_run<double, float>(P, s) : batch_run<float, float>(P, s);
}
}  // namespace

extern "C" size_t bse_batch_eigh_ws(int32_t nb, const int64_t *h_n, int32_t h_fp64,
                                    int32_t prec) {
  (void)h_fp64;
  if (check_batch(nb, h_n, prec)) return 0;
  return batch_ws_bytes(nb, h_n, prec == BSE_FP64, nullptr, nullptr, nullptr,
                        pre_bound(nb, h_n));
}

extern "C" int32_t bse_batch_eigh_plan(int32_t nb, const int64_t *h_n, const void *const *h_Hmu,
                                       const int64_t *h_ld, int32_t h_fp64,
                                       const void *const *h_Bmu, int32_t prec,
                                       double *const *h_omega, double *const *h_pole,
                                       double *const *h_osc, void *ws, size_t ws_bytes,
                                       int64_t *h_plan, bse_stream stream) {
  int32_t st = check_batch(nb, h_n, prec);
  if (st) return st;
  if (!h_Hmu || !h_ld || !h_Bmu || !h_omega || !h_pole || !h_osc || !h_plan)
    return fail(BSE_EINVAL, "NULL argument array");
  for (int b = 0; b < nb; ++b) {
    if (!h_Hmu[b] || !h_Bmu[b] || !h_omega[b] || !h_pole[b] || !h_osc[b])
      return fail(BSE_EINVAL, "block %d: NULL pointer", b);
    if (h_ld[b] < h_n[b]) return fail(BSE_ESHAPE, "block %d: ld < n", b);
  }
  const bool a64 = prec == BSE_FP64;
  std::vector<int> order(nb);
  for (int b = 0; b < nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return h_n[x] > h_n[y]; });
  std::vector<int64_t> ns(nb);
  for (int b = 0; b < nb; ++b) ns[b] = h_n[order[b]];
  std::vector<size_t> offs;
  size_t desc_off = 0, pre_off = 0;
  const size_t need = batch_ws_bytes(nb, ns.data(), a64, &offs, &desc_off, &pre_off,
                                     pre_bound(nb, ns.data()));
  if (!ws || ws_bytes < need)
    return fail(BSE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  BatchPlan P;
  P.nb = nb;
  P.h_fp64 = h_fp64 ? 1 : 0;
  P.prec = prec;
  P.wpr = 4;
  P.ws = (char *)ws;
  P.n = ns;
  P.d_desc = (Desc *)(P.ws + desc_off);
  P.d_pre = (int *)(P.ws + pre_off);
  std::vector<Desc> D(nb);
  for (int b = 0; b < nb; ++b) {
    const int o = order[b];
    ws_layout(ns[b], a64, &D[b], P.ws + offs[b]);
    D[b].H = h_Hmu[o];
    D[b].ld = h_ld[o];
    D[b].B = (const double2 *)h_Bmu[o];
    D[b].omega = h_omega[o];
    D[b].pole = h_pole[o];
    D[b].osc = h_osc[o];
  }
  hipStream_t s = (hipStream_t)stream;
  BSE_HIP_CHECK(hipMemcpyAsync(P.d_desc, D.data(), nb * sizeof(Desc), hipMemcpyHostToDevice, s));
  st = upload_tables(P, s);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  const int64_t id = g_next_plan++;
  g_plans[id] = std::move(P);
  *h_plan = id;
  return BSE_OK;
}

extern "C" int32_t bse_batch_eigh_run(int64_t plan, bse_stream stream) {
  BatchPlan P;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(plan);
    if (it == g_plans.end()) return fail(BSE_EINVAL, "unknown plan %lld", (long long)plan);
    P = it->second;
  }
  return run_plan(P, (hipStream_t)stream);
}

extern "C" int32_t bse_batch_eigh_tune(int64_t plan, bse_stream stream, int32_t *h_wpr,
                                       int32_t *h_tile) {
  BatchPlan P;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(plan);
    if (it == g_plans.end()) return fail(BSE_EINVAL, "unknown plan %lld", (long long)plan);
    P = it->second;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  BSE_HIP_CHECK(hipEventCreate(&e0));
  BSE_HIP_CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_w = 4, best_t = 0;
  // every row split of the HEMV kernel with either trailing-update tile
  for (int t : {0, 1})
    for (int w : {4, 2, 1}) {
      P.wpr = w;
      P.htile = t;
      int32_t st = upload_tables(P, s);
      if (!st) st = run_plan(P, s);  // warm-up
      if (!st) {
        BSE_HIP_CHECK(hipEventRecord(e0, s));
        st = run_plan(P, s);
        BSE_HIP_CHECK(hipEventRecord(e1, s));
        BSE_HIP_CHECK(hipEventSynchronize(e1));
      }
      if (st) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return st;
      }
      float ms = 0;
      BSE_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_w = w;
        best_t = t;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P.wpr = best_w;
  P.htile = best_t;
  int32_t st = upload_tables(P, s);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans[plan] = P;
  if (h_wpr) *h_wpr = best_w;
  if (h_tile) *h_tile = best_t ? HerTile<float, 1>::BN : HerTile<float, 0>::BN;
  return BSE_OK;
}

extern "C" int32_t bse_batch_eigh_config(int64_t plan, int32_t wpr, int32_t tile,
                                         bse_stream stream) {
  if (wpr != 1 && wpr != 2 && wpr != 4) return fail(BSE_EINVAL, "waves per row %d (1, 2, 4)", wpr);
  if (tile != HerTile<float, 0>::BN && tile != HerTile<float, 1>::BN)
    return fail(BSE_EINVAL, "tile %d (%d or %d)", tile, HerTile<float, 0>::BN,
                HerTile<float, 1>::BN);
  BatchPlan P;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(plan);
    if (it == g_plans.end()) return fail(BSE_EINVAL, "unknown plan %lld", (long long)plan);
    P = it->second;
  }
  P.wpr = wpr;
  P.htile = tile == HerTile<float, 1>::BN ? 1 : 0;
  const int32_t st = upload_tables(P, (hipStream_t)stream);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans[plan] = P;
  return BSE_OK;
}

extern "C" int32_t bse_batch_eigh_free(int64_t plan) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (!g_plans.erase(plan)) return fail(BSE_EINVAL, "unknown plan %lld", (long long)plan);
  return BSE_OK;
}
