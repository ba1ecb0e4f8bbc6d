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
//     trailing matrix is updated lazily (A - V W^dag - W V^dag); after the panel
//     the rank-2 NBK update runs on MFMA.  Three kernels per column, one per
//     global dependency: k_hemv2 (reflector scalars from the column norm, then
//     y = A22 v, bound by HBM bandwidth), k_w (w = tau (y - V q - W p)), k_col
//     (finish w with its global dot product, update the next column, partial
//     norm and panel dot products for the next reflector).  The panel and all
//     scalar work are FP64; A is stored in FP64 or (prec FP32) FP32.
//  3. T is real symmetric tridiagonal (the reflectors make the subdiagonal
//     real).  All eigenvalues by bisection on Sturm counts (one thread per
//     eigenvalue, FP64).  Because Q0 Q maps e_1 to e_1,
//     |B_l|^2 = beta0^2 z_l(0)^2 with z_l the eigenvectors of T, and for a
//     cluster of (numerically) degenerate eigenvalues the summed weight is the
//     residue of G(z) = [(z - T)^-1]_00 = 1 / (z - d_0 - e_0^2 / (z - d_1 - ...))
//     at the cluster.  It is computed by the trapezoidal rule on a circle
//     around the cluster whose radius is the geometric mean of the cluster
//     width and the distance to the next eigenvalue (error decays like
//     (width / distance)^(M/2) with M nodes); off the real axis the continued
//     fraction has no vanishing pivots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bse_internal.h"
#include "mfma_tile.h"

namespace bse {
namespace {

constexpr int ENT = 256;     // threads per workgroup
constexpr int NBK = 32;      // panel width
constexpr int RNT = 1024;    // threads of the single-workgroup kernels

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return double2{a.x - b.x, a.y - b.y}; }

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

// Block-wide sum of one double (RNT or ENT threads); result valid in all threads.
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

struct Ws {
  void *A;
  int64_t lda;
  double2 *V, *W;    // [n][NBK]
  double2 *col;      // [n] updated current column
  double2 *y;        // [n] hemv output
  double2 *wraw;     // [n]
  double2 *vbuf;     // [n] current reflector
  double2 *part;     // [PMAX][2 NBK] panel dot partials (k_col)
  double2 *part2;    // [PMAX]
  double *part3;     // [PMAX]
  double2 *pq;       // [2 NBK]
  double2 *tau;      // [n + 1], index j + 1
  double2 *scl;      // [n + 1]
  double *d, *e;     // [n]
  double *e2;        // [n] squared subdiagonal
  double *tsc;       // [8] tridiagonal scalars
  double *beta0;     // [1]
};
constexpr int PMAX = 1024;

// rows per wave of k_hemv: at most 512 workgroups of 4 waves (PMAX partials)
int hemv_rpw(int64_t m) { return (int)std::max<int64_t>(1, (m + 4 * 512 - 1) / (4 * 512)); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t ws_layout(int64_t n, bool a_fp64, Ws *w, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const int64_t lda = (n + 15) / 16 * 16;
  Ws t;
  t.lda = lda;
  t.A = take(size_t(n) * lda * (a_fp64 ? 16 : 8));
  t.V = (double2 *)take(size_t(n) * NBK * 16);
  t.W = (double2 *)take(size_t(n) * NBK * 16);
  t.col = (double2 *)take(size_t(n) * 16);
  t.y = (double2 *)take(size_t(n) * 16);
  t.wraw = (double2 *)take(size_t(n) * 16);
  t.vbuf = (double2 *)take(size_t(n) * 16);
  t.part = (double2 *)take(size_t(PMAX) * 2 * NBK * 16);
  t.part2 = (double2 *)take(size_t(PMAX) * 16);
  t.part3 = (double *)take(size_t(PMAX) * 8);
  t.pq = (double2 *)take(2 * NBK * 16);
  t.tau = (double2 *)take(size_t(n + 1) * 16);
  t.scl = (double2 *)take(size_t(n + 1) * 16);
  t.d = (double *)take(size_t(n) * 8);
  t.e = (double *)take(size_t(n) * 8);
  t.e2 = (double *)take(size_t(n) * 8);
  t.tsc = (double *)take(8 * 8);
  t.beta0 = (double *)take(8);
  if (w) *w = t;
  return off;
}

// ---------------------------------------------------------------------------
template <typename TH, typename TA>
__global__ void k_copy_in(int64_t n, const TH *__restrict__ H, int64_t ldh, TA *__restrict__ A,
                          int64_t lda) {
  typedef typename C2T<TH>::t CH;
  typedef typename C2T<TA>::t CA;
  const int64_t r = blockIdx.y;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
       c += int64_t(gridDim.x) * blockDim.x) {
    const CH x = reinterpret_cast<const CH *>(H)[r * ldh + c];
    reinterpret_cast<CA *>(A)[r * lda + c] = CA{TA(x.x), TA(x.y)};
  }
}

// col[r] = B[r] (the "column" whose reflector maps B onto beta0 e_1)
__global__ void k_load_b(int64_t n, const double2 *__restrict__ B, double2 *__restrict__ col,
                         double *__restrict__ part3, int np3) {
  __shared__ double sh[ENT / 64];
  double s = 0;
  for (int64_t r = int64_t(blockIdx.x) * ENT + threadIdx.x; r < n; r += int64_t(gridDim.x) * ENT) {
    const double2 b = B[r];
    col[r] = b;
    if (r >= 1) s += b.x * b.x + b.y * b.y;
  }
  s = block_sum<ENT>(s, sh);
  if (threadIdx.x == 0) part3[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int i = gridDim.x; i < np3; ++i) part3[i] = 0;
}

// Reflector of column jr (acting on rows jr+1..n-1) with LAPACK's zlarfg
// semantics, (I - tau v v^dag)^dag (alpha, x) = (beta, 0) and
// v = (1, x / (alpha - beta)), followed by y[r] = sum_{c > jr} A[r][c] v[c]
// for r > jr (one wave per row).  Every workgroup recomputes the scalars from
// the column norm partials (a few dozen values); workgroup 0 stores them, the
// panel dot products p_l = V[:,l]^dag v and q_l = W[:,l]^dag v (l < ir, from
// k_col's partials) and the zeros of v above row jr+1.  v is formed on the fly
// from the updated column, and each wave stores v and V[:, ir] for its rows.
template <typename TA>
__global__ __launch_bounds__(ENT) void k_hemv2(int64_t n, int64_t jr, int64_t j0, int ir, int rpw,
                                               const TA *__restrict__ A, int64_t lda,
                                               const double2 *__restrict__ col,
                                               const double *__restrict__ part3,
                                               const double2 *__restrict__ partd, int np3,
                                               double *__restrict__ d, double *__restrict__ e,
                                               double *__restrict__ beta0,
                                               double2 *__restrict__ tau,
                                               double2 *__restrict__ scl,
                                               double2 *__restrict__ vbuf,
                                               double2 *__restrict__ V,
                                               const double2 *__restrict__ W,
                                               double2 *__restrict__ y, double2 *__restrict__ pq) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t m0 = jr + 1;
  double s = 0;
  for (int p = threadIdx.x; p < np3; p += ENT) s += part3[p];
  const double xn2 = block_sum<ENT>(s, sh);
  const double2 al = col[m0];
  double beta;
  double2 t = {0, 0}, sc = {0, 0};
  if (xn2 == 0.0 && al.y == 0.0) {
    beta = al.x;
  } else {
    const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
    beta = al.x >= 0 ? -nrm : nrm;
    t = double2{(beta - al.x) / beta, -al.y / beta};
    const double2 den = {al.x - beta, al.y};
    const double dd = den.x * den.x + den.y * den.y;
    sc = double2{den.x / dd, -den.y / dd};
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      if (jr >= 0) {
        d[jr] = col[jr].x;
        e[jr] = beta;
      } else {
        beta0[0] = beta;
      }
      tau[jr + 1] = t;
      scl[jr + 1] = sc;
    }
    if (threadIdx.x < 2 * NBK) {  // panel dot products for k_w
      const int slot = threadIdx.x, l = slot % NBK;
      double2 acc = {0, 0};
      if (l < ir) {
        for (int p = 0; p < np3; ++p) acc = cadd(acc, partd[int64_t(p) * 2 * NBK + slot]);
        const double2 head = slot < NBK ? V[m0 * NBK + l] : W[m0 * NBK + l];
        acc = cadd(double2{head.x, -head.y}, cmul(sc, acc));
      }
      pq[slot] = acc;
    }
    for (int64_t r = std::max<int64_t>(0, ir >= 0 ? j0 : 0) + threadIdx.x; r < m0; r += ENT) {
      vbuf[r] = double2{0, 0};
      if (ir >= 0) V[r * NBK + ir] = double2{0, 0};
    }
  }
  const int64_t rbase = m0 + (int64_t(blockIdx.x) * (ENT / 64) + wv) * rpw;
  for (int rr = 0; rr < rpw; ++rr) {
    const int64_t r = rbase + rr;
    if (r >= n) break;
    const CA *arow = reinterpret_cast<const CA *>(A) + r * lda;
    double sr = 0, si = 0;
    for (int64_t c = m0 + lane; c < n; c += 64) {
      const double2 a = to_d2(arow[c]);
      const double2 v = c == m0 ? double2{1, 0} : cmul(col[c], sc);
      sr += a.x * v.x - a.y * v.y;
      si += a.x * v.y + a.y * v.x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      y[r] = double2{sr, si};
      const double2 v = r == m0 ? double2{1, 0} : cmul(col[r], sc);
      vbuf[r] = v;
      if (ir >= 0) V[r * NBK + ir] = v;
    }
  }
}

// wraw[r] = tau_j (y[r] - sum_l V[r][l] q_l - sum_l W[r][l] p_l), partial conj(w).v
__global__ __launch_bounds__(ENT) void k_w(int64_t n, int64_t m0, int i, int64_t jt,
                                           const double2 *__restrict__ V,
                                           const double2 *__restrict__ W,
                                           const double2 *__restrict__ y,
                                           const double2 *__restrict__ pq,
                                           const double2 *__restrict__ vbuf,
                                           const double2 *__restrict__ tau,
                                           double2 *__restrict__ wraw,
                                           double2 *__restrict__ part2) {
  __shared__ double sh[ENT / 64];
  __shared__ double2 spq[2 * NBK];
  if (threadIdx.x < 2 * NBK) spq[threadIdx.x] = pq[threadIdx.x];
  __syncthreads();
  const int64_t r = m0 + int64_t(blockIdx.x) * ENT + threadIdx.x;
  double sr = 0, si = 0;
  if (r < n) {
    double2 w = y[r];
    for (int l = 0; l < i; ++l) {
      w = csub(w, cmul(V[r * NBK + l], spq[NBK + l]));
      w = csub(w, cmul(W[r * NBK + l], spq[l]));
    }
    w = cmul(tau[jt], w);
    wraw[r] = w;
    const double2 c = cmulc(w, vbuf[r]);
    sr = c.x;
    si = c.y;
  }
  sr = block_sum<ENT>(sr, sh);
  si = block_sum<ENT>(si, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = double2{sr, si};
}

// Finish W[:, i] = wraw + alpha v (alpha = -tau_j (w^dag v) / 2) for column j
// (fin != 0), then update column jr (panel index ir) with the panel's
// reflectors: col[r] = A[r][jr] - sum_{l < ir} (V[r][l] conj(W[jr][l]) +
// W[r][l] conj(V[jr][l])).  Per workgroup it stores the partial |col[r]|^2 and
// the partial sums conj(V[r][l]) col[r], conj(W[r][l]) col[r] (l < ir) over
// rows r >= jr + 2, which k_hemv2 turns into the next reflector and its panel
// dot products.  For jr = n - 1 it stores the last diagonal element.
template <typename TA>
__global__ __launch_bounds__(ENT) void k_col(int64_t n, int64_t rlo, int fin, int64_t j, int i,
                                             int64_t j0, int64_t jr, int ir,
                                             const TA *__restrict__ A, int64_t lda,
                                             double2 *__restrict__ V, double2 *__restrict__ W,
                                             const double2 *__restrict__ wraw,
                                             const double2 *__restrict__ vbuf,
                                             const double2 *__restrict__ part2, int np2,
                                             const double2 *__restrict__ tau,
                                             double2 *__restrict__ col,
                                             double *__restrict__ part3,
                                             double2 *__restrict__ partd,
                                             double *__restrict__ d) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  __shared__ double2 swj[NBK], svj[NBK];
  __shared__ double2 scol[ENT];
  __shared__ double2 sdot[4][2 * NBK];
  double2 alpha = {0, 0};
  if (fin) {
    double sr = 0, si = 0;
    for (int p = threadIdx.x; p < np2; p += ENT) {
      sr += part2[p].x;
      si += part2[p].y;
    }
    sr = block_sum<ENT>(sr, sh);
    si = block_sum<ENT>(si, sh);
    const double2 t = tau[j + 1];
    alpha = cmul(double2{-0.5 * t.x, -0.5 * t.y}, double2{sr, si});
  }
  if (jr >= 0 && threadIdx.x < NBK) {
    const int l = threadIdx.x;
    double2 wv = {0, 0}, vv = {0, 0};
    if (l < ir) {
      vv = V[jr * NBK + l];
      if (fin && l == i)
        wv = cadd(wraw[jr], cmul(alpha, vbuf[jr]));
      else
        wv = W[jr * NBK + l];
    }
    swj[l] = wv;
    svj[l] = vv;
  }
  __syncthreads();
  const int64_t r = rlo + int64_t(blockIdx.x) * ENT + threadIdx.x;
  double s = 0;
  double2 a = {0, 0};
  if (r < n) {
    if (fin && r >= j0) {
      const double2 w = r >= j + 1 ? cadd(wraw[r], cmul(alpha, vbuf[r])) : double2{0, 0};
      W[r * NBK + i] = w;
    }
    if (jr >= 0 && r >= jr) {
      a = to_d2(reinterpret_cast<const CA *>(A)[r * lda + jr]);
      for (int l = 0; l < ir; ++l) {
        const double2 vrl = V[r * NBK + l];
        const double2 wrl = (fin && l == i) ? (r >= j + 1 ? cadd(wraw[r], cmul(alpha, vbuf[r]))
                                                          : double2{0, 0})
                                            : W[r * NBK + l];
        // V[r][l] conj(W[jr][l]) + W[r][l] conj(V[jr][l])
        a = csub(a, cmul(vrl, double2{swj[l].x, -swj[l].y}));
        a = csub(a, cmul(wrl, double2{svj[l].x, -svj[l].y}));
      }
      col[r] = a;
      if (r == n - 1 && jr == n - 1) d[n - 1] = a.x;
      if (r >= jr + 2) s = a.x * a.x + a.y * a.y;
    }
  }
  s = block_sum<ENT>(s, sh);
  if (threadIdx.x == 0) part3[blockIdx.x] = s;
  if (ir > 0) {
    // partial panel dot products over this workgroup's rows r >= jr + 2
    scol[threadIdx.x] = (r < n && r >= jr + 2) ? a : double2{0, 0};
    __syncthreads();  // also orders the W[:, i] stores above
    const int slot = threadIdx.x % (2 * NBK), q = threadIdx.x / (2 * NBK), l = slot % NBK;
    double2 acc = {0, 0};
    if (l < ir) {
      const int64_t rb = rlo + int64_t(blockIdx.x) * ENT;
      for (int t = q * 64; t < q * 64 + 64; ++t) {
        const int64_t rr = rb + t;
        if (rr >= n) break;
        const double2 c = scol[t];
        if (c.x == 0.0 && c.y == 0.0) continue;
        const double2 m = slot < NBK ? V[rr * NBK + l] : W[rr * NBK + l];
        acc = cadd(acc, cmulc(m, c));
      }
    }
    sdot[q][slot] = acc;
    __syncthreads();
    if (threadIdx.x < 2 * NBK) {
      double2 t4 = {0, 0};
      for (int qq = 0; qq < 4; ++qq) t4 = cadd(t4, sdot[qq][threadIdx.x]);
      partd[int64_t(blockIdx.x) * 2 * NBK + threadIdx.x] = t4;
    }
  }
}

// Initial two-sided reflection: A -= v w^dag + w v^dag with w = wraw + alpha v.
template <typename TA>
__global__ __launch_bounds__(ENT) void k_rank2(int64_t n, TA *__restrict__ A, int64_t lda,
                                               const double2 *__restrict__ wraw,
                                               const double2 *__restrict__ vbuf,
                                               const double2 *__restrict__ part2, int np2,
                                               const double2 *__restrict__ tau) {
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
  const int64_t r = blockIdx.y;
  const double2 vr = vbuf[r], wr = cadd(wraw[r], cmul(alpha, vr));
  for (int64_t c = int64_t(blockIdx.x) * ENT + threadIdx.x; c < n; c += int64_t(gridDim.x) * ENT) {
    const double2 vc = vbuf[c], wc = cadd(wraw[c], cmul(alpha, vc));
    CA *p = reinterpret_cast<CA *>(A) + r * lda + c;
    double2 a = to_d2(*p);
    a = csub(a, cmul(vr, double2{wc.x, -wc.y}));
    a = csub(a, cmul(wr, double2{vc.x, -vc.y}));
    *p = CA{TA(a.x), TA(a.y)};
  }
}

// Trailing update on MFMA: A[r][c] -= sum_l V[r][l] conj(W[c][l]) + W[r][l] conj(V[c][l])
// for r, c >= c0; real GEMM with K = 4 nbk (x conj(y) interleave, see bse_build).
template <typename T> struct HerTile;
template <> struct HerTile<float> { static constexpr int BM = 128, BN = 64, BK = 32; };
template <> struct HerTile<double> { static constexpr int BM = 128, BN = 64, BK = 16; };

template <typename T>
__global__ __launch_bounds__(ENT) void k_her2k(int64_t n, int64_t c0, int nbk,
                                               const double2 *__restrict__ V,
                                               const double2 *__restrict__ W, T *__restrict__ A,
                                               int64_t lda) {
  constexpr int BM = HerTile<T>::BM, BN = HerTile<T>::BN, BK = HerTile<T>::BK;
  constexpr int P = Pitch<T, BK>::value, MI = BM / 32, NI = BN / 32, KC = BK / 2;
  constexpr int NA = (BM / 2) * KC / ENT, NB = BN * KC / ENT;
  __shared__ __attribute__((aligned(16))) T As[BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[BN * P];
  typedef typename C2T<T>::t C2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t a0 = c0 + int64_t(blockIdx.y) * (BM / 2), b0 = c0 + int64_t(blockIdx.x) * BN;
  if (a0 >= n || b0 >= n) return;
  typename Mfma<T>::acc_t acc[MI][NI];
  acc_zero<T, MI, NI>(acc);
  const int wm0 = (wv >> 1) * (BM / 2), wn0 = (wv & 1) * (BN / 2);
  const int K2 = 2 * nbk;  // complex reduction length: [V | W] against [W | V]
  for (int i0 = 0; i0 < K2; i0 += KC) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + ENT * u, r = it / KC, ii = it % KC, I = i0 + ii;
      const int64_t a = a0 + r;
      double2 x = {0, 0};
      if (a < n && I < K2) x = I < nbk ? V[a * NBK + I] : W[a * NBK + (I - nbk)];
      *reinterpret_cast<C2 *>(As + (2 * r) * P + 2 * ii) = C2{T(x.x), T(x.y)};
      *reinterpret_cast<C2 *>(As + (2 * r + 1) * P + 2 * ii) = C2{T(x.y), T(-x.x)};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + ENT * u, r = it / KC, ii = it % KC, I = i0 + ii;
      const int64_t b = b0 + r;
      double2 x = {0, 0};
      if (b < n && I < K2) x = I < nbk ? W[b * NBK + I] : V[b * NBK + (I - nbk)];
      *reinterpret_cast<C2 *>(Bs + r * P + 2 * ii) = C2{T(x.x), T(x.y)};
    }
    __syncthreads();
    mfma_slab<T, MI, NI, BK>(acc, As, Bs, wm0, wn0, lane);
    __syncthreads();
  }
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int64_t b = b0 + wn0 + 16 * ni + r16;
      const int64_t a = a0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (a + h < n && b < n) {
          C2 *p = reinterpret_cast<C2 *>(A) + (a + h) * lda + b;
          C2 x = *p;
          x.x -= acc[mi][ni][2 * h];
          x.y -= acc[mi][ni][2 * h + 1];
          *p = x;
        }
    }
}

// ---------------------------------------------------------------------------
// tridiagonal eigenvalues (bisection) and cluster weights
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
__global__ __launch_bounds__(RNT) void k_tri_prep(int64_t n, const double *__restrict__ d,
                                                  const double *__restrict__ e, double ctol_rel,
                                                  double *__restrict__ e2,
                                                  double *__restrict__ sc) {
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
    for (int i = 1; i < RNT / 64; ++i) {
      lo = fmin(lo, s_lo[i]);
      hi = fmax(hi, s_hi[i]);
      tn = fmax(tn, s_tn[i]);
    }
    lo = fmin(lo, s_lo[0]);
    hi = fmax(hi, s_hi[0]);
    tn = fmax(tn, s_tn[0]);
    const double pivmin = 1e-100 * fmax(1.0, tn);
    const double pad = 4.4e-16 * fmax(1.0, tn) * double(n) + pivmin;
    sc[0] = lo - pad;
    sc[1] = hi + pad;
    sc[2] = tn;
    sc[3] = pivmin;
    sc[4] = ctol_rel * fmax(1.0, tn);
  }
}

// number of eigenvalues of T below x (LDL^T Sturm sequence with pivot guard)
__device__ __forceinline__ int sturm_count(const double *__restrict__ d,
                                           const double *__restrict__ e2, int64_t n, double x,
                                           double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int64_t k = 1; k < n; ++k) {
    q = d[k] - x - e2[k - 1] * rcp64(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
}

__global__ void k_bisect(int64_t n, const double *__restrict__ d, const double *__restrict__ e2,
                         const double *__restrict__ sc, double *__restrict__ omega) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = sc[0], b = sc[1];
  const double pivmin = sc[3];
  for (int it = 0; it < 128; ++it) {
    const double mid = 0.5 * (a + b);
    if (mid <= a || mid >= b) break;
    if (b - a <= 2.3e-16 * fmax(fabs(a), fabs(b)) + pivmin) break;
    if (sturm_count(d, e2, n, mid, pivmin) > i)
      b = mid;
    else
      a = mid;
  }
  omega[i] = 0.5 * (a + b);
}

// Weights: a cluster is a maximal run of eigenvalues whose consecutive gaps
// are <= sc[4]; its head (first index) gets the cluster centre as pole and
// beta0^2 times the residue of G(z) = [(z - T)^-1]_00 as strength, the other
// members get zero strength.
constexpr int NCONT = 64;  // trapezoidal nodes on the circle
__global__ void k_weights(int64_t n, const double *__restrict__ d, const double *__restrict__ e2,
                          const double *__restrict__ sc, const double *__restrict__ beta0,
                          const double *__restrict__ omega, double *__restrict__ pole,
                          double *__restrict__ osc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ctol = sc[4];
  const double li = omega[i];
  if (i > 0 && li - omega[i - 1] <= ctol) {
    pole[i] = li;
    osc[i] = 0.0;
    return;
  }
  int64_t j = i;
  while (j + 1 < n && omega[j + 1] - omega[j] <= ctol) ++j;
  const double c = 0.5 * (omega[i] + omega[j]), half = 0.5 * (omega[j] - omega[i]);
  double g = 1e300;
  if (i > 0) g = fmin(g, c - omega[i - 1]);
  if (j + 1 < n) g = fmin(g, omega[j + 1] - c);
  if (g > 1e299) g = fmax(1.0, sc[2]);
  const double rad = sqrt(fmax(half, 1e-6 * g) * g);
  double wsum = 0.0;
  for (int m = 0; m < NCONT / 2; ++m) {
    const double th = 6.283185307179586 * (m + 0.5) / NCONT;
    const double zx = c + rad * cos(th), zy = rad * sin(th);
    // h = z - d_{n-1}; h = z - d_k - e_k^2 / h, k = n-2 .. 0; G = 1 / h
    double hx = zx - d[n - 1], hy = zy;
    for (int64_t k = n - 2; k >= 0; --k) {
      const double inv = e2[k] / (hx * hx + hy * hy);
      hx = zx - d[k] - hx * inv;
      hy = zy + hy * inv;
    }
    const double den = hx * hx + hy * hy;
    const double gx = hx / den, gy = -hy / den;
    // Re[G (z - c)] with z - c = rad (cos, sin)
    wsum += gx * rad * cos(th) - gy * rad * sin(th);
  }
  pole[i] = c;
  osc[i] = beta0[0] * beta0[0] * wsum * 2.0 / NCONT;
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" size_t bse_block_eigh_ws(int64_t n, int32_t h_fp64, int32_t prec, int32_t nrefine) {
  (void)h_fp64;
  (void)nrefine;
  if (n < 1) return 0;
  return ws_layout(n, prec == BSE_FP64, nullptr, nullptr);
}

namespace bse {
template <typename TH, typename TA>
int32_t eigh_run(int64_t n, const void *Hmu, int64_t ld, const void *Bmu, int32_t prec,
                 double *omega, double *pole, double *osc, void *ws, hipStream_t s) {
  Ws w;
  ws_layout(n, sizeof(TA) == 8, &w, (char *)ws);
  TA *A = (TA *)w.A;
  const int64_t lda = w.lda;
  {
    dim3 g((unsigned)std::min<int64_t>((n + ENT - 1) / ENT, 64), (unsigned)n);
    BSE_LAUNCH("k_copy_in", (k_copy_in<TH, TA>), g, dim3(ENT), 0, s, n, (const TH *)Hmu, ld, A, lda);
  }
  auto nwg_rows = [](int64_t m) { return (unsigned)std::max<int64_t>(1, (m + ENT - 1) / ENT); };
  auto hemv = [&](int64_t jr, int64_t j0, int ir, int np3) {
    const int64_t m = n - (jr + 1);
    const int rpw = hemv_rpw(m);
    const unsigned gh = (unsigned)std::max<int64_t>(1, (m + 4 * rpw - 1) / (4 * rpw));
    BSE_LAUNCH("k_hemv2", k_hemv2<TA>, dim3(gh), dim3(ENT), 0, s, n, jr, j0, ir, rpw, A, lda,
               w.col, w.part3, w.part, np3, w.d, w.e, w.beta0, w.tau, w.scl, w.vbuf, w.V, w.W,
               w.y, w.pq);
  };
  // ---- initial reflection: B -> beta0 e_1, A <- Q0^dag A Q0 ----
  {
    const unsigned g = std::min<unsigned>(nwg_rows(n), PMAX);
    BSE_LAUNCH("k_load_b", k_load_b, dim3(g), dim3(ENT), 0, s, n, (const double2 *)Bmu, w.col,
               w.part3, (int)g);
    hemv(-1, 0, -1, (int)g);
    const unsigned gw = nwg_rows(n);
    BSE_LAUNCH("k_w", k_w, dim3(gw), dim3(ENT), 0, s, n, int64_t(0), 0, int64_t(0), w.V, w.W, w.y,
               w.pq, w.vbuf, w.tau, w.wraw, w.part2);
    dim3 gr((unsigned)std::min<int64_t>((n + ENT - 1) / ENT, 16), (unsigned)n);
    BSE_LAUNCH("k_rank2", k_rank2<TA>, gr, dim3(ENT), 0, s, n, A, lda, w.wraw, w.vbuf, w.part2,
               (int)gw, w.tau);
    BSE_HIP_CHECK(hipGetLastError());
  }
  // ---- blocked tridiagonalisation ----
  for (int64_t j0 = 0; j0 < n; j0 += NBK) {
    const int nbk = (int)std::min<int64_t>(NBK, n - j0);
    // first column of the panel: no pending panel updates
    unsigned gc = nwg_rows(n - j0);
    BSE_LAUNCH("k_col", k_col<TA>, dim3(gc), dim3(ENT), 0, s, n, j0, 0, int64_t(-1), 0, j0, j0, 0,
               A, lda, w.V, w.W, w.wraw, w.vbuf, w.part2, 0, w.tau, w.col, w.part3, w.part, w.d);
    for (int i = 0; i < nbk; ++i) {
      const int64_t j = j0 + i;
      if (j + 1 >= n) break;  // the last diagonal element is stored by k_col
      hemv(j, j0, i, (int)gc);
      const int64_t m0 = j + 1, m = n - m0;
      const unsigned gw = nwg_rows(m);
      BSE_LAUNCH("k_w", k_w, dim3(gw), dim3(ENT), 0, s, n, m0, i, j + 1, w.V, w.W, w.y, w.pq,
                 w.vbuf, w.tau, w.wraw, w.part2);
      const bool more = (i + 1 < nbk);  // next column still in this panel
      const int64_t jr = more ? j + 1 : int64_t(-1);
      gc = nwg_rows(n - j0);
      BSE_LAUNCH("k_col", k_col<TA>, dim3(gc), dim3(ENT), 0, s, n, j0, 1, j, i, j0, jr,
                 more ? i + 1 : 0, A, lda, w.V, w.W, w.wraw, w.vbuf, w.part2, (int)gw, w.tau,
                 w.col, w.part3, w.part, w.d);
    }
    BSE_HIP_CHECK(hipGetLastError());
    // trailing update of the rows/columns after the panel
    const int64_t c0 = j0 + nbk;
    if (c0 < n) {
      constexpr int BM = HerTile<TA>::BM, BN = HerTile<TA>::BN;
      const int64_t m = n - c0;
      dim3 g((unsigned)((m + BN - 1) / BN), (unsigned)((2 * m + BM - 1) / BM));
      BSE_LAUNCH("k_her2k", k_her2k<TA>, g, dim3(ENT), 0, s, n, c0, nbk, w.V, w.W, A, lda);
      BSE_HIP_CHECK(hipGetLastError());
    }
  }
  // ---- tridiagonal eigenvalues and optical weights ----
  const double eps_w = sizeof(TA) == 8 ? 2.2e-16 : 1.2e-7;
  const double ctol_rel = 8.0 * eps_w * std::sqrt(double(n));
  BSE_LAUNCH("k_tri_prep", k_tri_prep, dim3(1), dim3(RNT), 0, s, n, w.d, w.e, ctol_rel, w.e2, w.tsc);
  BSE_LAUNCH("k_bisect", k_bisect, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n, w.d, w.e2,
             w.tsc, omega);
  BSE_LAUNCH("k_weights", k_weights, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n, w.d, w.e2,
             w.tsc, w.beta0, omega, pole, osc);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}
}  // namespace bse

extern "C" int32_t bse_block_eigh(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64,
                                  const void *Bmu, int32_t prec, int32_t nrefine, double *omega,
                                  double *pole, double *osc, void *ws, size_t ws_bytes,
                                  bse_stream stream) {
  if (n < 1) return fail(BSE_ESHAPE, "n must be >= 1");
  if (n > 64 * 1024) return fail(BSE_ESHAPE, "n too large");
  if (!Hmu || !Bmu || !omega || !pole || !osc) return fail(BSE_EINVAL, "NULL pointer");
  if (ld < n) return fail(BSE_ESHAPE, "ld < n");
  if (prec != BSE_FP64 && prec != BSE_FP32) return fail(BSE_EINVAL, "unsupported precision");
  if (nrefine != 0) return fail(BSE_EUNSUPPORTED, "refinement is not implemented yet");
  const size_t need = ws_layout(n, prec == BSE_FP64, nullptr, nullptr);
  if (!ws || ws_bytes < need)
    return fail(BSE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  if (prec == BSE_FP64)
    return h_fp64 ? eigh_run<double, double>(n, Hmu, ld, Bmu, prec, omega, pole, osc, ws, s)
                  : eigh_run<float, double>(n, Hmu, ld, Bmu, prec, omega, pole, osc, ws, s);
  return h_fp64 ? eigh_run<double, float>(n, Hmu, ld, Bmu, prec, omega, pole, osc, ws, s)
                : eigh_run<float, float>(n, Hmu, ld, Bmu, prec, omega, pole, osc, ws, s);
}
