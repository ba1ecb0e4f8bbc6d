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
//     the rank-2 NBK update runs on MFMA.  Per column: K_refl (one workgroup:
//     reflector scalars), K_hemv (y = A22 v plus the panel dot products, bound
//     by HBM bandwidth), K_reduce, K_w (w = tau (y - V q - W p)), K_col
//     (finish w, update the next column).  The panel and all scalar work are
//     FP64; A is stored in FP64 or (prec FP32) FP32.
//  3. T is real symmetric tridiagonal (the reflectors make the subdiagonal
//     real).  All eigenvalues by bisection on Sturm counts (one thread per
//     eigenvalue, FP64).  Because Q0 Q maps e_1 to e_1,
//     |B_l|^2 = beta0^2 z_l(0)^2 with z_l the eigenvectors of T; only the
//     leading unreduced block of T (the Krylov space of B_mu) has z_l(0) != 0,
//     and there z_l(0)^2 = 1 / h'(Omega_l) for the continued fraction
//     h(x) = x - d_0 - e_0^2 / (x - d_1 - e_1^2 / ...), whose zeros are the
//     block's eigenvalues.
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
  double2 *part;     // [PMAX][2 NBK]
  double2 *part2;    // [PMAX]
  double *part3;     // [PMAX]
  double2 *pq;       // [2 NBK]
  double2 *tau;      // [n + 1], index j + 1
  double2 *scl;      // [n + 1]
  double *d, *e;     // [n]
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

// Reflector for column jr (acting on rows jr+1..n-1), LAPACK zlarfg semantics:
// (I - tau v v^dag)^dag (alpha, x) = (beta, 0), v = (1, x / (alpha - beta)).
// Writes d[jr], e[jr] (or beta0 for jr = -1), tau, scale, vbuf and V[:, ir].
__global__ __launch_bounds__(RNT) void k_refl(int64_t n, int64_t jr, int64_t j0, int ir,
                                              const double2 *__restrict__ col,
                                              const double *__restrict__ part3, int np3,
                                              double *__restrict__ d, double *__restrict__ e,
                                              double *__restrict__ beta0, double2 *__restrict__ tau,
                                              double2 *__restrict__ scl,
                                              double2 *__restrict__ vbuf,
                                              double2 *__restrict__ V) {
  __shared__ double sh[RNT / 64];
  __shared__ double2 s_scale;
  double s = 0;
  for (int i = threadIdx.x; i < np3; i += RNT) s += part3[i];
  const double xn2 = block_sum<RNT>(s, sh);
  if (threadIdx.x == 0) {
    if (jr >= 0) d[jr] = col[jr].x;
    double2 t = {0, 0}, sc = {0, 0};
    if (jr + 1 < n) {
      const double2 al = col[jr + 1];
      double beta;
      if (xn2 == 0.0 && al.y == 0.0) {
        beta = al.x;
      } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
        beta = al.x >= 0 ? -nrm : nrm;
        t = double2{(beta - al.x) / beta, -al.y / beta};
        const double2 den = {al.x - beta, al.y};  // 1 / (alpha - beta)
        const double dd = den.x * den.x + den.y * den.y;
        sc = double2{den.x / dd, -den.y / dd};
      }
      if (jr >= 0)
        e[jr] = beta;
      else
        beta0[0] = beta;
    }
    tau[jr + 1] = t;
    scl[jr + 1] = sc;
    s_scale = sc;
  }
  __syncthreads();
  const double2 sc = s_scale;
  const int64_t lo = jr < 0 ? 0 : std::min<int64_t>(jr, j0);
  for (int64_t r = lo + threadIdx.x; r < n; r += RNT) {
    double2 v = {0, 0};
    if (r == jr + 1)
      v = double2{1, 0};
    else if (r > jr + 1)
      v = cmul(col[r], sc);
    if (r >= 0) vbuf[r] = v;
    if (ir >= 0 && r >= j0) V[r * NBK + ir] = v;
  }
}

// y[r] = sum_{c >= m0} A[r][c] v[c] for r >= m0, plus the panel dot products
// p_l = sum_r conj(V[r][l]) v[r], q_l = sum_r conj(W[r][l]) v[r] (l < i) over
// this workgroup's rows.  One wave per row.
template <typename TA>
__global__ __launch_bounds__(ENT) void k_hemv(int64_t n, int64_t m0, int i, int rpw,
                                              const TA *__restrict__ A, int64_t lda,
                                              const double2 *__restrict__ vbuf,
                                              const double2 *__restrict__ V,
                                              const double2 *__restrict__ W,
                                              double2 *__restrict__ y, double2 *__restrict__ part) {
  typedef typename C2T<TA>::t CA;
  __shared__ double2 sdot[ENT / 64][2 * NBK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t rbase = m0 + (int64_t(blockIdx.x) * (ENT / 64) + wv) * rpw;
  double2 dp = {0, 0}, dq = {0, 0};  // lane l < i: p_l, q_l partial; lane holds index lane
  for (int rr = 0; rr < rpw; ++rr) {
    const int64_t r = rbase + rr;
    if (r >= n) break;
    const CA *arow = reinterpret_cast<const CA *>(A) + r * lda;
    double sr = 0, si = 0;
    for (int64_t c = m0 + lane; c < n; c += 64) {
      const double2 a = to_d2(arow[c]);
      const double2 v = vbuf[c];
      sr += a.x * v.x - a.y * v.y;
      si += a.x * v.y + a.y * v.x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) y[r] = double2{sr, si};
    if (lane < i) {
      const double2 vr = vbuf[r];
      dp = cadd(dp, cmulc(V[r * NBK + lane], vr));
      dq = cadd(dq, cmulc(W[r * NBK + lane], vr));
    }
  }
  if (lane < NBK) {
    sdot[wv][lane] = dp;
    sdot[wv][NBK + lane] = dq;
  }
  __syncthreads();
  if (threadIdx.x < 2 * NBK) {
    double2 s = {0, 0};
    for (int w = 0; w < ENT / 64; ++w) s = cadd(s, sdot[w][threadIdx.x]);
    part[int64_t(blockIdx.x) * 2 * NBK + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(RNT) void k_reduce(int np, int i, const double2 *__restrict__ part,
                                                double2 *__restrict__ pq) {
  // pq[l] = sum over workgroups of part[.][l] for l < i (p) and NBK + l (q)
  __shared__ double2 sh[RNT];
  const int slot = threadIdx.x % (2 * NBK), grp = threadIdx.x / (2 * NBK);
  constexpr int G = RNT / (2 * NBK);
  double2 s = {0, 0};
  for (int p = grp; p < np; p += G) s = cadd(s, part[int64_t(p) * 2 * NBK + slot]);
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 2 * NBK) {
    double2 t = {0, 0};
    for (int g = 0; g < G; ++g) t = cadd(t, sh[g * 2 * NBK + threadIdx.x]);
    pq[threadIdx.x] = t;
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
// W[r][l] conj(V[jr][l])), and partial |col[r]|^2 over r >= jr + 2.
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
                                             double *__restrict__ part3) {
  typedef typename C2T<TA>::t CA;
  __shared__ double sh[ENT / 64];
  __shared__ double2 swj[NBK], svj[NBK];
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
  if (r < n) {
    if (fin && r >= j0) {
      const double2 w = r >= j + 1 ? cadd(wraw[r], cmul(alpha, vbuf[r])) : double2{0, 0};
      W[r * NBK + i] = w;
    }
    if (jr >= 0 && r >= jr) {
      double2 a = to_d2(reinterpret_cast<const CA *>(A)[r * lda + jr]);
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
      if (r >= jr + 2) s = a.x * a.x + a.y * a.y;
    }
  }
  s = block_sum<ENT>(s, sh);
  if (threadIdx.x == 0) part3[blockIdx.x] = s;
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
// tridiagonal eigenvalues (bisection) and leading-block weights
// ---------------------------------------------------------------------------
__device__ int sturm_count(const double *d, const double *e, int64_t lo, int64_t hi, double x,
                           double pivmin) {
  // number of eigenvalues of T[lo..hi] below x
  int cnt = 0;
  double q = 1.0;
  for (int64_t k = lo; k <= hi; ++k) {
    const double off = k > lo ? e[k - 1] : 0.0;
    q = d[k] - x - (k > lo ? off * off / q : 0.0);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
}

__device__ double bisect(const double *d, const double *e, int64_t lo, int64_t hi, int64_t idx,
                         double glo, double ghi, double pivmin) {
  double a = glo, b = ghi;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (a + b);
    if (mid <= a || mid >= b) break;
    if (b - a <= 2.2e-16 * fmax(fabs(a), fabs(b)) + pivmin) break;
    if (sturm_count(d, e, lo, hi, mid, pivmin) > idx)
      b = mid;
    else
      a = mid;
  }
  return 0.5 * (a + b);
}

__global__ void k_tridiag(int64_t n, const double *__restrict__ d, const double *__restrict__ e,
                          const double *__restrict__ beta0, double split_rel,
                          double *__restrict__ omega, double *__restrict__ pole,
                          double *__restrict__ osc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // norm and Gershgorin interval of T
  double tn = 0, glo = 1e300, ghi = -1e300;
  for (int64_t k = 0; k < n; ++k) {
    const double r = (k > 0 ? fabs(e[k - 1]) : 0.0) + (k + 1 < n ? fabs(e[k]) : 0.0);
    glo = fmin(glo, d[k] - r);
    ghi = fmax(ghi, d[k] + r);
    tn = fmax(tn, fabs(d[k]) + r);
  }
  const double pivmin = 1e-100 * fmax(1.0, tn);
  const double pad = 4.4e-16 * fmax(1.0, tn) * n + pivmin;
  glo -= pad;
  ghi += pad;
  omega[i] = bisect(d, e, 0, n - 1, i, glo, ghi, pivmin);
  // leading unreduced block [0, s]
  const double tol = split_rel * tn;
  int64_t s = n - 1;
  for (int64_t k = 0; k + 1 < n; ++k)
    if (fabs(e[k]) <= tol) {
      s = k;
      break;
    }
  double p = 0, w = 0;
  if (i <= s) {
    double blo = 1e300, bhi = -1e300;
    for (int64_t k = 0; k <= s; ++k) {
      const double r = (k > 0 ? fabs(e[k - 1]) : 0.0) + (k < s ? fabs(e[k]) : 0.0);
      blo = fmin(blo, d[k] - r);
      bhi = fmax(bhi, d[k] + r);
    }
    p = bisect(d, e, 0, s, i, blo - pad, bhi + pad, pivmin);
    // h(x) = x - d_k - e_k^2 / h_{k+1}, h' = 1 + (e_k^2 / h_{k+1}^2) h'_{k+1}
    double h = p - d[s], hp = 1.0;
    for (int64_t k = s - 1; k >= 0; --k) {
      if (fabs(h) < pivmin) h = h < 0 ? -pivmin : pivmin;
      const double t = e[k] * e[k] / h;
      hp = 1.0 + (t / h) * hp;
      h = p - d[k] - t;
    }
    w = beta0[0] * beta0[0] / hp;
  }
  pole[i] = p;
  osc[i] = w;
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
    hipLaunchKernelGGL((k_copy_in<TH, TA>), g, dim3(ENT), 0, s, n, (const TH *)Hmu, ld, A, lda);
  }
  auto nwg_rows = [](int64_t m) { return (unsigned)std::max<int64_t>(1, (m + ENT - 1) / ENT); };
  // ---- initial reflection: B -> beta0 e_1 ----
  {
    const unsigned g = std::min<unsigned>(nwg_rows(n), PMAX);
    hipLaunchKernelGGL(k_load_b, dim3(g), dim3(ENT), 0, s, n, (const double2 *)Bmu, w.col,
                       w.part3, (int)g);
    hipLaunchKernelGGL(k_refl, dim3(1), dim3(RNT), 0, s, n, int64_t(-1), int64_t(0), -1, w.col,
                       w.part3, (int)g, w.d, w.e, w.beta0, w.tau, w.scl, w.vbuf, w.V);
    const int rpw = hemv_rpw(n);
    const unsigned gh = (unsigned)((n + 4 * rpw - 1) / (4 * rpw));
    hipLaunchKernelGGL(k_hemv<TA>, dim3(gh), dim3(ENT), 0, s, n, int64_t(0), 0, rpw, A, lda,
                       w.vbuf, w.V, w.W, w.y, w.part);
    const unsigned gw = nwg_rows(n);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RNT), 0, s, 0, 0, w.part, w.pq);
    hipLaunchKernelGGL(k_w, dim3(gw), dim3(ENT), 0, s, n, int64_t(0), 0, int64_t(0), w.V, w.W, w.y,
                       w.pq, w.vbuf, w.tau, w.wraw, w.part2);
    dim3 gr((unsigned)std::min<int64_t>((n + ENT - 1) / ENT, 16), (unsigned)n);
    hipLaunchKernelGGL(k_rank2<TA>, gr, dim3(ENT), 0, s, n, A, lda, w.wraw, w.vbuf, w.part2,
                       (int)gw, w.tau);
    BSE_HIP_CHECK(hipGetLastError());
  }
  // ---- blocked tridiagonalisation ----
  int np2 = 0;
  for (int64_t j0 = 0; j0 < n; j0 += NBK) {
    const int nbk = (int)std::min<int64_t>(NBK, n - j0);
    // first column of the panel: plain copy (no pending panel updates)
    {
      const unsigned g = nwg_rows(n - j0);
      hipLaunchKernelGGL(k_col<TA>, dim3(g), dim3(ENT), 0, s, n, j0, 0, int64_t(-1), 0, j0, j0, 0,
                         A, lda, w.V, w.W, w.wraw, w.vbuf, w.part2, 0, w.tau, w.col, w.part3);
      hipLaunchKernelGGL(k_refl, dim3(1), dim3(RNT), 0, s, n, j0, j0, 0, w.col, w.part3, (int)g,
                         w.d, w.e, w.beta0, w.tau, w.scl, w.vbuf, w.V);
    }
    for (int i = 0; i < nbk; ++i) {
      const int64_t j = j0 + i;
      if (j + 1 >= n) break;  // last diagonal element already recorded
      const int64_t m0 = j + 1, m = n - m0;
      const int rpw = hemv_rpw(m);
      const unsigned gh = (unsigned)((m + 4 * rpw - 1) / (4 * rpw));
      hipLaunchKernelGGL(k_hemv<TA>, dim3(gh), dim3(ENT), 0, s, n, m0, i, rpw, A, lda, w.vbuf,
                         w.V, w.W, w.y, w.part);
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RNT), 0, s, (int)gh, i, w.part, w.pq);
      const unsigned gw = nwg_rows(m);
      hipLaunchKernelGGL(k_w, dim3(gw), dim3(ENT), 0, s, n, m0, i, j + 1, w.V, w.W, w.y, w.pq,
                         w.vbuf, w.tau, w.wraw, w.part2);
      np2 = (int)gw;
      const bool more = (i + 1 < nbk);  // next column still in this panel
      const int64_t jr = more ? j + 1 : int64_t(-1);
      const unsigned gc = nwg_rows(n - j0);
      hipLaunchKernelGGL(k_col<TA>, dim3(gc), dim3(ENT), 0, s, n, j0, 1, j, i, j0, jr,
                         more ? i + 1 : 0, A, lda, w.V, w.W, w.wraw, w.vbuf, w.part2, np2, w.tau,
                         w.col, w.part3);
      if (more)
        hipLaunchKernelGGL(k_refl, dim3(1), dim3(RNT), 0, s, n, jr, j0, i + 1, w.col, w.part3,
                           (int)gc, w.d, w.e, w.beta0, w.tau, w.scl, w.vbuf, w.V);
    }
    BSE_HIP_CHECK(hipGetLastError());
    // trailing update of the rows/columns after the panel
    const int64_t c0 = j0 + nbk;
    if (c0 < n) {
      constexpr int BM = HerTile<TA>::BM, BN = HerTile<TA>::BN;
      const int64_t m = n - c0;
      dim3 g((unsigned)((m + BN - 1) / BN), (unsigned)((2 * m + BM - 1) / BM));
      hipLaunchKernelGGL(k_her2k<TA>, g, dim3(ENT), 0, s, n, c0, nbk, w.V, w.W, A, lda);
      BSE_HIP_CHECK(hipGetLastError());
    }
  }
  const double split_rel = (sizeof(TA) == 8 ? 2.2e-16 : 1.2e-7) * 64.0 * std::sqrt(double(n));
  hipLaunchKernelGGL(k_tridiag, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n, w.d, w.e,
                     w.beta0, split_rel, omega, pole, osc);
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
