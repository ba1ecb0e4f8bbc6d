// bse_build: the Tamm-Dancoff electron-hole Hamiltonian on MFMA.
//
//   H[(k v c),(k' v' c')] = delta (E_c(k) - E_v(k))
//        + (2/N_k) sum_I Mx[k,v,c,I] v_I conj(Mx[k',v',c',I])            exchange
//        - (1/N_k) sum_IJ conj(Mc[k,k'][c,c',I]) W_IJ(k-k') Mv[k,k'][v,v',J]   direct
//
// Paper: Eq. (BSE-eigval) with Eq. (w_interaction2) (vector-matrix-vector
// products over the mixed-basis index, prefactor 1/N_k); spin factor 2 on the
// bare exchange (Sec. II); the loop over q = k - k' is outermost (Sec. III.C.2).
//
// Three kernels, all dense contractions on MFMA 16x16x4 (f32 or f64):
//   k_exchange   writes every H element: diagonal + exchange (a complex
//                Hermitian rank-Nmb product, rows gathered through the k-orbit map)
//   k_direct_t   for a batch of q: T_q = Mv(k, k-q) W(q) for all k at once
//                (M = 2 nk nv^2 real rows, N = K = Nmb), written to workspace
//   k_direct_d   per pair (k, k-q): D = conj(Mc) T^T (2 nc^2 x nv^2, K = 2 Nmb)
//                and H -= D / N_k (each H element is owned by one pair)
// Complex products run as real GEMMs with the reduction index interleaved as
// (I, re/im): for x, y complex rows, x conj(y) = [(re, im).(re', im')] +
// i [(im, -re).(re', im')], and conj(x) y = [(re, im).(re', im')] +
// i [(-im, re).(re', im')].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "bse_internal.h"
#include "build_common.h"
#include "mfma_tile.h"

namespace bse {

namespace {

constexpr int NT = 256;

template <typename T> struct BuildTile;
template <> struct BuildTile<float> { static constexpr int BM = 128, BN = 128, BK = 32; };
template <> struct BuildTile<double> { static constexpr int BM = 128, BN = 128, BK = 16; };

// ---------------------------------------------------------------------------
// exchange + diagonal
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2, 8))) void k_exchange(int nk, int nv, int nc, int nmb,
                                                 const int32_t *__restrict__ korb,
                                                 const T *__restrict__ mx,
                                                 const double *__restrict__ vdiag,
                                                 const double *__restrict__ ev,
                                                 const double *__restrict__ ec, T *__restrict__ H,
                                                 int64_t ldh, double scale, int diag) {
  constexpr int BM = BuildTile<T>::BM, BN = BuildTile<T>::BN, BK = BuildTile<T>::BK;
  constexpr int P = Pitch<T, BK>::value, MI = BM / 32, NI = BN / 32, KC = BK / 2;
  constexpr int NA = (BM / 2) * KC / NT, NB = BN * KC / NT;
  __shared__ __attribute__((aligned(16))) T As[BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[BN * P];
  typedef typename Cplx<T>::type C2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = nv * nc;
  const int64_t N = int64_t(nk) * nb;
  const int64_t a0 = int64_t(blockIdx.y) * (BM / 2), b0 = int64_t(blockIdx.x) * BN;
  // row pointers of the rows this thread loads; rows past N read row 0 and
  // are zeroed by a mask, so no load sits behind a branch
  const C2 *arow[NA];
  const C2 *brow[NB];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int64_t a = a0 + (tid + NT * u) / KC;
    const int64_t ac = a < N ? a : 0;
    arow[u] = reinterpret_cast<const C2 *>(mx) + (int64_t(korb[ac / nb]) * nb + ac % nb) * nmb;
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int64_t b = b0 + (tid + NT * u) / KC;
    const int64_t bc = b < N ? b : 0;
    brow[u] = reinterpret_cast<const C2 *>(mx) + (int64_t(korb[bc / nb]) * nb + bc % nb) * nmb;
  }
  typename Mfma<T>::acc_t acc[MI][NI];
  acc_zero<T, MI, NI>(acc);
  const int wm0 = (wv >> 1) * (BM / 2), wn0 = (wv & 1) * (BN / 2);
  // every slab's loads are issued together from in-bounds addresses (entries
  // past nmb read entry nmb - 1 and are zeroed when staged): no load waits
  // behind a branch
  C2 xa[NA], xb[NB];
  T va[NA];
  auto load = [&](int i0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int I = min(i0 + (tid + NT * u) % KC, nmb - 1);
      xa[u] = arow[u][I];
      va[u] = T(vdiag[I]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) xb[u] = brow[u][min(i0 + (tid + NT * u) % KC, nmb - 1)];
  };
  for (int i0 = 0; i0 < nmb; i0 += KC) {
    load(i0);
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + NT * u, r = it / KC, i = it % KC;
      const T vI = (i0 + i < nmb && a0 + r < N) ? va[u] : T(0);
      const C2 x = xa[u];
      *reinterpret_cast<C2 *>(As + (2 * r) * P + 2 * i) = C2{x.x * vI, x.y * vI};
      *reinterpret_cast<C2 *>(As + (2 * r + 1) * P + 2 * i) = C2{x.y * vI, -x.x * vI};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + NT * u, r = it / KC, i = it % KC;
      const T m = (i0 + i < nmb && b0 + r < N) ? T(1) : T(0);
      *reinterpret_cast<C2 *>(Bs + r * P + 2 * i) = C2{xb[u].x * m, xb[u].y * m};
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
      for (int h = 0; h < 2; ++h) {
        const int64_t aa = a + h;
        if (aa < N && b < N) {
          double re = scale * double(acc[mi][ni][2 * h]);
          const double im = scale * double(acc[mi][ni][2 * h + 1]);
          if (diag && aa == b) {
            const int k = int(aa / nb), v = int((aa / nc) % nv), c = int(aa % nc);
            re += ec[int64_t(k) * nc + c] - ev[int64_t(k) * nv + v];
          }
          reinterpret_cast<C2 *>(H)[aa * ldh + b] = C2{T(re), T(im)};
        }
      }
    }
}

// ---------------------------------------------------------------------------
// direct term, stage 1: T_q[(k,v,v')][I] = sum_J Mv(k,k-q)[v,v',J] W_q[I][J]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_direct_t(int n1, int n2, int n3, int nv, int nmb, int q0,
                                                 const int32_t *__restrict__ qorb,
                                                 const int32_t *__restrict__ pidx,
                                                 const uint8_t *__restrict__ pconj,
                                                 const T *__restrict__ mv,
                                                 const T *__restrict__ w, T *__restrict__ Tq) {
  constexpr int BM = BuildTile<T>::BM, BN = BuildTile<T>::BN, BK = BuildTile<T>::BK;
  constexpr int P = Pitch<T, BK>::value, MI = BM / 32, NI = BN / 32;
  constexpr int NA = (BM / 2) * BK / NT, NB = BN * BK / NT;
  __shared__ __attribute__((aligned(16))) T As[BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[BN * P];
  typedef typename Cplx<T>::type C2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nk = n1 * n2 * n3, nvv = nv * nv;
  const int q = q0 + blockIdx.z;
  const int64_t M = int64_t(nk) * nvv;  // complex rows
  const int64_t r0 = int64_t(blockIdx.y) * (BM / 2);
  const int c0 = blockIdx.x * BN;
  const T *wq = w + int64_t(qorb[q]) * nmb * nmb;
  const C2 *arow[NA];
  T asgn[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int64_t r = r0 + (tid + NT * u) / BK;
    arow[u] = nullptr;
    asgn[u] = T(1);
    if (r < M) {
      const int k = int(r / nvv), vv = int(r % nvv), v = vv / nv, v2 = vv % nv;
      const int kq = kminus(k, q, n1, n2, n3);
      const int64_t p = int64_t(k) * nk + kq;
      const int cls = pidx[p];
      const bool cj = pconj[p] != 0;
      const int s1 = cj ? v2 : v, s2 = cj ? v : v2;
      arow[u] = reinterpret_cast<const C2 *>(mv) + ((int64_t(cls) * nv + s1) * nv + s2) * nmb;
      asgn[u] = cj ? T(-1) : T(1);
    }
  }
  typename Mfma<T>::acc_t acc[MI][NI];
  acc_zero<T, MI, NI>(acc);
  const int wm0 = (wv >> 1) * (BM / 2), wn0 = (wv & 1) * (BN / 2);
  for (int j0 = 0; j0 < nmb; j0 += BK) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + NT * u, r = it / BK, j = it % BK, J = j0 + j;
      C2 x = {T(0), T(0)};
      if (arow[u] && J < nmb) x = arow[u][J];
      As[(2 * r) * P + j] = x.x;
      As[(2 * r + 1) * P + j] = asgn[u] * x.y;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + NT * u, c = it / BK, j = it % BK, I = c0 + c, J = j0 + j;
      Bs[c * P + j] = (I < nmb && J < nmb) ? wq[int64_t(I) * nmb + J] : T(0);
    }
    __syncthreads();
    mfma_slab<T, MI, NI, BK>(acc, As, Bs, wm0, wn0, lane);
    __syncthreads();
  }
  C2 *out = reinterpret_cast<C2 *>(Tq) + int64_t(blockIdx.z) * M * nmb;
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int I = c0 + wn0 + 16 * ni + r16;
      const int64_t r = r0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (r + h < M && I < nmb)
          out[(r + h) * nmb + I] = C2{acc[mi][ni][2 * h], acc[mi][ni][2 * h + 1]};
    }
}

// ---------------------------------------------------------------------------
// direct term, stage 2: one wave per pair (k, k-q)
//   D[(c,c')][(v,v')] = sum_I conj(Mc(k,k-q)[c,c',I]) T_q[(k,v,v')][I]
//   H[(k v c),(k-q v' c')] -= D / N_k
// ---------------------------------------------------------------------------
constexpr int D_MB = 5;  // row blocks: 2 nc^2 <= 80
constexpr int D_NB = 3;  // column blocks: nv^2 <= 48

template <typename T>
__global__ __launch_bounds__(NT) void k_direct_d(int n1, int n2, int n3, int nv, int nc, int nmb,
                                                 int q0, const int32_t *__restrict__ pidx,
                                                 const uint8_t *__restrict__ pconj,
                                                 const T *__restrict__ mc,
                                                 const T *__restrict__ Tq, T *__restrict__ H,
                                                 int64_t ldh, double scale) {
  typedef typename Cplx<T>::type C2;
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nk = n1 * n2 * n3, nvv = nv * nv, ncc = nc * nc;
  const int k = blockIdx.x * (NT / 64) + wv;
  if (k >= nk) return;
  const int q = q0 + blockIdx.y;
  const int kq = kminus(k, q, n1, n2, n3);
  const int64_t p = int64_t(k) * nk + kq;
  const int cls = pidx[p];
  const bool cj = pconj[p] != 0;
  const T sg = cj ? T(-1) : T(1);
  const int mb = (2 * ncc + 15) / 16, nb = (nvv + 15) / 16;
  const int r16 = lane & 15, g = lane >> 4;
  // per-lane source rows
  const C2 *arow[D_MB];
  int at[D_MB];
#pragma unroll
  for (int mi = 0; mi < D_MB; ++mi) {
    const int R = 16 * mi + Mfma<T>::arow(r16);
    arow[mi] = nullptr;
    at[mi] = R & 1;
    if (mi < mb && R < 2 * ncc) {
      const int cc = R >> 1, c = cc / nc, c2 = cc % nc;
      const int s1 = cj ? c2 : c, s2 = cj ? c : c2;
      arow[mi] = reinterpret_cast<const C2 *>(mc) + ((int64_t(cls) * nc + s1) * nc + s2) * nmb;
    }
  }
  const C2 *brow[D_NB];
  const C2 *tbase = reinterpret_cast<const C2 *>(Tq) + int64_t(blockIdx.y) * nk * nvv * nmb;
#pragma unroll
  for (int ni = 0; ni < D_NB; ++ni) {
    const int C = 16 * ni + r16;
    brow[ni] = (ni < nb && C < nvv) ? tbase + (int64_t(k) * nvv + C) * nmb : nullptr;
  }
  acc_t acc[D_MB][D_NB];
#pragma unroll
  for (int mi = 0; mi < D_MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < D_NB; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[mi][ni][j] = T(0);
  for (int i0 = 0; i0 < nmb; i0 += 8) {
    const int I = i0 + 2 * g;
    typename Mfma<T>::frag_t af[D_MB], bf[D_NB];
#pragma unroll
    for (int mi = 0; mi < D_MB; ++mi) {
      C2 x0 = {T(0), T(0)}, x1 = {T(0), T(0)};
      if (arow[mi]) {
        if (I < nmb) x0 = arow[mi][I];
        if (I + 1 < nmb) x1 = arow[mi][I + 1];
      }
      const T a0 = x0.x, b0 = sg * x0.y, a1 = x1.x, b1 = sg * x1.y;
      if (at[mi] == 0) {
        af[mi][0] = a0; af[mi][1] = b0; af[mi][2] = a1; af[mi][3] = b1;
      } else {
        af[mi][0] = -b0; af[mi][1] = a0; af[mi][2] = -b1; af[mi][3] = a1;
      }
    }
#pragma unroll
    for (int ni = 0; ni < D_NB; ++ni) {
      C2 y0 = {T(0), T(0)}, y1 = {T(0), T(0)};
      if (brow[ni]) {
        if (I < nmb) y0 = brow[ni][I];
        if (I + 1 < nmb) y1 = brow[ni][I + 1];
      }
      bf[ni][0] = y0.x; bf[ni][1] = y0.y; bf[ni][2] = y1.x; bf[ni][3] = y1.y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int mi = 0; mi < D_MB; ++mi)
#pragma unroll
        for (int ni = 0; ni < D_NB; ++ni)
          if (mi < mb && ni < nb) acc[mi][ni] = Mfma<T>::mma(af[mi][i], bf[ni][i], acc[mi][ni]);
  }
  C2 *Hc = reinterpret_cast<C2 *>(H);
#pragma unroll
  for (int mi = 0; mi < D_MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < D_NB; ++ni) {
      if (mi >= mb || ni >= nb) continue;
      const int C = 16 * ni + r16;
      if (C >= nvv) continue;
      const int v = C / nv, v2 = C % nv;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cc = (16 * mi + 4 * g) / 2 + h;
        if (cc >= ncc) continue;
        const int c = cc / nc, c2 = cc % nc;
        const int64_t a = (int64_t(k) * nv + v) * nc + c;
        const int64_t b = (int64_t(kq) * nv + v2) * nc + c2;
        C2 hv = Hc[a * ldh + b];
        hv.x -= T(scale * double(acc[mi][ni][2 * h]));
        hv.y -= T(scale * double(acc[mi][ni][2 * h + 1]));
        Hc[a * ldh + b] = hv;
      }
    }
}

// Stores one 16-byte vector of complex Mv values as separate re / im LDS rows.
template <int VEC> __device__ __forceinline__ void split_store(float4 x, float *dre, float *dim,
                                                               int c, float sg) {
  *reinterpret_cast<float2 *>(dre + 2 * c) = float2{x.x, x.z};
  *reinterpret_cast<float2 *>(dim + 2 * c) = float2{sg * x.y, sg * x.w};
}
template <int VEC> __device__ __forceinline__ void split_store(double2 x, double *dre,
                                                               double *dim, int c, double sg) {
  dre[c] = x.x;
  dim[c] = sg * x.y;
}

// ---------------------------------------------------------------------------
// direct term, fused: one workgroup per (q, KC consecutive k), all Nmb rows.
//   stage 1  T^T[I][(k, t, vv')] = sum_J W_q[I][J] Re/Im(Mv(k, k-q)[vv'][J])
//            wave w owns rows I in [w 16 MI, (w+1) 16 MI), all KC k's;
//   stage 2  D[cc'][vv'] = sum_I conj(Mc(k, k-q)[cc'][I]) T[vv'][I]
//            straight from the accumulators: in the MFMA output layout lane
//            (g, c) holds T^T rows 4g + j at column c, which is exactly the
//            B operand of a 16x16x4 step whose K slot g is row 4g + j.  Each
//            wave contracts its own I range; the four partial D are summed in
//            LDS and subtracted from H.  T never leaves the registers.
// Requires nmb = 64 MI, nv^2 <= 16, nc^2 <= 16 NCB (NCB <= 3 row blocks of
// stage 2, a template parameter so that unused accumulators take no registers).
// ---------------------------------------------------------------------------
// SEED: the workgroup takes its q and KC k points from a work list (one k per
// pair-orbit representative, -1 for padding) and writes the blocks D of the
// representatives to drep[orbit][cc'][vv'] instead of subtracting them from H.
template <typename T, int MI, int KC, bool SEED, int NCB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : (MI >= 6 ? 1 : 2), 8))) void k_direct_fused(int n1, int n2, int n3, int nv, int nc,
                                                     const int32_t *__restrict__ qorb,
                                                     const int32_t *__restrict__ pidx,
                                                     const uint8_t *__restrict__ pconj,
                                                     const T *__restrict__ mv,
                                                     const T *__restrict__ mc,
                                                     const T *__restrict__ w, T *__restrict__ H,
                                                     int64_t ldh, double scale,
                                                     const int32_t *__restrict__ items,
                                                     T *__restrict__ drep) {
  constexpr int BK = 16, P = Pitch<T, BK>::value;  // 16-deep slabs: two workgroups per CU
  constexpr int NMB = 64 * MI;             // rows of W handled by the workgroup
  constexpr int NI = 2 * KC;               // column blocks: (k, re/im)
  constexpr int NCOL = 16 * NI;            // B rows in LDS
  constexpr int VEC = 16 / sizeof(T);      // elements per 16-byte load
  constexpr int NA = NMB * BK / VEC / NT;  // A loads per thread per slab
  constexpr int BPR = 2 * BK / VEC;        // 16-byte loads per B row per slab (BK complex)
  constexpr int NB = KC * 16 * BPR / NT;   // B loads per thread per slab
  static_assert(NA >= 1 && NB >= 1, "tile too small");
  constexpr int STAGE = (NMB + NCOL) * P;  // staging elements
  constexpr int RED = 4 * NCB * 16 * 16 * 2;
  constexpr bool SWZ = sizeof(T) == 4;      // swizzled FP32 rows (see below)
  constexpr int PP = SWZ ? BK : P;          // LDS row pitch
  constexpr int LDSN = SWZ ? (NMB + NCOL) * PP : STAGE;
  static_assert(!SWZ || BK == 16, "the FP32 swizzle assumes four chunks per row");
  auto swz = [](int row, int chunk) { return SWZ ? (chunk ^ ((row >> 1) & 3)) : chunk; };
  __shared__ __attribute__((aligned(16))) T lds[LDSN > RED ? LDSN : RED];
  T *As = lds, *Bs = lds + NMB * PP;
  typedef typename Cplx<T>::type C2;
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Mfma<T>::frag_t frag_t;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nk = n1 * n2 * n3, nvv = nv * nv, ncc = nc * nc;
  const int nmb = NMB;
  const int32_t *item = SEED ? items + int64_t(blockIdx.x) * (1 + 2 * KC) : nullptr;
  const int q = SEED ? item[0] : int(blockIdx.y);
  const int k0 = blockIdx.x * KC;
  auto kof = [&](int kk) { return SEED ? item[1 + kk] : k0 + kk; };
  auto kok = [&](int k) { return SEED ? k >= 0 : k < nk; };
  const T *wq = w + int64_t(qorb[q]) * nmb * nmb;
  // B-row sources: row = kk * 16 + vv' (re and im rows of one complex row)
  const C2 *brow[NB];
  T bsgn[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int it = tid + NT * u, row = it / BPR, kk = row / 16, vv = row % 16;
    const int k = kof(kk);
    brow[u] = nullptr;
    bsgn[u] = T(1);
    if (kok(k) && vv < nvv) {
      const int kq = kminus(k, q, n1, n2, n3);
      const int64_t p = int64_t(k) * nk + kq;
      const bool cj = pconj[p] != 0;
      const int v = vv / nv, v2 = vv % nv;
      const int s1 = cj ? v2 : v, s2 = cj ? v : v2;
      brow[u] = reinterpret_cast<const C2 *>(mv) +
                ((int64_t(pidx[p]) * nv + s1) * nv + s2) * nmb;
      bsgn[u] = cj ? T(-1) : T(1);
    }
  }
  acc_t acc[MI][NI];
  acc_zero<T, MI, NI>(acc);
  const int wm0 = wv * 16 * MI;
  // per-thread load slots of the W rows (A) and the split Mv rows (B)
  typedef typename std::conditional<VEC == 4, float4, double2>::type V16;
  // LDS rows of 16-byte chunks.  FP32: no padding, chunk c of row r stored at
  // c ^ ((r >> 1) & 3), so the eight lanes of one b128 access (eight rows at
  // one chunk for the MFMA fragments, two rows at four chunks for the stores)
  // hit eight distinct bank groups.  FP64: rows padded by one chunk.
  // thread slot u covers row tid / 4 + RSTEP u, chunk tid % 4: one base
  // address plus constant offsets (the swizzle does not change with u)
  constexpr int RSTEP = NT / (BK / VEC);
  static_assert(RSTEP % 8 == 0, "the FP32 swizzle must repeat every RSTEP rows");
  const T *wrow0;
  int aoff0;
  {
    const int row = tid / (BK / VEC), c = tid % (BK / VEC);
    wrow0 = wq + int64_t(row) * nmb + c * VEC;
    aoff0 = row * PP + swz(row, c) * VEC;
  }
  // a B row without data reads the first entries of mv (global memory, so
  // every load is a global one) and is zeroed by bmask
  const C2 *bsrc[NB];
  int bstride[NB], boff[NB], boff2[NB];
  T bmask[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int it = tid + NT * u, row = it / BPR, c = it % BPR, kk = row / 16, vv = row % 16;
    bsrc[u] = (brow[u] ? brow[u] : reinterpret_cast<const C2 *>(mv)) + (VEC == 4 ? 2 * c : c);
    bstride[u] = brow[u] ? 1 : 0;
    bmask[u] = brow[u] ? T(1) : T(0);
    const int r0 = (2 * kk) * 16 + vv, r1 = r0 + 16;  // real and imaginary rows
    if (VEC == 4) {  // two complex = four floats: the re pair and the im pair
      boff[u] = r0 * PP + swz(r0, c >> 1) * 4 + 2 * (c & 1);
      boff2[u] = r1 * PP + swz(r1, c >> 1) * 4 + 2 * (c & 1);
    } else {
      boff[u] = r0 * PP + c;
      boff2[u] = r1 * PP + c;
    }
  }
  // Several workgroups per CU hide the load latency better than an
  // in-register prefetch of the next slab or a second LDS buffer, which cost
  // registers and LDS and so workgroups per CU (measured: 0.47-0.50 of peak
  // against 0.68).
  const int r = lane & 15, g = lane >> 4;
  for (int j0 = 0; j0 < nmb; j0 += BK) {
    V16 ra[NA], rb[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u)
      ra[u] = *reinterpret_cast<const V16 *>(wrow0 + int64_t(u) * RSTEP * NMB + j0);
#pragma unroll
    for (int u = 0; u < NB; ++u) rb[u] = *reinterpret_cast<const V16 *>(bsrc[u] + bstride[u] * j0);
#pragma unroll
    for (int u = 0; u < NA; ++u) *reinterpret_cast<V16 *>(As + aoff0 + u * RSTEP * PP) = ra[u];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      V16 x = rb[u];
      if constexpr (VEC == 4) {
        x.x *= bmask[u]; x.y *= bmask[u]; x.z *= bmask[u]; x.w *= bmask[u];
      } else {
        x.x *= bmask[u]; x.y *= bmask[u];
      }
      split_store<VEC>(x, Bs + boff[u], Bs + boff2[u], 0, bsgn[u]);
    }
    __syncthreads();
    if (SWZ) {
      // B fragments held for the slab, A fragments one row block at a time
      // (fewer live registers: four waves per SIMD instead of three)
      frag_t fb[NI];
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const int row = 16 * ni + r;
        fb[ni] = lds_frag<T>(Bs + row * PP + swz(row, g) * 4);
      }
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) {
        const int row = wm0 + 16 * mi + r;
        const frag_t fa = lds_frag<T>(As + row * PP + swz(row, g) * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int ni = 0; ni < NI; ++ni)
            acc[mi][ni] = Mfma<T>::mma(fa[i], fb[ni][i], acc[mi][ni]);
      }
    } else {
      mfma_slab<T, MI, NI, BK>(acc, As, Bs, wm0, 0, lane);
    }
    __syncthreads();
  }
  // ---- stage 2 ----
  const int r16 = r;
  const int ncb = (ncc + 15) / 16;
  C2 *red = reinterpret_cast<C2 *>(lds);  // [4][NCB*16][16]
  C2 *Hc = reinterpret_cast<C2 *>(H);
  // Mc row (c, c') of this lane's A row in each c c' block: as stored (low
  // 16 bits) and band-swapped for a conjugated class (high 16 bits); -1 past
  // the last pair (that row reads the class's first row and is zeroed)
  int mrow[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int cc = 16 * cb + Mfma<T>::arow(r16), c = cc / nc, c2 = cc % nc;
    mrow[cb] = cc < ncc ? ((c2 * nc + c) << 16) | (c * nc + c2) : -1;
  }
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = kof(kk);
    acc_t dre[NCB], dim[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int j = 0; j < 4; ++j) dre[cb][j] = dim[cb][j] = T(0);
    int kq = 0;
    if (kok(k)) {
      kq = kminus(k, q, n1, n2, n3);
      const int64_t p = int64_t(k) * nk + kq;
      const bool cj = pconj[p] != 0;
      const T sg = cj ? T(-1) : T(1);
      const int cls = pidx[p];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if (cb >= ncb) break;
        const int mr = mrow[cb] < 0 ? 0 : cj ? mrow[cb] >> 16 : mrow[cb] & 0xffff;
        const T am = mrow[cb] < 0 ? T(0) : T(1), sgm = sg * am;
        const C2 *arowp = reinterpret_cast<const C2 *>(mc) + (int64_t(cls) * ncc + mr) * nmb;
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) {
          const int I0 = wm0 + 16 * mi + 4 * g;
          // four consecutive entries, 16-byte aligned (nmb and I0 multiples of 4)
          C2 m[4];
          const V16 *m16 = reinterpret_cast<const V16 *>(arowp + I0);
          if constexpr (VEC == 4) {
            const V16 a = m16[0], b = m16[1];
            m[0] = C2{T(a.x), T(a.y)};
            m[1] = C2{T(a.z), T(a.w)};
            m[2] = C2{T(b.x), T(b.y)};
            m[3] = C2{T(b.z), T(b.w)};
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) memcpy(&m[j], &m16[j], sizeof(C2));
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const T are = am * m[j].x, aim = sgm * m[j].y;   // Mc = are + i aim
            const T tre = acc[mi][2 * kk][j], tim = acc[mi][2 * kk + 1][j];
            // conj(Mc) T = (are tre + aim tim) + i (are tim - aim tre)
            dre[cb] = Mfma<T>::mma(are, tre, dre[cb]);
            dre[cb] = Mfma<T>::mma(aim, tim, dre[cb]);
            dim[cb] = Mfma<T>::mma(are, tim, dim[cb]);
            dim[cb] = Mfma<T>::mma(-aim, tre, dim[cb]);
          }
        }
      }
    }
    // partial D of this wave -> LDS, then the sum over waves -> H
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        red[(wv * NCB * 16 + 16 * cb + 4 * g + j) * 16 + r16] = C2{dre[cb][j], dim[cb][j]};
    __syncthreads();
    if (kok(k)) {
      for (int e = tid; e < ncc * nvv; e += NT) {
        const int cc = e / nvv, vv = e % nvv;
        C2 sum = {T(0), T(0)};
#pragma unroll
        for (int w4 = 0; w4 < 4; ++w4) {
          const C2 x = red[(w4 * NCB * 16 + cc) * 16 + vv];
          sum.x += x.x;
          sum.y += x.y;
        }
        if (SEED) {
          reinterpret_cast<C2 *>(drep)[int64_t(item[1 + KC + kk]) * ncc * nvv + e] = sum;
          continue;
        }
        const int c = cc / nc, c2 = cc % nc, v = vv / nv, v2 = vv % nv;
        const int64_t a = (int64_t(k) * nv + v) * nc + c;
        const int64_t b = (int64_t(kq) * nv + v2) * nc + c2;
        C2 hv = Hc[a * ldh + b];
        hv.x -= T(scale * double(sum.x));
        hv.y -= T(scale * double(sum.y));
        Hc[a * ldh + b] = hv;
      }
    }
    __syncthreads();
  }
}

template <typename T, int KC, bool SEED = false>
int32_t launch_fused(int MI, dim3 g, hipStream_t s, const bse_problem *p, void *H, int64_t ldh,
                     double scale, const int32_t *items = nullptr, void *drep = nullptr) {
  const int ncb = (p->nc * p->nc + 15) / 16;
  if (ncb < 1 || ncb > 3) return fail(BSE_EUNSUPPORTED, "fused direct kernel: nc^2 <= 48");
#define BSE_FUSED_NCB(M, C)                                                                   \
  BSE_LAUNCH(SEED ? "k_direct_seed" : "k_direct_fused", (k_direct_fused<T, M, KC, SEED, C>),  \
             g, dim3(NT), 0, s, p->grid[0], p->grid[1], p->grid[2], p->nv, p->nc, p->qorb,  \
             p->pidx, p->pconj, (const T *)p->mv, (const T *)p->mc, (const T *)p->w,        \
             (T *)H, ldh, scale, items, (T *)drep)
#define BSE_FUSED_CASE(M)                                                                     \
  case M:                                                                                   \
    if (ncb == 1) BSE_FUSED_NCB(M, 1);                                                      \
    else if (ncb == 2) BSE_FUSED_NCB(M, 2);                                                 \
    else BSE_FUSED_NCB(M, 3);                                                               \
    break;
  switch (MI) {
    BSE_FUSED_CASE(1)
    BSE_FUSED_CASE(2)
    BSE_FUSED_CASE(3)
    BSE_FUSED_CASE(4)
    BSE_FUSED_CASE(5)
    BSE_FUSED_CASE(6)
    default:
      return fail(BSE_EUNSUPPORTED, "fused direct kernel: nmb = 64 MI with MI <= 6");
  }
#undef BSE_FUSED_CASE
#undef BSE_FUSED_NCB
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// seed-mode assembly: every H element from the per-orbit pieces
//   H[(k v c),(k' v' c')] = X[(o(k) v c),(o(k') v' c')] + delta (E_c - E_v)
//                           - scale D[porb(k,k')][(c c')][(v v')]
// X: exchange between k-orbit representatives, D: direct blocks of the
// pair-orbit representatives.  One row per workgroup row, columns coalesced.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_seed_assemble(int nk, int nv, int nc,
                                                      const int32_t *__restrict__ korb,
                                                      const int32_t *__restrict__ porb,
                                                      const double *__restrict__ ev,
                                                      const double *__restrict__ ec,
                                                      const T *__restrict__ xs, int64_t ldx,
                                                      const T *__restrict__ drep,
                                                      T *__restrict__ H, int64_t ldh,
                                                      double scale) {
  typedef typename Cplx<T>::type C2;
  const int nb = nv * nc, ncc = nc * nc, nvv = nv * nv;
  const int64_t N = int64_t(nk) * nb;
  const int64_t nbx = (N + NT - 1) / NT;  // workgroups per row
  const int64_t a = int64_t(blockIdx.x) / nbx;
  const int64_t b = (int64_t(blockIdx.x) % nbx) * NT + threadIdx.x;
  if (b >= N) return;
  const int k = int(a / nb), ia = int(a % nb), v = ia / nc, c = ia % nc;
  const int k2 = int(b / nb), ib = int(b % nb), v2 = ib / nc, c2 = ib % nc;
  const C2 x = reinterpret_cast<const C2 *>(xs)[(int64_t(korb[k]) * nb + ia) * ldx +
                                                int64_t(korb[k2]) * nb + ib];
  const int64_t o = porb[int64_t(k) * nk + k2];
  const C2 d = reinterpret_cast<const C2 *>(drep)[(o * ncc + c * nc + c2) * nvv + v * nv + v2];
  double re = double(x.x) - scale * double(d.x), im = double(x.y) - scale * double(d.y);
  if (a == b) re += ec[int64_t(k) * nc + c] - ev[int64_t(k) * nv + v];
  reinterpret_cast<C2 *>(H)[a * ldh + b] = C2{T(re), T(im)};
}

bool fused_ok(const bse_problem *p) { return fused_shape(p->nmb, p->nv, p->nc); }

int32_t check_problem(const bse_problem *p, int32_t prec) {
  if (!p) return fail(BSE_EINVAL, "problem is NULL");
  if (prec != BSE_FP64 && prec != BSE_FP32 && prec != BSE_BF16X3)
    return fail(BSE_EINVAL, "unknown precision %d", prec);
  if ((prec == BSE_FP64) != (p->in_fp64 != 0))
    return fail(BSE_EINVAL, "input element type does not match the precision");
  if (p->grid[0] < 1 || p->grid[1] < 1 || p->grid[2] < 1) return fail(BSE_ESHAPE, "bad grid");
  const int64_t nk = int64_t(p->grid[0]) * p->grid[1] * p->grid[2];
  if (nk * nk >= (int64_t(1) << 31)) return fail(BSE_ESHAPE, "nk too large");
  if (p->nv < 1 || p->nc < 1 || p->nmb < 1) return fail(BSE_ESHAPE, "nv, nc, nmb must be >= 1");
  if (p->nv * p->nv > 16 * D_NB || 2 * p->nc * p->nc > 16 * D_MB)
    return fail(BSE_EUNSUPPORTED, "nv <= 6 and nc <= 6 are supported (got %d, %d)", p->nv, p->nc);
  if (p->nkorb < 1 || p->ncls < 1 || p->nqorb < 1) return fail(BSE_ESHAPE, "empty orbit tables");
  if (!p->korb || !p->qorb || !p->pidx || !p->pconj || !p->ev || !p->ec || !p->vdiag || !p->mx ||
      !p->mv || !p->mc || !p->w)
    return fail(BSE_EINVAL, "NULL device pointer in problem");
  return BSE_OK;
}

size_t per_q_bytes(const bse_problem *p, int32_t prec) {
  const size_t el = prec == BSE_FP64 ? 16 : 8;
  const size_t nk = size_t(p->grid[0]) * p->grid[1] * p->grid[2];
  return nk * size_t(p->nv) * p->nv * p->nmb * el;
}

}  // namespace

// used by other translation units (BF16 split form)
int32_t build_check_problem(const bse_problem *p, int32_t prec) { return check_problem(p, prec); }

size_t build_bf16x3_ws(const bse_problem *p);

}  // namespace bse

using namespace bse;

extern "C" size_t bse_build_ws_min(const bse_problem *p, int32_t prec) {
  if (check_problem(p, prec)) return 0;
  if (prec == BSE_BF16X3) return build_bf16x3_ws(p);
  if (fused_ok(p)) return 256;  // the fused direct terms need no buffer
  return per_q_bytes(p, prec);
}

extern "C" size_t bse_build_ws(const bse_problem *p, int32_t prec) {
  if (check_problem(p, prec)) return 0;
  if (prec == BSE_BF16X3) return build_bf16x3_ws(p);
  if (fused_ok(p)) return 256;
  const size_t pq = per_q_bytes(p, prec);
  const size_t nk = size_t(p->grid[0]) * p->grid[1] * p->grid[2];
  const size_t cap = size_t(1) << 30;  // 1 GiB of q-batch buffer is plenty to saturate
  return pq * std::max<size_t>(1, std::min(nk, cap / pq));
}

extern "C" int32_t bse_build(const bse_problem *p, int32_t prec, void *H, int64_t ldh, void *ws,
                             size_t ws_bytes, bse_stream stream) {
  int32_t st = check_problem(p, prec);
  if (st) return st;
  if (prec == BSE_BF16X3) return build_bf16x3(p, H, ldh, ws, ws_bytes, stream);
  const int n1 = p->grid[0], n2 = p->grid[1], n3 = p->grid[2];
  const int nk = n1 * n2 * n3;
  const int64_t N = int64_t(nk) * p->nv * p->nc;
  if (!H) return fail(BSE_EINVAL, "H is NULL");
  if (ldh < N) return fail(BSE_ESHAPE, "ldh %lld < N %lld", (long long)ldh, (long long)N);
  const bool fused = fused_ok(p);
  const size_t pq = per_q_bytes(p, prec);
  if (!fused && (!ws || ws_bytes < pq))
    return fail(BSE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, pq);
  const int qb = fused ? 1 : int(std::min<size_t>(nk, ws_bytes / pq));
  hipStream_t s = (hipStream_t)stream;
  const double inv_nk = 1.0 / nk;
  auto launch = [&](auto tag) -> int32_t {
    typedef decltype(tag) T;
    constexpr int BM = BuildTile<T>::BM, BN = BuildTile<T>::BN;
    dim3 gx((unsigned)((N + BN - 1) / BN), (unsigned)((2 * N + BM - 1) / BM));
    if (gx.y > 65535u) return fail(BSE_ESHAPE, "N too large for the exchange grid");
    BSE_LAUNCH("k_exchange", k_exchange<T>, gx, dim3(NT), 0, s, nk, p->nv, p->nc, p->nmb, p->korb,
                       (const T *)p->mx, p->vdiag, p->ev, p->ec, (T *)H, ldh, 2.0 * inv_nk, 1);
    BSE_HIP_CHECK(hipGetLastError());
    if (fused) {
      constexpr int KC = 2;  // k points per workgroup
      dim3 gf((unsigned)((nk + KC - 1) / KC), (unsigned)nk);
      return launch_fused<T, KC>(p->nmb / 64, gf, s, p, H, ldh, inv_nk);
    }
    const int64_t M = 2 * int64_t(nk) * p->nv * p->nv;
    for (int q0 = 0; q0 < nk; q0 += qb) {
      const int nq = std::min(qb, nk - q0);
      dim3 g1((unsigned)((p->nmb + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)nq);
      BSE_LAUNCH("k_direct_t", k_direct_t<T>, g1, dim3(NT), 0, s, n1, n2, n3, p->nv, p->nmb, q0,
                         p->qorb, p->pidx, p->pconj, (const T *)p->mv, (const T *)p->w, (T *)ws);
      BSE_HIP_CHECK(hipGetLastError());
      dim3 g2((unsigned)((nk + 3) / 4), (unsigned)nq);
      BSE_LAUNCH("k_direct_d", k_direct_d<T>, g2, dim3(NT), 0, s, n1, n2, n3, p->nv, p->nc, p->nmb, q0,
                         p->pidx, p->pconj, (const T *)p->mc, (const T *)ws, (T *)H, ldh, inv_nk);
      BSE_HIP_CHECK(hipGetLastError());
    }
    return BSE_OK;
  };
  if (prec == BSE_FP64) return launch(double(0));
  return launch(float(0));
}

// ===========================================================================
// seed (symmetry-accelerated) construction: the direct term is contracted for
// one representative pair per pair orbit (Sec. III.C.2: pairs related by an
// operation share their interaction elements), the exchange for one k point
// per k orbit, and H is assembled from these pieces.
// ===========================================================================
#include <map>
#include <mutex>
#include <vector>

namespace bse {
namespace {
constexpr int SEED_KC = 2;

struct SeedPlan {
  bse_problem p{};
  int32_t prec = 0;
  int nk = 0, nkorb = 0, nporb = 0, nitems = 0;
  int32_t *items = nullptr, *porb = nullptr, *ident = nullptr;
  void *xs = nullptr, *drep = nullptr;
  int64_t ldx = 0;
};
std::mutex g_seed_mu;
std::map<int64_t, SeedPlan> g_seeds;
int64_t g_seed_next = 1;

struct SeedLayout {
  size_t items, porb, ident, xs, drep, total;
};

SeedLayout seed_layout(const bse_problem *p, int32_t prec, int nkorb, int nporb, int nitems) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t el = prec == BSE_FP64 ? 16 : 8;
  const size_t nk = size_t(p->grid[0]) * p->grid[1] * p->grid[2];
  const size_t nb = size_t(p->nv) * p->nc;
  SeedLayout L;
  size_t off = 0;
  L.items = off;
  off += al(size_t(nitems) * (1 + 2 * SEED_KC) * 4);
  L.porb = off;
  off += al(nk * nk * 4);
  L.ident = off;
  off += al(size_t(nkorb) * 4);
  L.xs = off;
  off += al(size_t(nkorb) * nb * nkorb * nb * el);
  L.drep = off;
  off += al(size_t(nporb) * p->nc * p->nc * p->nv * p->nv * el);
  L.total = off;
  return L;
}

// tables of (group, grid) through the library's own host builder
int32_t seed_tables(int32_t group, const bse_problem *p, std::vector<int32_t> &porb,
                    std::vector<int32_t> &porb_rep, std::vector<int32_t> &korb, int &nkorb) {
  bse_dims d;
  int32_t st = bse_dims_get(group, p->grid, &d);
  if (st) return st;
  std::vector<int32_t> kperm(size_t(d.nops) * d.nk), krep(d.nkorb), pidx(size_t(d.nk) * d.nk),
      crep(d.ncls);
  std::vector<uint8_t> pconj(size_t(d.nk) * d.nk), css(d.ncls);
  porb.assign(size_t(d.nk) * d.nk, 0);
  porb_rep.assign(d.nporb, 0);
  korb.assign(d.nk, 0);
  bse_tables t{kperm.data(), korb.data(), krep.data(), porb.data(), porb_rep.data(),
               pidx.data(), pconj.data(), crep.data(), css.data()};
  st = bse_tables_build(group, p->grid, &t);
  nkorb = d.nkorb;
  return st;
}

// work list: representatives grouped by q, KC per item
void seed_items(const bse_problem *p, const std::vector<int32_t> &porb_rep,
                std::vector<int32_t> &items) {
  const int n1 = p->grid[0], n2 = p->grid[1], n3 = p->grid[2], nk = n1 * n2 * n3;
  std::vector<std::vector<int>> byq(nk);
  for (int o = 0; o < int(porb_rep.size()); ++o) {
    const int k = porb_rep[o] / nk, k2 = porb_rep[o] % nk;
    const int a1 = k / (n2 * n3), a2 = (k / n3) % n2, a3 = k % n3;
    const int b1 = k2 / (n2 * n3), b2 = (k2 / n3) % n2, b3 = k2 % n3;
    const int q = (((a1 - b1 + n1) % n1) * n2 + (a2 - b2 + n2) % n2) * n3 + (a3 - b3 + n3) % n3;
    byq[q].push_back(o);
  }
  items.clear();
  for (int q = 0; q < nk; ++q)
    for (size_t i = 0; i < byq[q].size(); i += SEED_KC) {
      items.push_back(q);
      for (int kk = 0; kk < SEED_KC; ++kk)
        items.push_back(i + kk < byq[q].size() ? porb_rep[byq[q][i + kk]] / nk : -1);
      for (int kk = 0; kk < SEED_KC; ++kk)
        items.push_back(i + kk < byq[q].size() ? byq[q][i + kk] : 0);
    }
}
}  // namespace
}  // namespace bse

extern "C" size_t bse_seed_ws(int32_t group, const bse_problem *p, int32_t prec) {
  if (check_problem(p, prec) || prec == BSE_BF16X3 || !fused_ok(p)) return 0;
  std::vector<int32_t> porb, prep, korb;
  int nkorb = 0;
  if (seed_tables(group, p, porb, prep, korb, nkorb)) return 0;
  std::vector<int32_t> items;
  seed_items(p, prep, items);
  return seed_layout(p, prec, nkorb, int(prep.size()), int(items.size() / (1 + 2 * SEED_KC)))
      .total;
}

extern "C" int32_t bse_seed_plan(int32_t group, const bse_problem *p, int32_t prec, void *ws,
                                 size_t ws_bytes, int64_t *h_plan, bse_stream stream) {
  int32_t st = check_problem(p, prec);
  if (st) return st;
  if (prec == BSE_BF16X3) return fail(BSE_EUNSUPPORTED, "seed construction: FP32 or FP64");
  if (!fused_ok(p))
    return fail(BSE_EUNSUPPORTED, "seed construction needs Nmb = 64 m (m <= 6), nv <= 4, nc <= 6");
  if (!h_plan) return fail(BSE_EINVAL, "plan is NULL");
  SeedPlan P;
  std::vector<int32_t> porb, prep, korb;
  st = seed_tables(group, p, porb, prep, korb, P.nkorb);
  if (st) return st;
  if (P.nkorb != p->nkorb) return fail(BSE_EINVAL, "group does not match the problem's orbits");
  std::vector<int32_t> items;
  seed_items(p, prep, items);
  P.p = *p;
  P.prec = prec;
  P.nk = p->grid[0] * p->grid[1] * p->grid[2];
  P.nporb = int(prep.size());
  P.nitems = int(items.size() / (1 + 2 * SEED_KC));
  const SeedLayout L = seed_layout(p, prec, P.nkorb, P.nporb, P.nitems);
  if (!ws || ws_bytes < L.total)
    return fail(BSE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  char *base = (char *)ws;
  P.items = (int32_t *)(base + L.items);
  P.porb = (int32_t *)(base + L.porb);
  P.ident = (int32_t *)(base + L.ident);
  P.xs = base + L.xs;
  P.drep = base + L.drep;
  P.ldx = int64_t(P.nkorb) * p->nv * p->nc;
  std::vector<int32_t> ident(P.nkorb);
  for (int i = 0; i < P.nkorb; ++i) ident[i] = i;
  hipStream_t s = (hipStream_t)stream;
  BSE_HIP_CHECK(hipMemcpyAsync(P.items, items.data(), items.size() * 4, hipMemcpyHostToDevice, s));
  BSE_HIP_CHECK(hipMemcpyAsync(P.porb, porb.data(), porb.size() * 4, hipMemcpyHostToDevice, s));
  BSE_HIP_CHECK(hipMemcpyAsync(P.ident, ident.data(), ident.size() * 4, hipMemcpyHostToDevice, s));
  BSE_HIP_CHECK(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(g_seed_mu);
  const int64_t id = g_seed_next++;
  g_seeds[id] = P;
  *h_plan = id;
  return BSE_OK;
}

extern "C" int32_t bse_build_seed(int64_t plan, void *H, int64_t ldh, bse_stream stream) {
  SeedPlan P;
  {
    std::lock_guard<std::mutex> lk(g_seed_mu);
    auto it = g_seeds.find(plan);
    if (it == g_seeds.end()) return fail(BSE_EINVAL, "unknown seed plan %lld", (long long)plan);
    P = it->second;
  }
  const bse_problem *p = &P.p;
  const int64_t N = int64_t(P.nk) * p->nv * p->nc;
  if (H && ldh < N) return fail(BSE_ESHAPE, "ldh %lld < N %lld", (long long)ldh, (long long)N);
  hipStream_t s = (hipStream_t)stream;
  const double inv_nk = 1.0 / P.nk;
  auto launch = [&](auto tag) -> int32_t {
    typedef decltype(tag) T;
    constexpr int BM = BuildTile<T>::BM, BN = BuildTile<T>::BN;
    const int64_t Nx = P.ldx;
    dim3 gx((unsigned)((Nx + BN - 1) / BN), (unsigned)((2 * Nx + BM - 1) / BM));
    BSE_LAUNCH("k_exchange", k_exchange<T>, gx, dim3(NT), 0, s, P.nkorb, p->nv, p->nc, p->nmb,
               P.ident, (const T *)p->mx, p->vdiag, p->ev, p->ec, (T *)P.xs, P.ldx,
               2.0 * inv_nk, 0);
    BSE_HIP_CHECK(hipGetLastError());
    int32_t st = launch_fused<T, SEED_KC, true>(p->nmb / 64, dim3((unsigned)P.nitems), s, p,
                                                nullptr, 0, 0.0, P.items, P.drep);
    if (st) return st;
    if (!H) return BSE_OK;  // pieces only (bse_project_seed reads them)
    dim3 ga((unsigned)(N * ((N + NT - 1) / NT)));
    BSE_LAUNCH("k_seed_assemble", k_seed_assemble<T>, ga, dim3(NT), 0, s, P.nk, p->nv, p->nc,
               p->korb, P.porb, p->ev, p->ec, (const T *)P.xs, P.ldx, (const T *)P.drep,
               (T *)H, ldh, inv_nk);
    BSE_HIP_CHECK(hipGetLastError());
    return BSE_OK;
  };
  if (P.prec == BSE_FP64) return launch(double(0));
  return launch(float(0));
}

namespace bse {
int32_t seed_pieces(int64_t plan, SeedPieces *out) {
  std::lock_guard<std::mutex> lk(g_seed_mu);
  auto it = g_seeds.find(plan);
  if (it == g_seeds.end()) return fail(BSE_EINVAL, "unknown seed plan %lld", (long long)plan);
  const SeedPlan &P = it->second;
  out->p = P.p;
  out->prec = P.prec;
  out->nk = P.nk;
  out->porb = P.porb;
  out->xs = P.xs;
  out->drep = P.drep;
  out->ldx = P.ldx;
  return BSE_OK;
}
}  // namespace bse

extern "C" int32_t bse_seed_free(int64_t plan) {
  std::lock_guard<std::mutex> lk(g_seed_mu);
  if (!g_seeds.erase(plan)) return fail(BSE_EINVAL, "unknown seed plan %lld", (long long)plan);
  return BSE_OK;
}
