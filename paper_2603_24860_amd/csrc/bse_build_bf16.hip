// Split-BF16 ("bf16x3") form of the H build on MFMA 16x16x32 bf16.
//
// Same contractions as the FP32 kernels (Eq. (BSE-eigval) with Eq.
// (w_interaction2): diagonal + (2/N_k) exchange - (1/N_k) direct, q outermost,
// Sec. III.C.2), with every FP32 operand x split as
//   hi = bf16(x), lo = bf16(x - hi)        (round to nearest even)
// and each product x y taken as hi hi' + hi lo' + lo hi' (three MFMAs, FP32
// accumulation); the dropped lo lo' term is below 2^-16 |x y|, so an element
// carries about 1e-5 relative error instead of FP32's 1e-7.
//
// v_mfma_f32_16x16x32_bf16: lane l supplies 8 consecutive K values of row
// (l & 15) of A and of column (l & 15) of B for K slot group (l >> 4); the
// f32 output layout is the one of the 16x16x4 f32 instruction (lane l holds
// column l & 15, rows 4 (l >> 4) + j).  Any per-lane K assignment is valid as
// long as A and B use the same one, which the kernels below guarantee.
//
//   k_exchange_bf3   every H element: diagonal + exchange, complex GEMM with
//                    the (I, re/im) interleaved reduction index
//   k_direct_bf3     fused direct term: stage 1 T^T = W_q Mv^T staged in LDS as
//                    bf16 hi/lo; stage 2 conj(Mc) T from the stage-1
//                    accumulators of two adjacent 16-row tiles (8 K values per
//                    lane), split in registers
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_internal.h"
#include "build_common.h"
#include "mfma_tile.h"

namespace bse {

int32_t build_check_problem(const bse_problem *p, int32_t prec);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int NT = 256;

__device__ __forceinline__ f32x4 mma3(f32x4 acc, bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// x -> hi = bf16(x), lo = bf16(x - hi), two values per conversion
// (v_cvt_pk_bf16_f32 rounds to nearest even; bf16 -> f32 is exact)
template <int N, typename V>
__device__ __forceinline__ void splitn(const float *x, V &h, V &l) {
  static_assert(N % 2 == 0, "values are split in pairs");
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    const f32x2 v = {x[i], x[i + 1]};
    const bf16x2 hp = __builtin_convertvector(v, bf16x2);
    const bf16x2 lp = __builtin_convertvector(v - __builtin_convertvector(hp, f32x2), bf16x2);
    h[i] = hp[0];
    h[i + 1] = hp[1];
    l[i] = lp[0];
    l[i + 1] = lp[1];
  }
}

// ---------------------------------------------------------------------------
// exchange + diagonal (tile 128 real rows x 128 columns, K slab 32)
// ---------------------------------------------------------------------------
constexpr int XBM = 128, XBN = 128, XBK = 32, XP = XBK + 8;

__global__ __launch_bounds__(NT) void k_exchange_bf3(int nk, int nv, int nc, int nmb,
                                                     const int32_t *__restrict__ korb,
                                                     const float *__restrict__ mx,
                                                     const double *__restrict__ vdiag,
                                                     const double *__restrict__ ev,
                                                     const double *__restrict__ ec,
                                                     float *__restrict__ H, int64_t ldh,
                                                     double scale) {
  constexpr int KC = XBK / 2;                       // complex I per slab
  constexpr int NA = (XBM / 2) * KC / NT, NB = XBN * KC / NT;
  constexpr int MI = XBM / 32, NI = XBN / 32;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[XBM * XP], Al[XBM * XP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[XBN * XP], Bl[XBN * XP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = nv * nc;
  const int64_t N = int64_t(nk) * nb;
  const int64_t a0 = int64_t(blockIdx.y) * (XBM / 2), b0 = int64_t(blockIdx.x) * XBN;
  // rows past N read row 0 and are zeroed when staged, entries past nmb read
  // entry nmb - 1: every load is issued from an in-bounds address, none
  // behind a branch
  const float2 *arow[NA];
  const float2 *brow[NB];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int64_t a = a0 + (tid + NT * u) / KC, ac = a < N ? a : 0;
    arow[u] = reinterpret_cast<const float2 *>(mx) + (int64_t(korb[ac / nb]) * nb + ac % nb) * nmb;
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int64_t b = b0 + (tid + NT * u) / KC, bc = b < N ? b : 0;
    brow[u] = reinterpret_cast<const float2 *>(mx) + (int64_t(korb[bc / nb]) * nb + bc % nb) * nmb;
  }
  f32x4 acc[MI][NI];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = f32x4{0, 0, 0, 0};
  const int wm0 = (wv >> 1) * (XBM / 2), wn0 = (wv & 1) * (XBN / 2);
  const int r = lane & 15, g = lane >> 4;
  for (int i0 = 0; i0 < nmb; i0 += KC) {
    float2 xa[NA], xb[NB];
    float va[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int I = min(i0 + (tid + NT * u) % KC, nmb - 1);
      xa[u] = arow[u][I];
      va[u] = float(vdiag[I]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) xb[u] = brow[u][min(i0 + (tid + NT * u) % KC, nmb - 1)];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + NT * u;
      va[u] = (i0 + it % KC < nmb && a0 + it / KC < N) ? va[u] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + NT * u;
      const bool ok = i0 + it % KC < nmb && b0 + it / KC < N;
      xb[u] = float2{ok ? xb[u].x : 0.f, ok ? xb[u].y : 0.f};
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int it = tid + NT * u, rr = it / KC, i = it % KC;
      const float re = xa[u].x * va[u], im = xa[u].y * va[u];
      const float e0[2] = {re, im}, e1[2] = {im, -re};
      bf16x2 h0, l0, h1, l1;
      splitn<2>(e0, h0, l0);
      splitn<2>(e1, h1, l1);
      *reinterpret_cast<bf16x2 *>(Ah + (2 * rr) * XP + 2 * i) = h0;
      *reinterpret_cast<bf16x2 *>(Al + (2 * rr) * XP + 2 * i) = l0;
      *reinterpret_cast<bf16x2 *>(Ah + (2 * rr + 1) * XP + 2 * i) = h1;
      *reinterpret_cast<bf16x2 *>(Al + (2 * rr + 1) * XP + 2 * i) = l1;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = tid + NT * u, rr = it / KC, i = it % KC;
      const float e[2] = {xb[u].x, xb[u].y};
      bf16x2 h, l;
      splitn<2>(e, h, l);
      *reinterpret_cast<bf16x2 *>(Bh + rr * XP + 2 * i) = h;
      *reinterpret_cast<bf16x2 *>(Bl + rr * XP + 2 * i) = l;
    }
    __syncthreads();
    bf16x8 ah[MI], al[MI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) {
      ah[mi] = *reinterpret_cast<const bf16x8 *>(Ah + (wm0 + 16 * mi + r) * XP + 8 * g);
      al[mi] = *reinterpret_cast<const bf16x8 *>(Al + (wm0 + 16 * mi + r) * XP + 8 * g);
    }
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(Bh + (wn0 + 16 * ni + r) * XP + 8 * g);
      const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(Bl + (wn0 + 16 * ni + r) * XP + 8 * g);
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) acc[mi][ni] = mma3(acc[mi][ni], ah[mi], al[mi], bh, bl);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int64_t b = b0 + wn0 + 16 * ni + r;
      const int64_t a = a0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t aa = a + h;
        if (aa < N && b < N) {
          double re = scale * double(acc[mi][ni][2 * h]);
          const double im = scale * double(acc[mi][ni][2 * h + 1]);
          if (aa == b) {
            const int k = int(aa / nb), v = int((aa / nc) % nv), c = int(aa % nc);
            re += ec[int64_t(k) * nc + c] - ev[int64_t(k) * nv + v];
          }
          reinterpret_cast<float2 *>(H)[aa * ldh + b] = float2{float(re), float(im)};
        }
      }
    }
}

// ---------------------------------------------------------------------------
// W_q (FP32, [nqorb][nmb][nmb]) -> hi and lo BF16 planes of the same layout,
// once per build: every workgroup of a q reads all of W_q, so splitting it in
// the direct kernel would repeat the same conversions N_k / KC times.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_split_w(int64_t n4, const float4 *__restrict__ w,
                                                bf16x4 *__restrict__ wh, bf16x4 *__restrict__ wl) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n4; i += int64_t(gridDim.x) * NT) {
    const float4 x = w[i];
    const float e[4] = {x.x, x.y, x.z, x.w};
    bf16x4 h, l;
    splitn<4>(e, h, l);
    wh[i] = h;
    wl[i] = l;
  }
}

// ---------------------------------------------------------------------------
// direct term, fused: one workgroup per (q, KC consecutive k), all Nmb rows.
//   stage 1  T^T[I][(k, t, vv')] = sum_J W_q[I][J] Re/Im(Mv(k, k-q)[vv'][J]);
//            wave w owns rows I in [w 16 MI, (w+1) 16 MI).  W comes from its
//            hi/lo planes in 16-byte pieces, Mv is split here; the next K
//            slab is loaded while the MFMAs of the current one run.
//   stage 2  D[cc'][vv'] = sum_I conj(Mc(k, k-q)[cc'][I]) T[vv'][I]: lane
//            (g, c) of tiles mi and mi+1 holds T rows 16 mi + 4 g + j and
//            16 (mi+1) + 4 g + j (j < 4) at column c, the 8 K values of one
//            16x16x32 step; the A operand reads Mc at the same I.  The four
//            real products go to four accumulators, so neither the sign of a
//            conjugated class nor the minus of the imaginary part costs a
//            split of its own.
// LDS rows have a pitch of 80 bytes; the writers of one 16-row group take rows
// 4 j + b with j varying fastest across lanes, which puts the rows that one
// LDS write cycle covers 320 bytes apart (distinct banks for 32 and for 64
// banks of 4 bytes); the 16-byte MFMA reads of rows r16 = 0..15 are spread by
// the 80-byte pitch.
// Requires nmb = 64 MI, nv^2 <= 16, nc^2 <= 48, KC = 2.
// ---------------------------------------------------------------------------
template <int MI, int KC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MI <= 4 ? 3 : 2, 8))) void k_direct_bf3(int n1, int n2, int n3, int nv, int nc,
                                                   const int32_t *__restrict__ qorb,
                                                   const int32_t *__restrict__ pidx,
                                                   const uint8_t *__restrict__ pconj,
                                                   const float *__restrict__ mv,
                                                   const float *__restrict__ mc,
                                                   const __bf16 *__restrict__ wh,
                                                   const __bf16 *__restrict__ wl,
                                                   float *__restrict__ H, int64_t ldh,
                                                   double scale) {
  constexpr int BK = 32, P = BK + 8;       // K slab (J) and bf16 row pitch
  constexpr int NMB = 64 * MI;             // rows I of W
  constexpr int NI = 2 * KC;               // column blocks: (k, re/im)
  constexpr int NCOL = 16 * NI;            // B rows in LDS
  constexpr int NA = NMB * (BK / 8) / NT;  // 16-byte pieces of each W plane per thread per slab
  static_assert(NA == MI && KC == 2, "one W row group of 64 per thread slot, 8 Mv pieces per row");
  constexpr int STAGE = 2 * (NMB + NCOL) * P * 2;  // bytes: hi + lo tiles
  constexpr int NCB = 3;                   // c c' row blocks of stage 2
  constexpr int RED = 4 * NCB * 16 * 16 * 8;       // bytes: float2 partial D per wave
  __shared__ __attribute__((aligned(16))) unsigned char lds[STAGE > RED ? STAGE : RED];
  __bf16 *Ah = reinterpret_cast<__bf16 *>(lds), *Al = Ah + NMB * P;
  __bf16 *Bh = Al + NMB * P, *Bl = Bh + NCOL * P;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nk = n1 * n2 * n3, nvv = nv * nv, ncc = nc * nc;
  const int q = blockIdx.y;
  const int k0 = blockIdx.x * KC;
  // W pieces: thread slot u covers row arow + 64 u, bf16 columns 8 ac .. 8 ac + 7 of the slab
  const int ac = tid & 3, arow = 16 * (tid >> 6) + 4 * ((tid >> 2) & 3) + ((tid >> 4) & 3);
  const int64_t wbase = (int64_t(qorb[q]) * NMB + arow) * NMB + 8 * ac;
  const int aoff = arow * P + 8 * ac;
  // Mv piece: complex values 4 bc .. 4 bc + 3 of row kk * 16 + vv'
  const int bc = tid & 7, bkk = tid >> 7, bvv = 4 * ((tid >> 3) & 3) + ((tid >> 5) & 3);
  const float4 *bsrc = reinterpret_cast<const float4 *>(mv) + 2 * bc;  // a readable row if masked
  float bre = 0.f, bim = 0.f;  // scale of the real and imaginary parts (0: no such row)
  {
    const int k = k0 + bkk;
    if (k < nk && bvv < nvv) {
      const int kq = kminus(k, q, n1, n2, n3);
      const int64_t p = int64_t(k) * nk + kq;
      const bool cj = pconj[p] != 0;
      const int v = bvv / nv, v2 = bvv % nv;
      const int s1 = cj ? v2 : v, s2 = cj ? v : v2;
      bsrc = reinterpret_cast<const float4 *>(mv) +
             (((int64_t(pidx[p]) * nv + s1) * nv + s2) * NMB) / 2 + 2 * bc;
      bre = 1.f;
      bim = cj ? -1.f : 1.f;
    }
  }
  const int boff = ((2 * bkk) * 16 + bvv) * P + 4 * bc;
  f32x4 acc[MI][NI];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = f32x4{0, 0, 0, 0};
  const int wm0 = wv * 16 * MI;
  const int r16 = lane & 15, g = lane >> 4;
  const u32x4 *whp = reinterpret_cast<const u32x4 *>(wh + wbase);
  const u32x4 *wlp = reinterpret_cast<const u32x4 *>(wl + wbase);
  constexpr int WU = 64 * NMB / 8;  // u32x4 stride of 64 W rows
  u32x4 pah[NA], pal[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    pah[u] = whp[WU * u];
    pal[u] = wlp[WU * u];
  }
  float4 pb0 = bsrc[0], pb1 = bsrc[1];
  for (int j0 = 0; j0 < NMB; j0 += BK) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      *reinterpret_cast<u32x4 *>(Ah + aoff + 64 * u * P) = pah[u];
      *reinterpret_cast<u32x4 *>(Al + aoff + 64 * u * P) = pal[u];
    }
    {
      // four complex values: real parts to the re row, (signed) imaginary parts to the im row
      const float er[4] = {bre * pb0.x, bre * pb0.z, bre * pb1.x, bre * pb1.z};
      const float ei[4] = {bim * pb0.y, bim * pb0.w, bim * pb1.y, bim * pb1.w};
      bf16x4 hr, lr, hi, li;
      splitn<4>(er, hr, lr);
      splitn<4>(ei, hi, li);
      *reinterpret_cast<bf16x4 *>(Bh + boff) = hr;
      *reinterpret_cast<bf16x4 *>(Bl + boff) = lr;
      *reinterpret_cast<bf16x4 *>(Bh + boff + 16 * P) = hi;
      *reinterpret_cast<bf16x4 *>(Bl + boff + 16 * P) = li;
    }
    __syncthreads();
    {
      // the next slab, in flight during the MFMAs (the last slab fetches itself again)
      const int jn = min(j0 + BK, NMB - BK);
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        pah[u] = whp[WU * u + jn / 8];
        pal[u] = wlp[WU * u + jn / 8];
      }
      pb0 = bsrc[jn / 2];
      pb1 = bsrc[jn / 2 + 1];
    }
    bf16x8 bh[NI], bl[NI];
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      bh[ni] = *reinterpret_cast<const bf16x8 *>(Bh + (16 * ni + r16) * P + 8 * g);
      bl[ni] = *reinterpret_cast<const bf16x8 *>(Bl + (16 * ni + r16) * P + 8 * g);
    }
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(Ah + (wm0 + 16 * mi + r16) * P + 8 * g);
      const bf16x8 al = *reinterpret_cast<const bf16x8 *>(Al + (wm0 + 16 * mi + r16) * P + 8 * g);
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = mma3(acc[mi][ni], ah, al, bh[ni], bl[ni]);
    }
    __syncthreads();
  }
  // ---- stage 2 ----
  const int ncb = (ncc + 15) / 16;
  float2 *red = reinterpret_cast<float2 *>(lds);  // [4][NCB*16][16]
  float2 *Hc = reinterpret_cast<float2 *>(H);
  // Mc row (c, c') of this lane's A rows in each c c' block: as stored (low
  // 16 bits) and band-swapped for a conjugated class (high 16 bits); -1 past
  // the last pair
  int mrow[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int cc = 16 * cb + r16, c = cc / nc, c2 = cc % nc;
    mrow[cb] = cc < ncc ? ((c2 * nc + c) << 16) | (c * nc + c2) : -1;
  }
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = k0 + kk;
    // Re Mc Re T, Im Mc Im T, Re Mc Im T, Im Mc Re T (Mc as stored)
    f32x4 d_rr[NCB], d_ii[NCB], d_ri[NCB], d_ir[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) d_rr[cb] = d_ii[cb] = d_ri[cb] = d_ir[cb] = f32x4{0, 0, 0, 0};
    int kq = 0;
    float sg = 1.f;
    if (k < nk) {
      kq = kminus(k, q, n1, n2, n3);
      const int64_t p = int64_t(k) * nk + kq;
      const bool cj = pconj[p] != 0;
      sg = cj ? -1.f : 1.f;
      const int cls = pidx[p];
#pragma unroll
      for (int mp = 0; mp < MI; mp += 2) {
        const bool two = mp + 1 < MI;
        float tre[8], tim[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          tre[j] = acc[mp][2 * kk][j];
          tim[j] = acc[mp][2 * kk + 1][j];
          tre[4 + j] = two ? acc[two ? mp + 1 : mp][2 * kk][j] : 0.f;
          tim[4 + j] = two ? acc[two ? mp + 1 : mp][2 * kk + 1][j] : 0.f;
        }
        bf16x8 trh, trl, tih, til;
        splitn<8>(tre, trh, trl);
        splitn<8>(tim, tih, til);
        const int I0 = wm0 + 16 * mp + 4 * g;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          if (cb >= ncb) break;
          const int mr = mrow[cb] < 0 ? -1 : cj ? mrow[cb] >> 16 : mrow[cb] & 0xffff;
          float are[8], aim[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) are[j] = aim[j] = 0.f;
          if (mr >= 0) {
            const float4 *src = reinterpret_cast<const float4 *>(
                reinterpret_cast<const float2 *>(mc) + (int64_t(cls) * ncc + mr) * NMB);
            // Mc at I0 .. I0+3 and (second tile) I0+16 .. I0+19
            const float4 m0 = src[I0 / 2], m1 = src[I0 / 2 + 1];
            const float4 m2 = two ? src[(I0 + 16) / 2] : float4{0, 0, 0, 0};
            const float4 m3 = two ? src[(I0 + 16) / 2 + 1] : float4{0, 0, 0, 0};
            are[0] = m0.x; aim[0] = m0.y; are[1] = m0.z; aim[1] = m0.w;
            are[2] = m1.x; aim[2] = m1.y; are[3] = m1.z; aim[3] = m1.w;
            are[4] = m2.x; aim[4] = m2.y; are[5] = m2.z; aim[5] = m2.w;
            are[6] = m3.x; aim[6] = m3.y; are[7] = m3.z; aim[7] = m3.w;
          }
          bf16x8 arh, arl, aih, ail;
          splitn<8>(are, arh, arl);
          splitn<8>(aim, aih, ail);
          d_rr[cb] = mma3(d_rr[cb], arh, arl, trh, trl);
          d_ii[cb] = mma3(d_ii[cb], aih, ail, tih, til);
          d_ri[cb] = mma3(d_ri[cb], arh, arl, tih, til);
          d_ir[cb] = mma3(d_ir[cb], aih, ail, trh, trl);
        }
      }
    }
    // partial D of this wave -> LDS, then the sum over waves -> H.  With
    // Mc = re + i sg im:  conj(Mc) T = (re Re T + sg im Im T) + i (re Im T - sg im Re T)
    __syncthreads();  // stage-1 tiles (kk = 0) or the previous reduction are no longer read
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        red[(wv * NCB * 16 + 16 * cb + 4 * g + j) * 16 + r16] =
            float2{d_rr[cb][j] + sg * d_ii[cb][j], d_ri[cb][j] - sg * d_ir[cb][j]};
    __syncthreads();
    if (k < nk) {
      for (int e = tid; e < ncc * nvv; e += NT) {
        const int cc = e / nvv, vv = e % nvv;
        float2 sum = {0.f, 0.f};
#pragma unroll
        for (int w4 = 0; w4 < 4; ++w4) {
          const float2 x = red[(w4 * NCB * 16 + cc) * 16 + vv];
          sum.x += x.x;
          sum.y += x.y;
        }
        const int c = cc / nc, c2 = cc % nc, v = vv / nv, v2 = vv % nv;
        const int64_t a = (int64_t(k) * nv + v) * nc + c;
        const int64_t b = (int64_t(kq) * nv + v2) * nc + c2;
        float2 hv = Hc[a * ldh + b];
        hv.x -= float(scale * double(sum.x));
        hv.y -= float(scale * double(sum.y));
        Hc[a * ldh + b] = hv;
      }
    }
  }
}

}  // namespace

// workspace of the split-BF16 build: the hi and lo BF16 planes of W
// ([nqorb][nmb][nmb] each)
size_t build_bf16x3_ws(const bse_problem *p) {
  const size_t planes = size_t(p->nqorb) * p->nmb * p->nmb * 2 * sizeof(__bf16);
  return std::max<size_t>(256, (planes + 255) / 256 * 256);
}

int32_t build_bf16x3(const bse_problem *p, void *H, int64_t ldh, void *ws, size_t ws_bytes,
                     bse_stream stream) {
  const int n1 = p->grid[0], n2 = p->grid[1], n3 = p->grid[2];
  const int nk = n1 * n2 * n3;
  const int64_t N = int64_t(nk) * p->nv * p->nc;
  if (!H) return fail(BSE_EINVAL, "H is NULL");
  if (ldh < N) return fail(BSE_ESHAPE, "ldh %lld < N %lld", (long long)ldh, (long long)N);
  if (!fused_shape(p->nmb, p->nv, p->nc))
    return fail(BSE_EUNSUPPORTED,
                "split-BF16 build needs Nmb = 64 m (m <= 6), nv <= 4 and nc <= 6");
  if (!ws || ws_bytes < build_bf16x3_ws(p))
    return fail(BSE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes,
                build_bf16x3_ws(p));
  if (reinterpret_cast<uintptr_t>(ws) % 16 != 0)
    return fail(BSE_EINVAL, "workspace must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const double inv_nk = 1.0 / nk;
  dim3 gx((unsigned)((N + XBN - 1) / XBN), (unsigned)((2 * N + XBM - 1) / XBM));
  if (gx.y > 65535u) return fail(BSE_ESHAPE, "N too large for the exchange grid");
  BSE_LAUNCH("k_exchange_bf3", k_exchange_bf3, gx, dim3(NT), 0, s, nk, p->nv, p->nc, p->nmb,
             p->korb, (const float *)p->mx, p->vdiag, p->ev, p->ec, (float *)H, ldh,
             2.0 * inv_nk);
  BSE_HIP_CHECK(hipGetLastError());
  const int64_t nw = int64_t(p->nqorb) * p->nmb * p->nmb;  // a multiple of 4096
  __bf16 *wh = reinterpret_cast<__bf16 *>(ws), *wl = wh + nw;
  const int64_t n4 = nw / 4;
  BSE_LAUNCH("k_split_w", k_split_w, dim3((unsigned)std::min<int64_t>((n4 + NT - 1) / NT, 8192)),
             dim3(NT), 0, s, n4, (const float4 *)p->w, (bf16x4 *)wh, (bf16x4 *)wl);
  BSE_HIP_CHECK(hipGetLastError());
  constexpr int KC = 2;
  dim3 gf((unsigned)((nk + KC - 1) / KC), (unsigned)nk);
#define BSE_BF3_CASE(M)                                                                       \
  case M:                                                                                   \
    BSE_LAUNCH("k_direct_bf3", (k_direct_bf3<M, KC>), gf, dim3(NT), 0, s, n1, n2, n3, p->nv,  \
               p->nc, p->qorb, p->pidx, p->pconj, (const float *)p->mv, (const float *)p->mc, \
               wh, wl, (float *)H, ldh, inv_nk);                                         \
    break;
  switch (p->nmb / 64) {
    BSE_BF3_CASE(1)
    BSE_BF3_CASE(2)
    BSE_BF3_CASE(3)
    BSE_BF3_CASE(4)
    BSE_BF3_CASE(5)
    BSE_BF3_CASE(6)
    default:
      return fail(BSE_EUNSUPPORTED, "split-BF16 direct kernel: nmb = 64 m with m <= 6");
  }
#undef BSE_BF3_CASE
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}

}  // namespace bse
