// bse_project_blocks: H_mu = U_mu^T H U_mu and B_mu = U_mu^T B.
//
// Paper: Eq. (projection) and Eq. (transformationU), Sec. III.C.4: the
// transformation is done irrep by irrep and U is sparse (block diagonal over
// k orbits, at most |S| d_max^2 non-zeros per basis vector); the band indices
// are spectators, so
//   H_mu[(O,j,v,c),(O',j',v',c')] =
//       sum_{k in O, k' in O'} U_O[k,j] H[(k,v,c),(k',v',c')] U_O'[k',j'].
//
// Kernel k_project: one workgroup per (row band (v,c), column orbit O', row
// orbit O).  The members of both orbits and both bases are staged in LDS once.
// The H rows (k,v,c), k in O, restricted to the columns of O' (|O'| runs of
// nv nc contiguous complex values) are fetched RU rows at a time, up to PCH
// elements, with every load of a chunk issued before any is stored to LDS.
// Each chunk is contracted with U_O' (thread = output column (j', v', c')) and
// accumulated, times U_O[k, j], into registers.  Each H element is read exactly
// once per projected block; the kernel is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <vector>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int PNT = 256;
constexpr int PMAXR = 9;     // basis vectors per orbit: d_mu m_mu(O) <= d_max^2
constexpr int PMAXCOL = 2;   // output columns per thread: r' nv nc <= 512
constexpr int PMAXL = 48;    // orbit size <= |S|
constexpr int PCH = 2048;    // H elements per chunk (8 per thread)

// Source of the H elements when projecting straight from the seed pieces
// (f1 without materialising H): every element is formed as the seed assembly
// forms it,
//   H[(k v c),(k' v' c')] = X[(o(k) v c),(o(k') v' c')] + delta (E_c - E_v)
//                           - scale D[porb(k,k')][(c c')][(v v')],
// and rounded to T, so the projected block equals the projection of the
// assembled H exactly.
struct SeedSrc {
  const int32_t *korb, *porb;
  const double *ev, *ec;
  const void *xs, *drep;
  int64_t ldx;
  int nk;
  double scale;
};

// PAIR (FP32 H, nv nc even): two entries per 16-byte load; a run of nv nc
// entries starts at an even entry, so a pair never straddles two runs.
template <typename T, bool SEEDSRC, int NCT, bool PAIR = false>
__global__ __launch_bounds__(PNT) __attribute__((amdgpu_waves_per_eu(NCT == 1 && !SEEDSRC && sizeof(T) == 4 ? 6 : 1, 8))) void k_project(int nv, int nc, const T *__restrict__ H,
                                                 int64_t ldh, const int32_t *__restrict__ mem_off,
                                                 const int32_t *__restrict__ members,
                                                 const int64_t *__restrict__ orb_off,
                                                 const int32_t *__restrict__ orb_dim,
                                                 const int64_t *__restrict__ ub_off,
                                                 const double *__restrict__ ub, T *__restrict__ Hmu,
                                                 int64_t ldmu, SeedSrc sd) {
  typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type C2;
  __shared__ C2 rows[PCH];
  __shared__ double u1s[PMAXL * PMAXR], u2s[PMAXL * PMAXR];
  __shared__ int32_t m1s[PMAXL], m2s[PMAXL];
  __shared__ int32_t o1s[SEEDSRC ? PMAXL : 1], o2s[SEEDSRC ? PMAXL : 1];  // k orbits of the members
  __shared__ int32_t pps[SEEDSRC ? PMAXL * PMAXL : 1];  // pair orbits of the member pairs
  const int nb = nv * nc;
  const int band = blockIdx.x;        // (v, c) of the output rows
  // orbit ids grow with orbit size on the simple grids, so the largest (longest)
  // orbit pairs are dispatched first and do not form a tail
  const int o2 = gridDim.y - 1 - blockIdx.y, o1 = gridDim.z - 1 - blockIdx.z;
  const int r1 = orb_dim[o1], r2 = orb_dim[o2];
  if (r1 == 0 || r2 == 0) return;
  const int L1 = mem_off[o1 + 1] - mem_off[o1], L2 = mem_off[o2 + 1] - mem_off[o2];
  // orbits have at most |S| members and bases at most d_mu^2 vectors (the
  // host checks PMAXL nb <= PCH); anything else is not a valid block
  if (L1 > PMAXL || L2 > PMAXL || r1 > PMAXR || r2 > PMAXR) return;
  const int32_t *m1 = members + mem_off[o1], *m2 = members + mem_off[o2];
  for (int i = threadIdx.x; i < L1 * r1; i += PNT) u1s[i] = ub[ub_off[o1] + i];
  for (int i = threadIdx.x; i < L2 * r2; i += PNT) u2s[i] = ub[ub_off[o2] + i];
  if (threadIdx.x < L2) m2s[threadIdx.x] = m2[threadIdx.x];
  if (threadIdx.x < L1) m1s[threadIdx.x] = m1[threadIdx.x];
  if constexpr (SEEDSRC) {
    if (threadIdx.x < L2) o2s[threadIdx.x] = sd.korb[m2[threadIdx.x]];
    if (threadIdx.x < L1) o1s[threadIdx.x] = sd.korb[m1[threadIdx.x]];
    for (int q = threadIdx.x; q < L1 * L2; q += PNT)
      pps[q] = sd.porb[int64_t(m1[q / L2]) * sd.nk + m2[q % L2]];
  }
  const int ncol = r2 * nb, per = L2 * nb;
  const int RU = PCH / per;  // rows per chunk (>= 1)
  double accr[NCT][PMAXR], acci[NCT][PMAXR];  // NCT output columns per thread
#pragma unroll
  for (int t = 0; t < NCT; ++t)
#pragma unroll
    for (int j = 0; j < PMAXR; ++j) accr[t][j] = acci[t][j] = 0.0;
  const int v = band / nc, c = band % nc;
  __syncthreads();  // m1s, m2s
  // chunk loads go to registers; the next chunk's loads are in flight while
  // the current one is contracted from LDS
  static_assert(!PAIR || (sizeof(T) == 4 && !SEEDSRC), "pairs: FP32 H only");
  constexpr int NL = PAIR ? PCH / (2 * PNT) : PCH / PNT;  // loads per thread and chunk
  typedef typename std::conditional<PAIR, float4, C2>::type LV;
  LV x[NL];
  // every load is issued unconditionally from a clamped, in-bounds index and
  // entries past the chunk are zeroed afterwards, so the loads do not wait on
  // one another
  auto fetch = [&](int i0) {
    const int nr = std::min(RU, L1 - i0);
    if constexpr (PAIR) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int q = threadIdx.x + PNT * u;
        const int e = std::min(2 * q, nr * per - 2);
        const int ii = e / per, rem = e - ii * per, i2 = rem / nb, b2 = rem - i2 * nb;
        const int64_t a = (int64_t(m1s[i0 + ii]) * nv + v) * nc + c;
        x[u] = *reinterpret_cast<const float4 *>(reinterpret_cast<const C2 *>(H) + a * ldh +
                                                 int64_t(m2s[i2]) * nb + b2);
      }
#pragma unroll
      for (int u = 0; u < NL; ++u)
        if (2 * (threadIdx.x + PNT * u) >= nr * per) x[u] = LV{0, 0, 0, 0};
      return;
    } else {
#pragma unroll
    for (int u = 0; u < PCH / PNT; ++u) {
      const int e0 = threadIdx.x + PNT * u;
      const int e = std::min(e0, nr * per - 1);
      const int ii = e / per, rem = e - ii * per, i2 = rem / nb, b2 = rem - i2 * nb;
      if constexpr (SEEDSRC) {
        const int k = m1s[i0 + ii], k2 = m2s[i2], ia = v * nc + c;
        const int v2 = b2 / nc, c2 = b2 % nc;
        const C2 xe = reinterpret_cast<const C2 *>(sd.xs)[(int64_t(o1s[i0 + ii]) * nb + ia) * sd.ldx +
                                                          int64_t(o2s[i2]) * nb + b2];
        const int64_t o = pps[(i0 + ii) * L2 + i2];
        const C2 d = reinterpret_cast<const C2 *>(sd.drep)[(o * (nc * nc) + c * nc + c2) * (nv * nv) +
                                                           v * nv + v2];
        double re = double(xe.x) - sd.scale * double(d.x), im = double(xe.y) - sd.scale * double(d.y);
        if (k == k2 && ia == b2) re += sd.ec[int64_t(k) * nc + c] - sd.ev[int64_t(k) * nv + v];
        x[u] = C2{T(re), T(im)};
      } else {
        const int64_t a = (int64_t(m1s[i0 + ii]) * nv + v) * nc + c;
        x[u] = reinterpret_cast<const C2 *>(H)[a * ldh + int64_t(m2s[i2]) * nb + b2];
      }
    }
#pragma unroll
    for (int u = 0; u < PCH / PNT; ++u)
      if (threadIdx.x + PNT * u >= nr * per) x[u] = C2{0, 0};
    }
  };
  fetch(0);
  for (int i0 = 0; i0 < L1; i0 += RU) {
    const int nr = std::min(RU, L1 - i0);
    __syncthreads();  // the previous chunk has been consumed
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      if constexpr (PAIR)
        reinterpret_cast<float4 *>(rows)[threadIdx.x + PNT * u] = x[u];
      else
        rows[threadIdx.x + PNT * u] = x[u];
    }
    __syncthreads();
    if (i0 + RU < L1) fetch(i0 + RU);
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      const int col = threadIdx.x + PNT * t;
      if (col >= ncol) break;
      const int j2 = col / nb, b2 = col % nb;
      for (int ii = 0; ii < nr; ++ii) {
        double zr = 0, zi = 0;
        for (int i2 = 0; i2 < L2; ++i2) {
          const C2 h = rows[ii * per + i2 * nb + b2];
          const double u = u2s[i2 * r2 + j2];
          zr += u * double(h.x);
          zi += u * double(h.y);
        }
#pragma unroll
        for (int j = 0; j < PMAXR; ++j)
          if (j < r1) {
            const double u = u1s[(i0 + ii) * r1 + j];
            accr[t][j] += u * zr;
            acci[t][j] += u * zi;
          }
      }
    }
  }
  const int64_t rbase = orb_off[o1] + band, cbase = orb_off[o2];
#pragma unroll
  for (int t = 0; t < NCT; ++t) {
    const int col = threadIdx.x + PNT * t;
    if (col >= ncol) break;
#pragma unroll
    for (int j = 0; j < PMAXR; ++j)
      if (j < r1)
        reinterpret_cast<C2 *>(Hmu)[(rbase + int64_t(j) * nb) * ldmu + cbase + col] =
            C2{T(accr[t][j]), T(acci[t][j])};
  }
}

// B_mu[(O,j,b)] = sum_{k in O} U_O[k,j] B[(k,b)]; one thread per output element.
__global__ void k_project_vec(int nkorb, int nb, const int32_t *__restrict__ mem_off,
                              const int32_t *__restrict__ members,
                              const int64_t *__restrict__ orb_off,
                              const int32_t *__restrict__ orb_dim,
                              const int64_t *__restrict__ ub_off, const double *__restrict__ ub,
                              const double2 *__restrict__ B, double2 *__restrict__ Bmu) {
  const int o = blockIdx.x;
  const int r = orb_dim[o], L = mem_off[o + 1] - mem_off[o];
  const int32_t *m = members + mem_off[o];
  const double *U = ub + ub_off[o];
  for (int e = threadIdx.x; e < r * nb; e += blockDim.x) {
    const int j = e / nb, b = e % nb;
    double sr = 0, si = 0;
    for (int i = 0; i < L; ++i) {
      const double2 x = B[int64_t(m[i]) * nb + b];
      sr += U[i * r + j] * x.x;
      si += U[i * r + j] * x.y;
    }
    Bmu[orb_off[o] + e] = double2{sr, si};
  }
}

// |B_mu|^2 = sum over the block's orbits and basis vectors of |sum_{k in O}
// U_O[k,j] B[(k,b)]|^2, one workgroup per block (fixed summation order).
constexpr int DNT = 256;
__global__ __launch_bounds__(DNT) void k_dipole_norm(int nkorb, int nb,
                                                     const int32_t *__restrict__ mem_off,
                                                     const int32_t *__restrict__ members,
                                                     const int32_t *__restrict__ orb_dim,
                                                     const int64_t *__restrict__ ub_off,
                                                     const double *__restrict__ ub,
                                                     const double2 *__restrict__ B,
                                                     double *__restrict__ out) {
  __shared__ double sh[DNT];
  double acc = 0;
  for (int o = 0; o < nkorb; ++o) {
    const int r = orb_dim[o], L = mem_off[o + 1] - mem_off[o];
    const int32_t *m = members + mem_off[o];
    const double *U = ub + ub_off[o];
    for (int e = threadIdx.x; e < r * nb; e += DNT) {
      const int j = e / nb, b = e % nb;
      double sr = 0, si = 0;
      for (int i = 0; i < L; ++i) {
        const double2 x = B[int64_t(m[i]) * nb + b];
        sr += U[i * r + j] * x.x;
        si += U[i * r + j] * x.y;
      }
      acc += sr * sr + si * si;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = DNT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// The dipole-active block: the largest weight, if it exceeds rel times the
// total (the first such block on ties); -1 when no block carries weight.
__global__ void k_dipole_select(int nblk, const double *__restrict__ w, double rel,
                                int32_t *__restrict__ active) {
  if (threadIdx.x != 0) return;
  double tot = 0;
  for (int i = 0; i < nblk; ++i) tot += w[i];
  int best = -1;
  for (int i = 0; i < nblk; ++i)
    if (w[i] > rel * tot && (best < 0 || w[i] > w[best])) best = i;
  *active = best;
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" int32_t bse_dipole_weights(const bse_problem *p, const void *B, int32_t nblk,
                                      const bse_block *blk, double *weights, int32_t *active,
                                      bse_stream stream) {
  if (!p || !B || !weights || !active) return fail(BSE_EINVAL, "NULL pointer");
  if (nblk < 1 || !blk) return fail(BSE_EINVAL, "bad block list");
  const int n1 = p->grid[0], n2 = p->grid[1], n3 = p->grid[2];
  if (n1 < 1 || n2 < 1 || n3 < 1 || p->nv < 1 || p->nc < 1 || p->nkorb < 1)
    return fail(BSE_ESHAPE, "bad problem sizes");
  const int64_t nb = int64_t(p->nv) * p->nc, N = int64_t(n1) * n2 * n3 * nb;
  hipStream_t s = (hipStream_t)stream;
  for (int ib = 0; ib < nblk; ++ib) {
    const bse_block &b = blk[ib];
    if (b.n < 0 || !b.mem_off || !b.members || !b.orb_off || !b.orb_dim || !b.ub_off || !b.ubasis)
      return fail(BSE_EINVAL, "block %d has NULL arrays", ib);
    if (b.n > N) return fail(BSE_ESHAPE, "block %d larger than N", ib);
  }
  for (int ib = 0; ib < nblk; ++ib) {
    const bse_block &b = blk[ib];
    BSE_LAUNCH("k_dipole_norm", k_dipole_norm, dim3(1), dim3(DNT), 0, s, p->nkorb, (int)nb,
               b.mem_off, b.members, b.orb_dim, b.ub_off, b.ubasis, (const double2 *)B,
               weights + ib);
  }
  BSE_LAUNCH("k_dipole_select", k_dipole_select, dim3(1), dim3(64), 0, s, nblk,
             (const double *)weights, 1e-12, active);
  BSE_HIP_CHECK(hipGetLastError());
  return BSE_OK;
}

extern "C" int32_t bse_project_blocks(const bse_problem *p, const void *H, int64_t ldh,
                                      int32_t h_fp64, const void *B, int32_t nblk,
                                      const bse_block *blk, void *const *Hmu,
                                      const int64_t *ldmu, void *const *Bmu, bse_stream stream) {
  if (!p) return fail(BSE_EINVAL, "problem is NULL");
  if (nblk < 0 || (nblk > 0 && !blk)) return fail(BSE_EINVAL, "bad block list");
  const int n1 = p->grid[0], n2 = p->grid[1], n3 = p->grid[2];
  if (n1 < 1 || n2 < 1 || n3 < 1 || p->nv < 1 || p->nc < 1 || p->nkorb < 1)
    return fail(BSE_ESHAPE, "bad problem sizes");
  const int64_t nk = int64_t(n1) * n2 * n3, nb = int64_t(p->nv) * p->nc, N = nk * nb;
  if (nb > 128 * PMAXCOL * 2) return fail(BSE_EUNSUPPORTED, "nv nc too large for projection");
  hipStream_t s = (hipStream_t)stream;
  if (int64_t(PMAXL) * nb > PCH) return fail(BSE_EUNSUPPORTED, "nv nc too large for projection");
  for (int ib = 0; ib < nblk; ++ib) {
    const bse_block &b = blk[ib];
    if (b.n < 0 || !b.mem_off || !b.members || !b.orb_off || !b.orb_dim || !b.ub_off || !b.ubasis)
      return fail(BSE_EINVAL, "block %d has NULL arrays", ib);
    if (b.n > N) return fail(BSE_ESHAPE, "block %d larger than N", ib);
    if (Hmu && Hmu[ib]) {
      if (!H) return fail(BSE_EINVAL, "H is NULL");
      if (ldh < N) return fail(BSE_ESHAPE, "ldh < N");
      if (!ldmu || ldmu[ib] < b.n) return fail(BSE_ESHAPE, "ldmu[%d] < n", ib);
      if (9 * nb > PNT * PMAXCOL)
        return fail(BSE_EUNSUPPORTED, "r' nv nc exceeds %d columns", PNT * PMAXCOL);
      dim3 g((unsigned)nb, (unsigned)p->nkorb, (unsigned)p->nkorb);
      const bool one = 9 * nb <= PNT;  // every output column of a block row in one thread
#define BSE_PROJ(T, NCT, PR)                                                                  \
  BSE_LAUNCH("k_project", (k_project<T, false, NCT, PR>), g, dim3(PNT), 0, s, p->nv, p->nc,   \
             (const T *)H, ldh, b.mem_off, b.members, b.orb_off, b.orb_dim, b.ub_off, b.ubasis, \
             (T *)Hmu[ib], ldmu[ib], SeedSrc{})
      // pairs of FP32 entries need nv nc even and 16-byte aligned rows
      const bool pair = nb % 2 == 0 && ldh % 2 == 0 && (reinterpret_cast<uintptr_t>(H) & 15) == 0;
      if (h_fp64) {
        if (one) BSE_PROJ(double, 1, false); else BSE_PROJ(double, 2, false);
      } else if (pair) {
        if (one) BSE_PROJ(float, 1, true); else BSE_PROJ(float, 2, true);
      } else {
        if (one) BSE_PROJ(float, 1, false); else BSE_PROJ(float, 2, false);
      }
#undef BSE_PROJ
      BSE_HIP_CHECK(hipGetLastError());
    }
    if (Bmu && Bmu[ib]) {
      if (!B) return fail(BSE_EINVAL, "B is NULL");
      BSE_LAUNCH("k_project_vec", k_project_vec, dim3((unsigned)p->nkorb), dim3(256), 0, s, p->nkorb,
                         (int)nb, b.mem_off, b.members, b.orb_off, b.orb_dim, b.ub_off, b.ubasis,
                         (const double2 *)B, (double2 *)Bmu[ib]);
      BSE_HIP_CHECK(hipGetLastError());
    }
  }
  return BSE_OK;
}

extern "C" int32_t bse_project_seed(int64_t plan, int32_t nblk, const bse_block *blk,
                                    void *const *Hmu, const int64_t *ldmu, bse_stream stream) {
  SeedPieces sp;
  const int32_t st = seed_pieces(plan, &sp);
  if (st) return st;
  const bse_problem *p = &sp.p;
  if (nblk < 0 || (nblk > 0 && !blk)) return fail(BSE_EINVAL, "bad block list");
  const int64_t nb = int64_t(p->nv) * p->nc, N = int64_t(sp.nk) * nb;
  if (int64_t(PMAXL) * nb > PCH || 9 * nb > PNT * PMAXCOL)
    return fail(BSE_EUNSUPPORTED, "nv nc too large for projection");
  hipStream_t s = (hipStream_t)stream;
  const SeedSrc sd{p->korb, sp.porb, p->ev, p->ec, sp.xs, sp.drep, sp.ldx, sp.nk, 1.0 / sp.nk};
  for (int ib = 0; ib < nblk; ++ib) {
    if (!Hmu || !Hmu[ib]) continue;
    const bse_block &b = blk[ib];
    if (b.n < 0 || !b.mem_off || !b.members || !b.orb_off || !b.orb_dim || !b.ub_off || !b.ubasis)
      return fail(BSE_EINVAL, "block %d has NULL arrays", ib);
    if (b.n > N) return fail(BSE_ESHAPE, "block %d larger than N", ib);
    if (!ldmu || ldmu[ib] < b.n) return fail(BSE_ESHAPE, "ldmu[%d] < n", ib);
    dim3 g((unsigned)nb, (unsigned)p->nkorb, (unsigned)p->nkorb);
    const bool one = 9 * nb <= PNT;
#define BSE_PROJS(T, NCT)                                                                     \
  BSE_LAUNCH("k_project_seed", (k_project<T, true, NCT>), g, dim3(PNT), 0, s, p->nv, p->nc,   \
             nullptr, 0, b.mem_off, b.members, b.orb_off, b.orb_dim, b.ub_off, b.ubasis,       \
             (T *)Hmu[ib], ldmu[ib], sd)
    if (sp.prec == BSE_FP64) {
      if (one) BSE_PROJS(double, 1); else BSE_PROJS(double, 2);
    } else {
      if (one) BSE_PROJS(float, 1); else BSE_PROJS(float, 2);
    }
#undef BSE_PROJS
    BSE_HIP_CHECK(hipGetLastError());
  }
  return BSE_OK;
}
