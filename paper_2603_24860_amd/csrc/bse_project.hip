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
// orbit O).  For every k in O it stages the H row (k,v,c) restricted to the
// columns of O' (|O'| runs of nv nc contiguous complex values) in LDS, contracts
// it with U_O' (thread = output column (j', v', c')), and accumulates
// U_O[k, j] times that into registers.  Each H element is read exactly once
// per projected block; the kernel is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <vector>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int PNT = 256;
constexpr int PMAXR = 9;     // basis vectors per orbit: d_mu m_mu(O) <= d_max^2
constexpr int PMAXCOL = 2;   // output columns per thread: r' nv nc <= 512

template <typename T>
__global__ __launch_bounds__(PNT) void k_project(int nv, int nc, const T *__restrict__ H,
                                                 int64_t ldh, const int32_t *__restrict__ mem_off,
                                                 const int32_t *__restrict__ members,
                                                 const int64_t *__restrict__ orb_off,
                                                 const int32_t *__restrict__ orb_dim,
                                                 const int64_t *__restrict__ ub_off,
                                                 const double *__restrict__ ub, T *__restrict__ Hmu,
                                                 int64_t ldmu, int maxL) {
  typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type C2;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int nb = nv * nc;
  const int band = blockIdx.x;        // (v, c) of the output rows
  const int o2 = blockIdx.y, o1 = blockIdx.z;
  const int r1 = orb_dim[o1], r2 = orb_dim[o2];
  if (r1 == 0 || r2 == 0) return;
  const int L1 = mem_off[o1 + 1] - mem_off[o1], L2 = mem_off[o2 + 1] - mem_off[o2];
  if (L2 > maxL || r1 > PMAXR || r2 > PMAXR) return;  // outside the LDS sizing
  const int32_t *m1 = members + mem_off[o1], *m2 = members + mem_off[o2];
  const double *U1 = ub + ub_off[o1], *U2 = ub + ub_off[o2];
  C2 *row = reinterpret_cast<C2 *>(smem);                  // [L2 * nb]
  double *u2s = reinterpret_cast<double *>(row + L2 * nb);  // [L2 * r2]
  for (int i = threadIdx.x; i < L2 * r2; i += PNT) u2s[i] = U2[i];
  const int ncol = r2 * nb;
  double accr[PMAXCOL][PMAXR], acci[PMAXCOL][PMAXR];
#pragma unroll
  for (int t = 0; t < PMAXCOL; ++t)
#pragma unroll
    for (int j = 0; j < PMAXR; ++j) accr[t][j] = acci[t][j] = 0.0;
  const int v = band / nc, c = band % nc;
  for (int i = 0; i < L1; ++i) {
    const int64_t a = (int64_t(m1[i]) * nv + v) * nc + c;
    const C2 *hrow = reinterpret_cast<const C2 *>(H) + a * ldh;
    __syncthreads();
    for (int e = threadIdx.x; e < L2 * nb; e += PNT) {
      const int i2 = e / nb, b2 = e % nb;
      row[e] = hrow[int64_t(m2[i2]) * nb + b2];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PMAXCOL; ++t) {
      const int col = threadIdx.x + PNT * t;
      if (col >= ncol) break;
      const int j2 = col / nb, b2 = col % nb;
      double zr = 0, zi = 0;
      for (int i2 = 0; i2 < L2; ++i2) {
        const C2 h = row[i2 * nb + b2];
        const double u = u2s[i2 * r2 + j2];
        zr += u * double(h.x);
        zi += u * double(h.y);
      }
#pragma unroll
      for (int j = 0; j < PMAXR; ++j)
        if (j < r1) {
          const double u = U1[i * r1 + j];
          accr[t][j] += u * zr;
          acci[t][j] += u * zi;
        }
    }
  }
  const int64_t rbase = orb_off[o1] + band, cbase = orb_off[o2];
#pragma unroll
  for (int t = 0; t < PMAXCOL; ++t) {
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

}  // namespace
}  // namespace bse

using namespace bse;

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
  // largest orbit (LDS size) from the host: members are device data, so the
  // bound |O| <= |S| (48) is used
  const int maxL = 48;
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
      const size_t csz = h_fp64 ? 16 : 8;
      const size_t lds = size_t(maxL) * nb * csz + size_t(maxL) * PMAXR * 8;
      if (lds > 160 * 1024) return fail(BSE_EUNSUPPORTED, "projection tile exceeds LDS");
      dim3 g((unsigned)nb, (unsigned)p->nkorb, (unsigned)p->nkorb);
      if (h_fp64)
        BSE_LAUNCH("k_project", k_project<double>, g, dim3(PNT), lds, s, p->nv, p->nc,
                           (const double *)H, ldh, b.mem_off, b.members, b.orb_off, b.orb_dim,
                           b.ub_off, b.ubasis, (double *)Hmu[ib], ldmu[ib], maxL);
      else
        BSE_LAUNCH("k_project", k_project<float>, g, dim3(PNT), lds, s, p->nv, p->nc,
                           (const float *)H, ldh, b.mem_off, b.members, b.orb_off, b.orb_dim,
                           b.ub_off, b.ubasis, (float *)Hmu[ib], ldmu[ib], maxL);
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
