// Geometry of the block eigensolver: launch constants, per-launch workgroup
// counts and the workspace layout of one block.  Shared by the kernels
// (bse_eigh.hip) and a host-only build that checks every launch's index
// ranges against the layout (tests/eigh_layout_check.cpp).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#if !defined(__HIP__)
// host-only build: the HIP qualifiers vanish and double2 is a plain pair
#define __host__
#define __device__
#define __forceinline__ inline
struct double2 {
  double x, y;
};
#endif

namespace bse {

constexpr int ENT = 256;     // threads per workgroup
constexpr int NBK = 32;      // panel width
constexpr int RNT = 1024;    // threads of the single-workgroup kernels
constexpr int PMAX = 1024;   // partial-sum records read by k_colA (k_colB writes <= 65536 / 64)
constexpr int RB_ROWS = 64;  // rows per k_colB workgroup
// partial-sum record of one k_colB workgroup (complex entries):
//   [0] (S1, 0) = sum |col|^2, [1 + l] BV_l, [1 + NBK + l] BW_l
constexpr int PS = 1 + 2 * NBK;

constexpr int NBMAX = 1024;  // blocks in one batched solve
constexpr int NGRID = 4096;  // grid points of the shared first bisection step (64 x 64)
constexpr int CMAX = 8;      // cluster members refined per eigenvalue cluster
constexpr int KMAX = 256;    // eigenvalues refinable per solve

constexpr int RB = 64;        // rows per k_colB workgroup
constexpr int TP = RB + 1;    // LDS pitch of one panel column

// The update is Hermitian: from HER_TRI tile rows on (mirror), only tiles on
// or below the diagonal are computed (by >= bx) and an off-diagonal tile also
// subtracts the conjugate transpose of its update from the mirror tile,
// staged through LDS so that those writes are row-contiguous too.  Smaller
// trailing blocks keep every tile, for the parallelism.
// Tiles of the trailing update: S = 0 is 64 x 64 complex entries (BM = 128
// real rows, BN = 64 complex columns), S = 1 is 32 x 32 (more workgroups for
// small blocks; the batched solver's autotuner chooses).  From HER_TRI_M
// trailing rows on, only the tiles on or below the diagonal are computed.
constexpr int64_t HER_TRI_M = 2048;
template <typename T, int S = 0> struct HerTile;
template <> struct HerTile<float, 0> { static constexpr int BM = 128, BN = 64, BK = 32; };
template <> struct HerTile<double, 0> { static constexpr int BM = 128, BN = 64, BK = 16; };
template <> struct HerTile<float, 1> { static constexpr int BM = 64, BN = 32, BK = 32; };
template <> struct HerTile<double, 1> { static constexpr int BM = 64, BN = 32, BK = 16; };
__host__ __device__ __forceinline__ bool her_tri(int64_t t, int bn) { return t * bn >= HER_TRI_M; }

// One block's working set.  Partial-sum buffers are sized by the block:
// k_colB and k_col0 write at most ceil(n / 64) records, k_colA at most n sums,
// the initial reflection ceil(n / 256).
struct Desc {
  int64_t n, ld, lda, ldv;
  const void *H;             // H_mu [n][ld]
  const double2 *B;          // B_mu [n]
  void *A;                   // working copy [n][lda]
  double2 *V, *W;            // [NBK][ldv] column major
  double2 *col;              // [n] current column
  double2 *y;                // [n] y = A22 v
  double2 *ys;               // [slots][ldys] partial sums of y of the tile forms (n > TILE_M + 1)
  int64_t ldys;
  double2 *wraw;             // [n] initial reflection: w before the alpha v term
  double2 *vbuf;             // [n] initial reflector
  double2 *partb0, *partb1;  // [R][PS] partial sums of k_colB / k_col0 (alternating)
  double2 *parta;            // [max(n, 1)] partial sums of conj(y) v of k_colA
  double2 *bred;             // [2 NBK] panel dot products of k_colB's records, reduced by k_colA
  double2 *part2;            // [ceil(n / 256)] initial reflection: partial w^dag v
  double *part3;             // [ceil(n / 256)] initial reflection: partial norm
  double2 *scl;              // [n + 1] reflector scale 1 / (alpha - beta), index j + 1
  double2 *tau;              // [n + 1], index j + 1
  double *d, *e;             // [n]
  double *e2;                // [n] squared subdiagonal
  double *tsc;               // [8] tridiagonal scalars
  int *bgrid;                // [NGRID] Sturm counts on a uniform grid over the Gershgorin interval
  double *beta0;             // [1]
  int32_t *status;           // [4] solve status, see bse_block_eigh_status
  double *omega, *pole, *osc;  // outputs [n]
  // refinement of the lowest K eigenvalues (K = 0: none)
  int64_t K;
  double2 *Vall;             // [n][ldv] every reflector (column j: reflector of column j)
  double *Z;                 // [K][n] eigenvectors of T
  double2 *X;                // [K][n] their back-transforms
  double *rqp;               // [K][cdiv(n, HXR)][2] partial Rayleigh quotients
  double *scr;               // [K][6 CMAX n] inverse-iteration scratch
  double *wref;              // [K] refined eigenvalues
  double2 *Tm;               // [cdiv(n - 1, NBK)][NBK][NBK] block-reflector factors T
  int32_t *clo;              // [n] first index of each eigenvalue's cluster in the weights
  // two-stage reduction (full -> band of width SBW -> tridiagonal); null
  // unless the block takes that path
  double2 *pb;               // [n][SBW] current panel, FP64 (reflectors below its diagonal)
  double2 *grec;             // [2][nw][SBW] partial Gram rows of the next panel column
  double2 *srec;             // [nw][SBW][SBW] partial columns of V^dag V
  double2 *sbt;              // [SBW][SBW] block-reflector factor T of the panel
  double2 *sbz;              // [SBW][SBW] Z = T^dag V^dag X
  double2 *sbsc;             // [2][SBW] tau of each panel column, (beta, 0) of each
  double2 *ptop;             // [2][SBW] row c of the panel before column c's reflector
  void *u;                   // [SBW][ldv] U = V T in the storage type of A
  double2 *xp;               // [SBNS][SBW][ldv] split-K partial sums of X = A22 U
  double2 *yrec;             // [nw][SBW][SBW] partial sums of V^dag X
  double2 *band;             // [n][LDB] lower band of the reduced matrix, column by column
  double2 *rfl;              // [n][SBW] latest reflector of each bulge-chasing sweep
  double2 *rtau;             // [n] its tau
  double2 *sink;             // [SINK] target of the stores of masked lanes (never read)
  // two-stage reduction with refinement (K > 0): every reflector of both
  // stages, for the back-transformation; null otherwise
  double2 *rall;             // chase, packed: sweep i at g_bc_off(n, i), rows i + 1 .. n - 1;
                             // each task's first entry (u_0 = 1) holds its tau
  double2 *vrow;             // stage 1, panel p (m rows) at g_sb_voff(n, p) SBW: [SBW][m]
  double2 *bxw;              // [cdiv(n, BPR)][K][SBW] partial V^dag x of the stage-1 back-transformation
};

// Two-stage reduction of large single blocks.  Stage 1 reduces A to a lower
// band of half-width SBW (panels of SBW columns: a QR of the panel below the
// band, then the two-sided update of the trailing block, X = A22 V T on MFMA
// and the rank-2 SBW update); stage 2 chases the band down to tridiagonal
// form, one sweep per column, as tasks of one wave each.
constexpr int SBW = 32;      // band half-width = panel width
constexpr int LDB = 2 * SBW; // band pitch: the band and the fill of one bulge
constexpr int SBR = 64;      // panel rows per workgroup of the panel kernels
constexpr int SBNS = 8;      // K splits of the panel product X = A22 U
constexpr int SBHM = 64;     // rows of X per workgroup of that product
static_assert(SBW == NBK, "the stage-1 update reuses the NBK-wide trailing update");
constexpr int SINK = 256;    // entries of the store sink (lanes of one workgroup)

// ---------------------------------------------------------------------------
// launch geometry, shared by the host (single block) and the batched kernels
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
// The last at most MT rows of a block are reduced by one workgroup in LDS
// (k_tail), starting at the first panel boundary with at most MT rows left.
constexpr int MT = 96;     // largest trailing block reduced in LDS (147 KB)
constexpr int TNT = 512;   // threads of k_tail
static_assert(MT <= TNT, "k_tail: thread j keeps the scalars of column j");
__host__ __device__ __forceinline__ int64_t g_tail0(int64_t n) {
  return n <= MT ? 0 : cdiv(n - MT, NBK) * NBK;
}
__host__ __device__ __forceinline__ int64_t g_nwg(int64_t m) { return m < 1 ? 1 : cdiv(m, ENT); }
__host__ __device__ __forceinline__ int g_rpw(int64_t m) {
  return (int)(m < 2048 ? 1 : cdiv(m, 2048));
}
__host__ __device__ __forceinline__ int64_t g_copy_gx(int64_t n) {
  return cdiv(n, ENT) < 64 ? cdiv(n, ENT) : 64;
}
__host__ __device__ __forceinline__ int64_t g_rank2_gx(int64_t n) {
  return cdiv(n, ENT) < 16 ? cdiv(n, ENT) : 16;
}
__host__ __device__ __forceinline__ int64_t g_records(int64_t n) {
  return n < 64 ? 1 : cdiv(n, 64);
}
__host__ __device__ __forceinline__ int g_nbk(int64_t n, int64_t j0) {
  return (int)(n - j0 < NBK ? n - j0 : NBK);
}
// partial-sum records in front of k_colA of column jn (from k_col0 at a
// panel start, else from k_colB of column jn - 1)
__host__ __device__ __forceinline__ int g_np_in(int64_t n, int64_t jn) {
  return (int)(jn % NBK == 0 ? g_nwg(n - jn) : cdiv(n - jn, RB_ROWS));
}
// wpr = 0: the LDS-staged form of k_colA (LDS_RW rows per wave)
constexpr int LDS_RW = 2;
__host__ __device__ __forceinline__ int g_colA_wgs(int64_t m, int wpr) {
  const int64_t rt = wpr <= 0 ? 4 * LDS_RW : 4 / wpr;  // (the tile forms count tiles instead)
  return (int)(m < 1 ? 1 : cdiv(m, rt));
}
__host__ __device__ __forceinline__ int g_more(int64_t n, int64_t jn) {
  const int64_t j0 = jn - jn % NBK;
  return (jn % NBK) + 1 < g_nbk(n, j0) ? 1 : 0;
}
// waves per row of the single-block k_colA: one row per workgroup up to
// LDS_M trailing rows (latency-bound), the LDS-staged form above (measured
// best at n = 720, 2160 and 10080); the batched solve uses its tuned value
constexpr int64_t LDS_M = 1024;
inline int single_wpr(int64_t m) { return m > LDS_M ? 0 : 4; }

// Above TILE_M trailing rows the working copy is multiplied from its lower
// tiles only (the block is Hermitian): k_colA forms WPR = -1, -2, -3 with
// square tiles of 64, 128 and 256 entries (up to 2560, up to 6144 and above
// 6144 trailing rows, the best of a sweep of these switch points and of the
// form switch over 1024 to 2048 rows).  The tile grid of the trailing
// rows [m0, n) starts at m0 rounded down to 64; tile (i, j), i >= j, adds
// its row sums to slot j and, below the diagonal, the sums of its columns
// (conjugated) to slot i of the rows they belong to, so that
// y[r] = sum over the slots k of ys[k][r].
constexpr int64_t TILE_M = 2048;
__host__ __device__ constexpr int tile_of(int wpr) { return 32 << (-wpr); }
inline int tile_wpr(int64_t m) { return m <= 2560 ? -1 : (m <= 6144 ? -2 : -3); }
__host__ __device__ __forceinline__ int64_t g_tbase(int64_t m0) { return m0 & ~int64_t(63); }
__host__ __device__ __forceinline__ int64_t g_tblocks(int64_t n, int64_t m0, int t) {
  return cdiv(n - g_tbase(m0), t);
}
__host__ __device__ __forceinline__ int64_t g_tiles(int64_t n, int64_t m0, int t) {
  const int64_t b = g_tblocks(n, m0, t);
  return b * (b + 1) / 2;
}
// slots of ys needed by a block of n rows (every tile size it may use)
__host__ __device__ __forceinline__ int64_t g_yslots(int64_t n) {
  int64_t s = cdiv(std::min<int64_t>(n, 2560) + 63, 64);
  s = std::max<int64_t>(s, cdiv(std::min<int64_t>(n, 6144) + 63, 128));
  return std::max<int64_t>(s, cdiv(n + 63, 256));
}

// two-stage geometry: workgroups of the panel kernels over m panel rows
__host__ __device__ __forceinline__ int64_t g_sb_nw(int64_t m) { return m < 1 ? 1 : cdiv(m, SBR); }
// complex K of one split of the panel product (a multiple of the FP32 slab, 32)
__host__ __device__ __forceinline__ int64_t g_sb_kc(int64_t m) {
  return std::max<int64_t>(32, cdiv(cdiv(m, SBNS), 32) * 32);
}
// workgroups (and records) of the split sum k_sb_xred: 64 panel rows each
__host__ __device__ __forceinline__ int64_t g_sb_nx(int64_t m) { return m < 1 ? 1 : cdiv(m, 64); }
__host__ __device__ __forceinline__ int64_t g_sb_hemm_wgs(int64_t m) {
  return cdiv(m, SBHM) * SBNS;
}
// bulge chasing: task (i, k) is step k of sweep i (i = 0 .. n - 2,
// k = 0 .. (n - 2 - i) / SBW); launch t runs the tasks with 2 i + k = t
__host__ __device__ __forceinline__ int64_t g_bc_kmax(int64_t n, int64_t i) {
  return (n - 2 - i) / SBW;
}
__host__ __device__ __forceinline__ int64_t g_bc_ihi(int64_t n, int64_t t) {
  return std::min<int64_t>(t / 2, n - 2);
}
__host__ __device__ __forceinline__ int64_t g_bc_ilo(int64_t n, int64_t t) {
  const int64_t num = SBW * t - n + 2, den = 2 * SBW - 1;
  return num <= 0 ? 0 : cdiv(num, den);
}
__host__ __device__ __forceinline__ int64_t g_bc_tmax(int64_t n) { return n < 2 ? -1 : 2 * (n - 2); }
// stored chase reflectors: sweep i covers rows i + 1 .. n - 1 (its tasks'
// row blocks, in order), packed after the sweeps before it
__host__ __device__ __forceinline__ int64_t g_bc_off(int64_t n, int64_t i) {
  return i * (n - 1) - i * (i - 1) / 2;
}
// panels of stage 1 (columns j0 = p SBW with rows below the band)
__host__ __device__ __forceinline__ int64_t g_sb_npan(int64_t n) {
  return n > SBW ? cdiv(n - SBW, SBW) : 0;
}
// back-transformation through the stage-1 panels: k_bp_part / k_bp_apply
// take BPR panel rows and BPV vectors per workgroup
constexpr int BPR = 512;
constexpr int BPV = 4;
// Rayleigh quotients of the refinement: k_hx_part takes HXR rows of H_mu
// (HXR / 4 per wave) against HXV vectors per workgroup
constexpr int HXR = 16;
constexpr int HXV = 4;
// back-transformation through the chase: k_bx_chase_lds (x in LDS, with
// SBW rows of padding) for blocks up to BXL - SBW rows, k_bx_chase above
constexpr int BXL = 10240;                // rows of x held in LDS
constexpr int BXT = 512;                  // threads of k_bx_chase_lds
constexpr int BXQ = 4;                    // rows per lane
constexpr int BXW = SBW / BXQ;            // lanes per task
constexpr int BXGL = BXT / BXW;           // tasks per round
constexpr int BXRL = ((BXL - 2) / SBW + 1 + BXGL - 1) / BXGL;  // rounds per sweep
static_assert(BXL * 16 <= 160 * 1024, "x of k_bx_chase_lds fills at most the LDS");
constexpr int BXC = 1024;                 // threads of k_bx_chase
constexpr int BXG = BXC / SBW;            // task groups
constexpr int BXU = 4;                    // tasks per group and batch
// rows of the stage-1 panels before panel p (panel p has n - SBW (p + 1) rows)
__host__ __device__ __forceinline__ int64_t g_sb_voff(int64_t n, int64_t p) {
  return p * (n - SBW) - SBW * (p * (p - 1) / 2);
}

// relative cluster tolerance of the weights: 8 eps sqrt(n) of the storage type of A
__host__ __device__ __forceinline__ double ctol_rel(int64_t n, bool a_fp64) {
  const double eps_w = a_fp64 ? 2.2e-16 : 1.2e-7;
  return 8.0 * eps_w * sqrt(double(n));
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lays out one block's workspace at base (nullptr: size only).
inline size_t ws_layout(int64_t n, bool a_fp64, Desc *w, char *base, int64_t K = 0,
                        bool two_stage = false) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const int64_t lda = (n + 15) / 16 * 16, ldv = (n + 63) / 64 * 64;
  const size_t R = size_t(g_records(n)), P2 = size_t(g_nwg(n));
  Desc t{};
  t.n = n;
  t.lda = lda;
  t.ldv = ldv;
  t.A = take(size_t(n) * lda * (a_fp64 ? 16 : 8));
  t.V = (double2 *)take(size_t(ldv) * NBK * 16);
  t.W = (double2 *)take(size_t(ldv) * NBK * 16);
  t.col = (double2 *)take(size_t(n) * 16);
  t.y = (double2 *)take(size_t(n) * 16);
  const bool tiles = n - 1 > TILE_M;
  const int64_t slots = tiles ? g_yslots(n) : 0;
  t.ldys = n;
  t.ys = tiles ? (double2 *)take(size_t(slots) * size_t(n) * 16) : nullptr;
  t.wraw = (double2 *)take(size_t(n) * 16);
  t.vbuf = (double2 *)take(size_t(n) * 16);
  t.partb0 = (double2 *)take(R * PS * 16);
  t.partb1 = (double2 *)take(R * PS * 16);
  t.parta = (double2 *)take(size_t(std::max<int64_t>(std::max<int64_t>(n, 1), slots * (slots + 1) / 2)) * 16);
  t.bred = (double2 *)take(2 * NBK * 16);
  t.part2 = (double2 *)take(P2 * 16);
  t.part3 = (double *)take(P2 * 8);
  t.scl = (double2 *)take(size_t(n + 1) * 16);
  t.tau = (double2 *)take(size_t(n + 1) * 16);
  t.d = (double *)take(size_t(n) * 8);
  t.e = (double *)take(size_t(n) * 8);
  t.e2 = (double *)take(size_t(n) * 8);
  t.tsc = (double *)take(8 * 8);
  t.bgrid = (int *)take(NGRID * 4);
  t.beta0 = (double *)take(8);
  t.status = (int32_t *)take(4 * 4);
  t.K = K;
  if (K > 0) {
    t.Vall = two_stage ? nullptr : (double2 *)take(size_t(n) * ldv * 16);
    t.Z = (double *)take(size_t(K) * n * 8);
    t.X = (double2 *)take(size_t(K) * n * 16);
    t.rqp = (double *)take(size_t(K) * size_t(cdiv(n, HXR)) * 16);
    t.scr = (double *)take(size_t(K) * (6 * CMAX) * n * 8);
    t.wref = (double *)take(size_t(K) * 8);
    t.Tm = (double2 *)take(size_t(std::max<int64_t>(cdiv(n - 1, NBK), 1)) * NBK * NBK * 16);
    t.clo = (int32_t *)take(size_t(n) * 4);
  }
  if (two_stage) {  // appended, so the regions above keep their offsets
    const size_t nw = size_t(g_sb_nw(n));
    t.pb = (double2 *)take(size_t(n) * SBW * 16);
    t.grec = (double2 *)take(2 * nw * SBW * 16);
    t.srec = (double2 *)take(nw * SBW * SBW * 16);
    t.sbt = (double2 *)take(SBW * SBW * 16);
    t.sbz = (double2 *)take(SBW * SBW * 16);
    t.sbsc = (double2 *)take(2 * SBW * 16);
    t.ptop = (double2 *)take(2 * SBW * 16);
    t.u = take(size_t(SBW) * ldv * (a_fp64 ? 16 : 8));
    t.xp = (double2 *)take(size_t(SBNS) * SBW * ldv * 16);
    t.yrec = (double2 *)take(size_t(g_sb_nx(n)) * SBW * SBW * 16);
    t.band = (double2 *)take(size_t(n) * LDB * 16);
    t.rfl = (double2 *)take(size_t(n) * SBW * 16);
    t.rtau = (double2 *)take(size_t(n) * 16);
    t.sink = (double2 *)take(SINK * 16);
    if (K > 0) {
      t.rall = (double2 *)take(size_t(std::max<int64_t>(g_bc_off(n, n - 1), 1)) * 16);
      t.vrow = (double2 *)take(size_t(std::max<int64_t>(g_sb_voff(n, g_sb_npan(n)), 1)) * SBW * 16);
      t.bxw = (double2 *)take(size_t(cdiv(n, BPR)) * K * SBW * 16);
    }
  }
  if (w) *w = t;
  return off;
}

// workgroups of one launch kind for one block (0 = the block is not active)
enum Kind { K_COPY, K_LOADB, K_HEMV0, K_W0, K_RANK2, K_COL0, K_COLA, K_COLB, K_HER2K, K_TRI,
            K_BISECT, K_WEIGHTS, K_TAIL, K_BGRID };

template <typename TA>
int64_t kind_wgs(int kind, int64_t n, int64_t j, int wpr, int htile = 0) {
  switch (kind) {
    case K_COPY: return n * g_copy_gx(n);
    case K_LOADB: return g_nwg(n);
    case K_HEMV0: return cdiv(n, 4 * g_rpw(n));
    case K_W0: return g_nwg(n);
    case K_RANK2: return n * g_rank2_gx(n);
    case K_COL0: return j < g_tail0(n) ? g_nwg(n - j) : 0;
    case K_COLA:
      if (j >= g_tail0(n)) return 0;
      return wpr < 0 ? g_tiles(n, j + 1, tile_of(wpr)) : g_colA_wgs(n - j - 1, wpr);
    case K_COLB: return j < g_tail0(n) ? cdiv(n - j - 1, RB) : 0;
    case K_HER2K: {
      if (j >= g_tail0(n)) return 0;
      const int64_t c0 = j + g_nbk(n, j), m = n - c0;
      const int bn = htile ? HerTile<TA, 1>::BN : HerTile<TA, 0>::BN;
      const int64_t t = cdiv(m, bn);  // tile rows (see b_her2k)
      return m > 0 ? (her_tri(t, bn) ? t * (t + 1) / 2 : t * t) : 0;
    }
    case K_TRI: return 1;
    case K_BGRID: return NGRID / ENT;
    default: return cdiv(n, 4);  // bisect, weights
  }
}

}  // namespace bse
