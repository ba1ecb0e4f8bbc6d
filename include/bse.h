/*
 * bse.h -- C ABI of the symmetry-blocked Bethe-Salpeter hot path for MI355X.
 *
 * The library builds the Tamm-Dancoff electron-hole Hamiltonian
 *     H[(k v c),(k' v' c')] = delta (E_c(k) - E_v(k))
 *                           + (2/N_k) sum_I Mx[k,v,c,I] v_I conj(Mx[k',v',c',I])
 *                           - (1/N_k) sum_IJ conj(Mc[k,k'][c,c',I]) W_IJ(k-k') Mv[k,k'][v,v',J]
 * (paper: Eq. (BSE-eigval) with the vector-matrix-vector form of Eq.
 * (w_interaction2); the spin factor 2 on the bare exchange for a non-magnetic
 * system is stated at the end of Sec. II), projects it onto symmetry-adapted
 * irrep blocks H_mu = U_mu^T H U_mu (Eq. (projection), Eq. (transformationU),
 * Sec. III.C.4), diagonalises the dipole-active block (Sec. III.D.1) and forms
 * eps2(w) (Eqs. (macro_diel), (reducible_polar), (oscillatorA)).
 *
 * Conventions shared by every entry point
 *   - k linear index  lin(k) = (k1 n2 + k2) n3 + k3; product index
 *     a = (k nv + v) nc + c; pair index p = k nk + k'; q = k - k' (mod grid).
 *   - Complex numbers are interleaved (re, im); all arrays are row-major.
 *   - Pointers named h_* are host memory; every other array pointer is device
 *     memory (hipMalloc / a torch CUDA tensor).  The caller owns all memory;
 *     the library never frees or keeps a caller pointer after a call returns.
 *   - Device work is enqueued on `stream` (a hipStream_t, NULL = default
 *     stream) and is complete when the stream is synchronised.
 *   - Every entry point validates shapes and ranges before launching anything
 *     and returns BSE_ESHAPE / BSE_EINVAL without touching outputs.  A HIP error
 *     maps to BSE_EDEVICE.  bse_last_error() returns a thread-local message for
 *     the last non-OK status.  No C++ exception crosses this interface.
 *   - Calls on one stream are serialised by the stream; concurrent calls on
 *     different streams are safe when their output buffers do not overlap.
 */
#ifndef BSE_H
#define BSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *bse_stream; /* hipStream_t */

enum {
  BSE_OK = 0,
  BSE_EINVAL = -1,       /* bad argument value (NULL pointer, unknown enum)  */
  BSE_ESHAPE = -2,       /* inconsistent or unsupported sizes                */
  BSE_EWORKSPACE = -3,   /* workspace smaller than the *_ws query requires   */
  BSE_EDEVICE = -4,      /* a HIP runtime call failed                        */
  BSE_ENOCONV = -5,      /* an iteration did not converge                    */
  BSE_EUNSUPPORTED = -6  /* valid request the library does not implement    */
};

enum { /* arithmetic of the contractions */
  BSE_FP64 = 0,   /* complex FP64 inputs, FP64 MFMA, FP64 H                   */
  BSE_FP32 = 1,   /* complex FP32 inputs, FP32 MFMA, FP32 H                   */
  BSE_BF16X3 = 2  /* FP32 inputs split hi+lo into BF16, three BF16 MFMA
                     products (hi*hi + hi*lo + lo*hi) accumulated in FP32     */
};

enum { BSE_GROUP_OH = 0, BSE_GROUP_D6H = 1 };

const char *bse_last_error(void);
const char *bse_version(void);

/* ---------------------------------------------------------------------------
 * Point groups (Sec. III.C.1, Eq. (sk); characters Sec. III.C.4, Eq. (LOT)).
 * Oh: the 48 signed permutation matrices acting on cubic reduced k.
 * D6h: 24 operations, reduced reciprocal basis b1 = (1, 1/sqrt3),
 * b2 = (0, 2/sqrt3); two-fold axes C2' along a1, a2, a1+a2.
 * ------------------------------------------------------------------------- */
int32_t bse_group_order(int32_t group);                  /* 48, 24, or <0    */
int32_t bse_group_nirreps(int32_t group);                /* 10, 12, or <0    */
/* h_kmat[nops][3][3]: integer action on reduced k; h_rcart[nops][3][3]:
 * Cartesian matrix (either may be NULL). */
int32_t bse_group_ops(int32_t group, int32_t *h_kmat, double *h_rcart);
/* name (NUL-terminated, <= 7 chars), dimension and characters chi[nops]. */
int32_t bse_group_irrep(int32_t group, int32_t irrep, char *h_name8, int32_t *h_dim,
                        double *h_chi);

/* ---------------------------------------------------------------------------
 * Integer tables (host).  Orbits under the group action on the grid
 * (Sec. III.C.2: pairs related by one operation share their elements; q loop
 * outermost).  Canonical orbit representative = smallest linear index; orbit
 * ids increase with the representative.  Pair orbits are taken under the
 * diagonal action (k,k') -> (s k, s k'); the swap partner of a pair orbit is
 * the orbit of (k', k).  A storage class is {orbit, swap partner}, stored once
 * in the orientation of the smaller orbit id; classes are numbered by that id.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t grid[3];
  int32_t nk, nops, nkorb, nporb, ncls;
} bse_dims;

typedef struct {              /* host buffers, sizes from bse_dims           */
  int32_t *kperm;             /* [nops][nk]   lin(A_s k mod grid)            */
  int32_t *korb;              /* [nk]         k-orbit id (also the q orbit)  */
  int32_t *korb_rep;          /* [nkorb]      representative k of each orbit */
  int32_t *porb;              /* [nk*nk]      pair-orbit id of (k,k')        */
  int32_t *porb_rep;          /* [nporb]      representative pair index      */
  int32_t *pidx;              /* [nk*nk]      storage class of (k,k')        */
  uint8_t *pconj;             /* [nk*nk]      1: M(k,k') is the band-conjugate
                                              transpose of the stored class */
  int32_t *cls_rep;           /* [ncls]       pair index of the stored orientation */
  uint8_t *cls_selfswap;      /* [ncls]       class orbit is its own swap partner */
} bse_tables;

int32_t bse_dims_get(int32_t group, const int32_t *h_grid3, bse_dims *h_out);
/* Any member pointer of `out` may be NULL to skip that table. */
int32_t bse_tables_build(int32_t group, const int32_t *h_grid3, const bse_tables *h_out);

/* ---------------------------------------------------------------------------
 * Symmetry-adapted basis of one irrep (host, FP64).  For every k orbit O the
 * projector P_mu = d_mu/|S| sum_s chi_mu(s) Gamma(s) (Eq. (projection)) is
 * applied to the orbit's unit vectors and the result orthonormalised
 * (Sec. III.C.4: the projector acts within one orbit, at most |S| d_max^2
 * non-zeros per vector).  The band indices are spectators (the single-particle
 * representation is the identity on bands), so the block basis is
 * U_O (x) identity(nv nc).  Block layout: orbits in id order, then the
 * orbit's r_O basis vectors, then (v, c) with c fastest:
 *     row = orb_off[O] + j nv nc + v nc + c.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t n;        /* block dimension                                       */
  int32_t nmem;     /* = nk                                                   */
  int64_t nub;      /* number of basis coefficients: sum_O |O| r_O            */
} bse_block_dims;

int32_t bse_block_dims_get(int32_t group, const int32_t *h_grid3, int32_t irrep, int32_t nv,
                           int32_t nc, bse_block_dims *h_out);
/* h_mem_off[nkorb+1], h_members[nk]: k points of each orbit, ascending;
 * h_orb_off[nkorb]: first block row; h_orb_dim[nkorb]: r_O;
 * h_ub_off[nkorb+1], h_ubasis[nub]: U_O row-major |O| x r_O (FP64). */
int32_t bse_block_basis(int32_t group, const int32_t *h_grid3, int32_t irrep, int32_t nv,
                        int32_t nc, int32_t *h_mem_off, int32_t *h_members,
                        int64_t *h_orb_off, int32_t *h_orb_dim, int64_t *h_ub_off,
                        double *h_ubasis);

/* Partner-resolved block of a vector irrep (T1u of Oh; E1u and A2u of D6h):
 * the projector P_pp = d_mu/|S| sum_s Gamma_mu(s)_pp Gamma(s) onto one row p
 * of the irrep, whose matrices for a vector irrep are the Cartesian rotation
 * matrices R_s themselves (p = 0, 1, 2 for x, y, z of T1u; 0, 1 for x, y of
 * E1u; 0 for z of A2u).  The block has 1/d_mu of the isotypic block's
 * dimension and every eigenvalue of the isotypic block once instead of d_mu
 * times (partner functions are degenerate); a dipole polarised along
 * Cartesian axis i lies entirely in the block of the row along i.  Same
 * output layout as bse_block_basis; other irreps: BSE_EUNSUPPORTED. */
int32_t bse_partner_block_dims_get(int32_t group, const int32_t *h_grid3, int32_t irrep,
                                   int32_t partner, int32_t nv, int32_t nc,
                                   bse_block_dims *h_out);
int32_t bse_partner_block_basis(int32_t group, const int32_t *h_grid3, int32_t irrep,
                                int32_t partner, int32_t nv, int32_t nc, int32_t *h_mem_off,
                                int32_t *h_members, int64_t *h_orb_off, int32_t *h_orb_dim,
                                int64_t *h_ub_off, double *h_ubasis);

/* ---------------------------------------------------------------------------
 * bse_build: H (N x N, N = nk nv nc) from orbit-compressed inputs.
 * Dense mode: every (k, k') pair is contracted (the kernels never assume that
 * symmetric pairs hold equal data).  All device pointers.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t grid[3];
  int32_t nv, nc, nmb;
  int32_t nkorb, ncls, nqorb;
  const int32_t *korb;   /* [nk]     k-orbit id of each k (indexes mx)          */
  const int32_t *qorb;   /* [nk]     q-orbit id of each q (indexes w)           */
  const int32_t *pidx;   /* [nk*nk]  storage class of (k,k') (indexes mv, mc)   */
  const uint8_t *pconj;  /* [nk*nk]  1: use the band-conjugate transpose        */
  const double *ev;      /* [nk][nv] valence energies (eV)                      */
  const double *ec;      /* [nk][nc] conduction energies (eV)                   */
  const double *vdiag;   /* [nmb]    diagonal bare Coulomb matrix v_I           */
  const void *mx;        /* [nkorb][nv][nc][nmb] complex                        */
  const void *mv;        /* [ncls][nv][nv][nmb]  complex                        */
  const void *mc;        /* [ncls][nc][nc][nmb]  complex                        */
  const void *w;         /* [nqorb][nmb][nmb]    real symmetric                 */
  int32_t in_fp64;       /* element type of mx, mv, mc, w: 1 double, 0 float    */
} bse_problem;

/* Workspace bytes that let bse_build run its direct term in the fewest passes
 * (capped; any size >= bse_build_ws_min works).  BF16X3 needs exactly
 * bse_build_ws_min = bse_build_ws: the BF16 hi and lo planes of W
 * (4 nqorb nmb^2 bytes), written at the start of every build; the workspace
 * must be 16-byte aligned (BSE_EWORKSPACE if smaller, BSE_EINVAL if
 * misaligned). */
size_t bse_build_ws(const bse_problem *p, int32_t prec);
size_t bse_build_ws_min(const bse_problem *p, int32_t prec);
/* H: complex double (prec FP64) or complex float (FP32, BF16X3), leading
 * dimension ldh >= N elements.  prec FP64 needs in_fp64 = 1, the others 0. */
int32_t bse_build(const bse_problem *p, int32_t prec, void *H, int64_t ldh, void *ws,
                  size_t ws_bytes, bse_stream stream);

/* ---------------------------------------------------------------------------
 * Seed (symmetry-accelerated) construction of the same H as bse_build
 * (Sec. III.C.2, Eq. (Wtrafo): pairs (s k, s k') related by an operation share
 * their interaction elements, and with band-trivial symmetry operations the
 * rotation of the bands is the identity).  The direct term is contracted only
 * for one representative pair per pair orbit and the exchange for one k point
 * per k orbit; a final pass writes every element of H from these pieces.
 *   bse_seed_ws     workspace bytes (0 on invalid input or unsupported shape)
 *   bse_seed_plan   builds the orbit tables of (group, p->grid) on the host,
 *                   the q-grouped work list, and uploads them into ws
 *                   (synchronises `stream`); *h_plan receives the plan id.  The
 *                   problem's device arrays must stay valid while the plan is
 *                   used (the plan keeps a copy of the struct).
 *   bse_build_seed  writes H (N x N, leading dimension ldh, complex of the
 *                   plan's precision) on `stream`; kernel launches only.
 *                   H = NULL computes the pieces only (for bse_project_seed).
 *   bse_project_seed  projects blocks straight from the pieces of the last
 *                   bse_build_seed on the plan, without materialising H: the
 *                   same bse_block descriptors and H_mu layout as
 *                   bse_project_blocks (Hmu[i], ldmu[i]; NULL skips a block),
 *                   element type of the plan's precision.  Every element of H
 *                   is formed on the fly as the assembly forms it and rounded
 *                   to that precision, so the result equals bse_project_blocks
 *                   of the assembled H exactly.  Kernel launches only; stream
 *                   order with bse_build_seed is the caller's.  B_mu still
 *                   comes from bse_project_blocks (H = NULL).  Errors:
 *                   BSE_EINVAL (unknown plan, NULL block arrays), BSE_ESHAPE
 *                   (ldmu < n), BSE_EUNSUPPORTED (nv nc too large).
 *   bse_seed_free   forgets the plan.
 * Precision FP32 or FP64; shapes as the fused direct kernel (Nmb = 64 m with
 * m <= 6, nv <= 4, nc <= 6), else BSE_EUNSUPPORTED.
 * ------------------------------------------------------------------------- */
size_t bse_seed_ws(int32_t group, const bse_problem *p, int32_t prec);
int32_t bse_seed_plan(int32_t group, const bse_problem *p, int32_t prec, void *ws,
                      size_t ws_bytes, int64_t *h_plan, bse_stream stream);
int32_t bse_build_seed(int64_t plan, void *H, int64_t ldh, bse_stream stream);
int32_t bse_seed_free(int64_t plan);

/* ---------------------------------------------------------------------------
 * bse_project_blocks: H_mu = U_mu^T H U_mu and B_mu = U_mu^T B for nblk blocks
 * (Eq. (transformationU) applied irrep-wise).  Per block, Hmu[i] may be NULL
 * (only B_mu wanted) and Bmu[i] may be NULL.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t n;                 /* block dimension                               */
  const int32_t *mem_off;    /* device [nkorb+1]                              */
  const int32_t *members;    /* device [nk]                                   */
  const int64_t *orb_off;    /* device [nkorb]                                */
  const int32_t *orb_dim;    /* device [nkorb]                                */
  const int64_t *ub_off;     /* device [nkorb+1]                              */
  const double *ubasis;      /* device [nub]                                  */
} bse_block;

/* H element type: h_fp64 = 1 complex double, 0 complex float; H_mu has the
 * same type with leading dimension ldmu[i] >= n.  B, B_mu: complex double. */
int32_t bse_project_blocks(const bse_problem *p, const void *H, int64_t ldh, int32_t h_fp64,
                           const void *B, int32_t nblk, const bse_block *h_blk,
                           void *const *h_Hmu, const int64_t *h_ldmu, void *const *h_Bmu,
                           bse_stream stream);
/* bse_project_seed: see the seed construction above (Sec. III.C.2 with
 * Eq. (transformationU)): blocks projected from a seed plan's pieces. */
int32_t bse_project_seed(int64_t plan, int32_t nblk, const bse_block *h_blk, void *const *h_Hmu,
                         const int64_t *h_ldmu, bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_dipole_weights: which irrep blocks the light couples to (Sec. III.D.1:
 * only blocks with a non-zero projected dipole contribute to eps2; Eq.
 * (oscillatorA) with B_mu = U_mu^T B).  For each of the nblk blocks (the
 * bse_block descriptors of bse_project_blocks) it computes
 *     weights[i] = |U_mu^T B|^2 = sum_l |B_l|^2 over that block's states,
 * and active[0] = the index of the block with the largest weight, provided
 * that weight exceeds 1e-12 of the sum over the listed blocks (the first such
 * block on ties), else -1.  Summed in a fixed order (bitwise reproducible).
 *   B        device complex double[N], N = nk nv nc.
 *   weights  device double[nblk] output;  active  device int32[1] output.
 * Errors: BSE_EINVAL (NULL pointers, nblk < 1, NULL block arrays),
 * BSE_ESHAPE (bad problem sizes, block larger than N).  Kernel launches
 * only, on `stream`.
 * ------------------------------------------------------------------------- */
int32_t bse_dipole_weights(const bse_problem *p, const void *B, int32_t nblk,
                           const bse_block *h_blk, double *weights, int32_t *active,
                           bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_block_eigh: eigenvalues of the Hermitian block and the oscillator
 * strengths |B_l|^2 = |A_l^dag B_mu|^2 (Eq. (oscillatorA)).
 * Method: a Householder reflection maps B_mu onto |B_mu| e_1; a blocked
 * Householder tridiagonalisation that leaves e_1 fixed follows; then
 * |B_l|^2 = |B_mu|^2 z_l(1)^2 with z_l the eigenvectors of the real
 * tridiagonal T, so eps2 needs no eigenvectors.  Only the leading unreduced
 * block of T (the Krylov space of B_mu) carries weight.
 * Outputs (device FP64): omega[n] all eigenvalues ascending (with
 * multiplicity); pole[n], osc[n]: the optical poles and their strengths,
 * padded with zero strength.  Hmu is read only.
 * prec: FP64 (all FP64), FP32 (FP32 storage of the working copy, its HEMV
 * and trailing updates; FP64 panel vectors, scalars and tridiagonal step).
 * The HEMV of trailing blocks above 2048 rows reads only their lower half;
 * its partial sums take up to max(49, (n + 63) / 256) x n x 16 B more
 * workspace (n > 2049).
 * nrefine = K in 0 .. 256: FP64 refinement of the lowest min(K, n)
 * eigenvalues against the stored Hmu: inverse iteration on T (members of a
 * cluster orthogonalised; the clusters are those of the optical weights:
 * gaps within 8 eps sqrt(n) |T| of the working storage, split at FP64
 * resolution where such a chain is wide), back-transformation through the kept
 * reflectors and the Rayleigh quotient Re(x^dag Hmu x) / |x|^2, which is exact
 * to O(delta^2 |Hmu|) for an eigenvector error delta; omega[0 .. K) then holds
 * the refined values (ascending) and the poles of clusters inside that range
 * are re-centred.  It removes the eigensolver's rounding, not errors already
 * in Hmu.  The workspace grows by about n^2 16 B (all reflectors of either
 * reduction) plus 400 K n B (inverse-iteration scratch) for K > 0.
 * Errors: n < 1 or n > 65536 (BSE_ESHAPE), NULL pointers or nrefine outside
 * 0 .. 256 (BSE_EINVAL), ws_bytes < bse_block_eigh_ws (BSE_EWORKSPACE).  The
 * call only enqueues kernels; eigenvalues it could not refine (clusters of
 * more than 8 members) or non-finite results are reported afterwards by
 * bse_block_eigh_status (BSE_ENOCONV).
 * ------------------------------------------------------------------------- */
size_t bse_block_eigh_ws(int64_t n, int32_t h_fp64, int32_t prec, int32_t nrefine);
int32_t bse_block_eigh(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64, const void *Bmu,
                       int32_t prec, int32_t nrefine, double *omega, double *pole,
                       double *osc, void *ws, size_t ws_bytes, bse_stream stream);

/* ---------------------------------------------------------------------------
 * Two-stage reduction of large blocks (the same outputs as bse_block_eigh).
 * Solves with n >= the switch point reduce H_mu in two
 * stages that both leave e_1 fixed: first to a lower band of half-width 32
 * (panels of 32 columns: a QR of the panel below the band with one reduction
 * per column, then the two-sided update A22 - V W^dag - W V^dag of the
 * trailing block with X = A22 V T formed on the matrix cores), then from the
 * band to the real tridiagonal by chasing each column's bulge down the band
 * (one task of one wave per step; launch t runs every step k of sweep i with
 * 2 i + k = t).  The tridiagonal step is the one above.  FP32 storage keeps
 * the working copy in FP32 (its products summed in FP64 every 128 terms);
 * the panel, the band and the chase are FP64.  The workspace grows by about
 * 6.5 KB per row of the block (66 MB at n = 10080).  With nrefine > 0 the
 * chase keeps every reflector it makes (n (n - 1) / 2 entries of 16 B) and
 * stage 1 every panel (about n^2 / 2 entries); the eigenvectors of T go back
 * through both, in reverse order, before the Rayleigh quotients.  The kept
 * chase is compiled apart from the plain one: the unrefined part of the
 * spectrum may differ from an unrefined solve in the last FP64 bits.
 * bse_block_eigh_set_two_stage(nmin) sets the switch point to nmin (>= 2;
 * default 4096) and returns the previous one; nmin < 0 only returns it.  It
 * is process-wide: query bse_block_eigh_ws after setting it, and do not
 * change it while solves sized under the old value are pending.  The
 * allocation-free and batched solvers keep the one-stage reduction.
 * ------------------------------------------------------------------------- */
int64_t bse_block_eigh_set_two_stage(int64_t nmin);

/* ---------------------------------------------------------------------------
 * bse_block_eigh_status: what the last solve on a workspace could not do.
 * Synchronises `stream` and reads four counters that every solve rewrites:
 *   h_status[0]  eigenvalues among the lowest min(nrefine, n) left unrefined
 *                (their omega is the unrefined FP64 bisection value): members
 *                of a degenerate cluster beyond its first 8, whose inverse
 *                iteration is not run, or a Rayleigh quotient that is not finite;
 *   h_status[1]  eigenvalues that are not finite (the tridiagonal step met a
 *                non-finite matrix; outputs undefined);
 *   h_status[2]  clusters that straddle the refinement bound K (their members
 *                below K are refined, their pole stays the unrefined centre);
 *   h_status[3]  0 (reserved).
 * Arguments n, prec, nrefine as in the solve; ws its workspace, or NULL for
 * the static workspace of bse_block_eigh_noalloc on the current device.
 * Returns BSE_ENOCONV when h_status[0] or h_status[1] is non-zero, else
 * BSE_OK; BSE_ESHAPE / BSE_EINVAL for bad arguments, BSE_EDEVICE when the copy
 * fails.  Not for use under graph capture (it copies to the host).
 * ------------------------------------------------------------------------- */
int32_t bse_block_eigh_status(int64_t n, int32_t prec, int32_t nrefine, const void *ws,
                              int32_t *h_status, bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_block_eigh_noalloc: bse_block_eigh for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, computation, kernels and results
 * as bse_block_eigh, without ws / ws_bytes: the workspace is a static device
 * array of bse_block_eigh_noalloc_max() bytes (128 MiB) in the library, one
 * per GPU, held from the first call on that GPU until the process ends.  No
 * hipMalloc, hipFree or allocating library call is made.  That fits, for
 * example, FP32 blocks up to n = 3900 without refinement and up to n = 1500
 * with nrefine = 100 (the limit is the one-stage bse_block_eigh_ws(n, ...) <=
the maximum: this solver always takes the one-stage reduction).
 * No part of the array needs to start at zero: every word a kernel reads was
 * written earlier in the same call.
 * The first call on a device looks up the array's device address (the
 * device must be current and `stream` must belong to it).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different host threads) race and give undefined results;
 * serialise them.  The outputs stay valid after later calls (they are the
 * caller's buffers, not the scratch).
 * Errors: those of bse_block_eigh; BSE_EWORKSPACE when the block needs more
 * workspace than the array holds; BSE_EINVAL when `stream` belongs to
 * another device than the current one; BSE_EDEVICE when the address lookup
 * fails.
 * ------------------------------------------------------------------------- */
size_t bse_block_eigh_noalloc_max(void);
int32_t bse_block_eigh_noalloc(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64,
                               const void *Bmu, int32_t prec, int32_t nrefine, double *omega,
                               double *pole, double *osc, bse_stream stream);

/* ---------------------------------------------------------------------------
 * Batched block eigensolver: the same computation as bse_block_eigh for nb
 * independent blocks (all irrep blocks of many systems, Sec. III.D.1 per
 * block), run in lockstep: every launch advances every block that still has
 * columns left by one step, so the per-column launch latency is paid once
 * per column of the largest block instead of once per column of every block.
 *   bse_batch_eigh_ws      workspace bytes for blocks of sizes h_n[nb]
 *   bse_batch_eigh_plan    validates the blocks, lays out the workspace, and
 *                          uploads the per-block descriptors and launch tables
 *                          (synchronises `stream`); returns a plan id in
 *                          *h_plan.  All pointers in the host arrays are device
 *                          pointers that must stay valid while the plan runs:
 *                          h_Hmu[b] (n x n, leading dim h_ld[b], complex double
 *                          if h_fp64 else complex float, read only), h_Bmu[b]
 *                          (complex double), h_omega/h_pole/h_osc[b] (double[n],
 *                          outputs as in bse_block_eigh).
 *   bse_batch_eigh_run     enqueues the whole solve on `stream`: kernel launches
 *                          only, so it may be captured into a HIP graph.
 *   bse_batch_eigh_tune    autotuner: times every combination of the HEMV
 *                          kernel's row split (1, 2 or 4 waves per row) and the
 *                          trailing update's tile (64 x 64 or 32 x 32 complex
 *                          entries) on this batch, keeps the fastest for the
 *                          plan and returns it in *h_wpr and *h_tile (tile edge
 *                          in entries; either may be NULL); runs the solve
 *                          several times (outputs are overwritten).  It
 *                          rewrites the plan's device launch tables: a graph
 *                          captured from bse_batch_eigh_run before a tune keeps
 *                          the old grid sizes and must not be replayed after
 *                          it (tune first, then capture).
 *   bse_batch_eigh_config  sets the row split (1, 2, 4) and tile edge (64, 32)
 *                          explicitly, as the tuner would (same caveat for
 *                          captured graphs; synchronises `stream`).
 *   bse_batch_eigh_free    forgets the plan (the caller frees the workspace).
 * Limits: 1 <= nb <= 1024 and 1 <= n <= 16384 per block (BSE_ESHAPE);
 * prec FP64 or FP32 (BSE_EINVAL).  Plans are kept per process; a plan must
 * not be run on two streams at once (the workspace is shared).
 * ------------------------------------------------------------------------- */
size_t bse_batch_eigh_ws(int32_t nb, const int64_t *h_n, int32_t h_fp64, int32_t prec);
int32_t bse_batch_eigh_plan(int32_t nb, const int64_t *h_n, const void *const *h_Hmu,
                            const int64_t *h_ld, int32_t h_fp64, const void *const *h_Bmu,
                            int32_t prec, double *const *h_omega, double *const *h_pole,
                            double *const *h_osc, void *ws, size_t ws_bytes, int64_t *h_plan,
                            bse_stream stream);
int32_t bse_batch_eigh_run(int64_t plan, bse_stream stream);
int32_t bse_batch_eigh_tune(int64_t plan, bse_stream stream, int32_t *h_wpr,
                            int32_t *h_tile);
int32_t bse_batch_eigh_config(int64_t plan, int32_t wpr, int32_t tile, bse_stream stream);
int32_t bse_batch_eigh_free(int64_t plan);

/* ---------------------------------------------------------------------------
 * bse_spectrum: eps2[j] = pref sum_l osc[l] [L(w_j - pole_l) + L(w_j + pole_l)],
 * L(x) = eta / (x^2 + eta^2); pref = 8 pi / N_k for the spin-degenerate case
 * (Eqs. (macro_diel), (reducible_polar)).  Device FP64 arrays.
 * ------------------------------------------------------------------------- */
int32_t bse_spectrum(int64_t n, const double *pole, const double *osc, double pref, double eta,
                     int64_t nw, const double *w, double *eps2, bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_eels: longitudinal excitons of one block from its optical poles
 * (Sec. III.D.2, Eqs. (secular), (eigenvec_xi)).  Adding the G = 0 Coulomb
 * term c B B^dag to H_mu leaves dark directions unchanged and moves every
 * weighted pole p_i (strength w_i) to a root x of
 *     1 - c sum_i w_i / (x - p_i) = 0,
 * one in each interval between consecutive weighted poles and one in
 * (p_m, p_m + c sum w), with strength 1 / (c^2 sum_i w_i / (x - p_i)^2).
 *   pole, osc   device double[n], the output of bse_block_eigh (ascending
 *               poles; entries with osc <= 1e-14 sum(osc), i.e. dark clusters
 *               and non-leading cluster members, are not poles of the sum)
 *   c           coupling > 0; 8 pi / N_k for the spin-degenerate exchange
 *               (the same prefactor as the exchange and eps2)
 *   xpole, xosc device double[n] outputs: the m roots (ascending) and their
 *               strengths, then n - m entries (0, 0); pass them to bse_spectrum
 *               for the loss spectrum.  They may not alias pole/osc.
 *   ws          device workspace of bse_eels_ws(n) bytes (caller owned).
 * Errors: BSE_ESHAPE (n < 1), BSE_EINVAL (NULL pointer, c <= 0),
 * BSE_EWORKSPACE.  Asynchronous on `stream`; launches kernels only.
 * ------------------------------------------------------------------------- */
size_t bse_eels_ws(int64_t n);
int32_t bse_eels(int64_t n, const double *pole, const double *osc, double c, double *xpole,
                 double *xosc, void *ws, size_t ws_bytes, bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_haydock: eps2 of one block without diagonalising it: Lanczos-Haydock,
 * which profits from the block-diagonal form of H as the eigensolver does
 * (Sec. III.D.1).  Lanczos on H_mu started from B_mu / |B_mu| (classical
 * recurrence, no reorthogonalisation):
 *     w = H v_j - b_j v_{j-1},  a_j = Re v_j^dag w,  w -= a_j v_j,
 *     b_{j+1} = |w|,  v_{j+1} = w / b_{j+1},
 * with b_0 = |B_mu| and v_{-1} = 0.
 *   Hmu    device, n x n, row-major with leading dimension ld >= n, complex
 *          double if h_fp64 else complex float; the full matrix (both
 *          triangles, as bse_project_blocks writes it) is read; read only.
 *   Bmu    device complex double[n].
 *   K      steps, 1 .. 2^20.
 *   a, b   device double outputs: a[0..K), b[0..K] (b[0] = |B_mu|, b[K] the
 *          norm of the last residual).  A residual that vanishes exactly
 *          (invariant Krylov space) zeroes the later coefficients.
 *   ws     device workspace of bse_haydock_ws(n) bytes (caller owned).
 * Cost: K dependent kernels, each reading H_mu once (FP64 arithmetic).
 * bse_haydock_spectrum: eps2(w_j) = pref b_0^2 (-Im G(w_j + i eta)
 * - Im G(-w_j + i eta)) with G(z) = 1 / (z - a_0 - b_1^2 / (z - a_1 - ...))
 * truncated after K levels (the resonant and antiresonant terms of
 * bse_spectrum; pref = 8 pi / N_k).  Device FP64 arrays.
 * Errors: BSE_ESHAPE (n < 1, n > 2^20, ld < n, nw < 0), BSE_EINVAL (NULL
 * pointer, K outside 1 .. 2^20, eta <= 0), BSE_EWORKSPACE.  Asynchronous.
 * ------------------------------------------------------------------------- */
size_t bse_haydock_ws(int64_t n);
int32_t bse_haydock(int64_t n, const void *Hmu, int64_t ld, int32_t h_fp64, const void *Bmu,
                    int32_t K, double *a, double *b, void *ws, size_t ws_bytes,
                    bse_stream stream);
int32_t bse_haydock_spectrum(int32_t K, const double *a, const double *b, double pref,
                             double eta, int64_t nw, const double *w, double *eps2,
                             bse_stream stream);

/* ---------------------------------------------------------------------------
 * bse_sync_probe: cost of one global dependency between two steps of a
 * lockstep solve on this device, the design input of the batched form (which
 * pays one per Householder step).  Times `steps` steps of `wgs` workgroups
 * in which every workgroup reads a value another one wrote in the previous
 * step:
 *   mode 0  one kernel launch per step, back to back on `stream`;
 *   mode 1  one cooperative (persistent) launch with a grid-wide barrier
 *           between steps (all workgroups must fit on the device at once).
 *   buf     device int32[2 wgs] scratch (caller owned, overwritten).
 * *h_us_per_step receives the mean time per step in microseconds.
 * Synchronises `stream`.  Errors: BSE_EINVAL (mode, NULL), BSE_ESHAPE (wgs
 * outside 1 .. 4096 or not co-resident for mode 1, steps outside 1 .. 10^6),
 * BSE_EUNSUPPORTED (no cooperative launch), BSE_EDEVICE.
 * ------------------------------------------------------------------------- */
int32_t bse_sync_probe(int32_t mode, int32_t wgs, int32_t steps, int32_t *buf,
                       double *h_us_per_step, bse_stream stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (host).  bse_prof_enable(prefix) brackets every subsequent
 * launch of a library kernel whose name starts with `prefix` with two HIP
 * events on the launch stream ("" or NULL disables; "k_" times every kernel).
 * bse_prof_collect() waits for the recorded events and adds their elapsed time
 * to per-name totals; bse_prof_get() reads name (<= 31 chars), total
 * milliseconds and launch count of entry i < bse_prof_count().  Timing adds
 * two event records per launch, so enable it only for the kernels measured.
 * ------------------------------------------------------------------------- */
int32_t bse_prof_enable(const char *prefix);
int32_t bse_prof_collect(void);
int32_t bse_prof_count(void);
int32_t bse_prof_get(int32_t i, char *h_name32, double *h_total_ms, int64_t *h_launches);
int32_t bse_prof_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
