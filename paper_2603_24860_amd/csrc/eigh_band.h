// Two-stage reduction of one large Hermitian block: full -> lower band of
// half-width SBW -> real symmetric tridiagonal.  Included by bse_eigh.hip
// inside its anonymous namespace (uses its complex helpers, the reflector
// convention `householder`, the MFMA tile core and the trailing update
// b_her2k).
//
// Both stages act only on rows >= 1, so e_1 stays fixed and the optical
// weights follow from the first components of the tridiagonal's
// eigenvectors, as for the one-stage reduction.
//
// Stage 1, panel j0 (columns j0 .. j0 + SBW - 1, panel rows p0 = j0 + SBW ..
// n - 1, m = n - p0 of them): the panel P = A[p0:, j0:j0+SBW] is factored
// P = Q R with Q = I - V T V^dag (reflectors with the zlarfg convention,
// one launch per column: the column's reflector comes from the reduced
// partial sums of its Gram row G_c[j] = sum_{r > c} conj(P[r][c]) P[r][j],
// because |x|^2 = G_c[c] and v^dag P[:, j] = P[c][j] + conj(s) G_c[j]; the
// same launch applies it to its rows and sums the next column's Gram row
// from the updated rows).  Then Q^dag A22 Q = A22 - V W^dag - W V^dag with
// X = A22 V T, Z = T^dag V^dag X and W = X - Z V / 2 (written out: V Z), and
// the update runs on the MFMA trailing-update kernel.
//
// Stage 2 (bulge chasing): sweep i annihilates column i below the
// subdiagonal with a reflector on rows i+1 .. i+SBW and applies it to the
// diagonal block of those rows; the right-hand application to the block
// below creates a bulge whose first column the next step annihilates, and so
// on down the band (the rest of each bulge is removed by later sweeps).  Step
// k of sweep i runs after step k + 1 of sweep i - 1, so launch t runs every
// step with 2 i + k = t.  The band with the fill of one bulge is stored
// column by column, band[c][r - c] for 0 <= r - c < 2 SBW.

// Component-wise select of complex values: a conditional on whole double2
// values can become a select between their memory objects and keep a
// register array in scratch memory.
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
  return double2{c ? a.x : b.x, c ? a.y : b.y};
}

// ---------------------------------------------------------------------------
// stage 1: panel factorisation
// ---------------------------------------------------------------------------
// Sum over the rows of a workgroup: thread t holds a[u] for columns
// 8 (t & 3) + u of its row; out[0 .. SBW) receives the column sums.
template <int NT = ENT>
__device__ __forceinline__ void sb_rowsum(double2 (&a)[8], double2 *sh, double2 *out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) {
      a[u].x += __shfl_xor(a[u].x, o, 64);
      a[u].y += __shfl_xor(a[u].y, o, 64);
    }
  if (lane < 4)
#pragma unroll
    for (int u = 0; u < 8; ++u) sh[wv * SBW + 8 * lane + u] = a[u];
  __syncthreads();
  if (tid < SBW) {
    double2 s = sh[tid];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) s = cadd(s, sh[w * SBW + tid]);
    out[tid] = s;
  }
}

// the value of column c of this thread's row (held by thread 4 row + c / 8).
// The entry is picked by a masked sum, not an index, so that the row stays
// in registers (a variable index would put the array in scratch memory);
// the rows hold finite values.
__device__ __forceinline__ double2 sb_rowval(const double2 (&x)[8], int c) {
  const int lane = threadIdx.x & 63, src = (lane & ~3) | (c >> 3);
  double2 v = {0, 0};
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double f = (c & 7) == u ? 1.0 : 0.0;
    v.x = fma(f, x[u].x, v.x);
    v.y = fma(f, x[u].y, v.y);
  }
  return double2{__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// panel -> pb (FP64) and the partial Gram row of column 0 (rows r >= 1)
template <typename TA>
__device__ __forceinline__ void b_sb_pstart(const Desc &D, int64_t j0, int wg) {
  typedef typename C2T<TA>::t CA;
  __shared__ double2 sh[(ENT / 64) * SBW];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0;
  const int tid = threadIdx.x, part = tid & 3, rl = tid >> 2;
  const CA *A = reinterpret_cast<const CA *>(D.A);
  double2 x[SBR / 64][8];
#pragma unroll
  for (int ch = 0; ch < SBR / 64; ++ch) {
    const int64_t r = int64_t(wg) * SBR + ch * 64 + rl;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      x[ch][u] = r < m ? to_d2(A[(p0 + r) * D.lda + j0 + 8 * part + u]) : double2{0, 0};
  }
  double2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = double2{0, 0};
#pragma unroll
  for (int ch = 0; ch < SBR / 64; ++ch) {
    const int64_t r = int64_t(wg) * SBR + ch * 64 + rl;
    const double2 x0 = sb_rowval(x[ch], 0);
    if (r < m) {
#pragma unroll
      for (int u = 0; u < 8; ++u) D.pb[r * SBW + 8 * part + u] = x[ch][u];
      if (r == 0)
#pragma unroll
        for (int u = 0; u < 8; ++u) D.ptop[8 * part + u] = x[ch][u];
      if (r >= 1)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = cadd(acc[u], cmulc(x0, x[ch][u]));
    }
  }
  sb_rowsum(acc, sh, D.grec + int64_t(wg) * SBW);
}

// Column c of the panel: reflector from the reduced Gram row, applied to this
// workgroup's rows (the reflector is stored below the diagonal of pb, beta on
// it), then the partial Gram row of column c + 1 and the partial column c of
// V^dag V.  Records of column c are read from grec[c & 1], those of c + 1
// written to grec[(c + 1) & 1].  Row c of the panel, which every workgroup
// needs, is read from ptop[c & 1], not from pb: the workgroup holding it
// rewrites it in pb during the same launch (a late workgroup would read the
// updated row); that workgroup writes row c + 1, as updated here, to
// ptop[(c + 1) & 1].  Thread t owns column j = t % SBW of the rows
// s + PS_ k (slot s = t / SBW, k = 0 .. SBR / PS_ - 1): row accesses are
// coalesced and every reduction over rows is local, then over the PS_ slots
// in LDS; the values of columns c and c + 1 that every thread of a row needs
// go through LDS too.
constexpr int PCT = 512;
constexpr int PS_ = PCT / SBW;   // row slots of a workgroup
constexpr int PK = SBR / PS_;    // rows per thread
static_assert(SBR % 64 == 0 && SBR % PS_ == 0, "panel rows: whole 64-row chunks and slots");
__device__ __forceinline__ void b_sb_pcol(const Desc &D, int64_t j0, int c, int nw, int wg) {
  __shared__ double2 red[PS_][SBW], red2[PS_][SBW];
  __shared__ double2 top[SBW], gs[SBW], vcol[SBR], vnext[SBR];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0;
  const int nref = (int)std::min<int64_t>(SBW, m);
  const int tid = threadIdx.x, j = tid % SBW, sl = tid / SBW;
  const int64_t rb = int64_t(wg) * SBR;
  // ---- loads, all issued before any is used: the records of column j,
  // the top entry of column j, this thread's rows of column j ----
  const double2 *rin = D.grec + int64_t(c & 1) * nw * SBW;
  constexpr int RU = 4;  // records per thread in registers (nw <= PS_ RU)
  double2 rr[RU];
#pragma unroll
  for (int u = 0; u < RU; ++u) rr[u] = rin[std::min(sl + PS_ * u, nw - 1) * SBW + j];
  const double2 tp = D.ptop[(c & 1) * SBW + j];
  double2 x[PK];
#pragma unroll
  for (int k = 0; k < PK; ++k) x[k] = D.pb[std::min<int64_t>(rb + sl + PS_ * k, m - 1) * SBW + j];
  double2 g = {0, 0};
#pragma unroll
  for (int u = 0; u < RU; ++u)
    if (sl + PS_ * u < nw) g = cadd(g, rr[u]);
  for (int w = sl + PS_ * RU; w < nw; w += PS_) g = cadd(g, rin[w * SBW + j]);
  red[sl][j] = g;
  if (sl == 0) top[j] = tp;
  if (j == c)
#pragma unroll
    for (int k = 0; k < PK; ++k) vcol[sl + PS_ * k] = x[k];  // P[r][c]
  __syncthreads();
  if (tid < SBW) {
    double2 s = red[0][tid];
#pragma unroll
    for (int q = 1; q < PS_; ++q) s = cadd(s, red[q][tid]);
    gs[tid] = s;
  }
  __syncthreads();
  double beta;
  double2 tau, sc;
  householder(top[c], gs[c].x, beta, tau, sc);
  const double2 wjj = cadd(top[j], cmulc(sc, gs[j]));  // v^dag P[:, j]
  if (wg == 0 && tid == 0) {
    D.sbsc[c] = tau;
    D.sbsc[SBW + c] = double2{beta, 0};
  }
  const double2 cw = cmul(cconj(tau), wjj);
  // ---- apply to this thread's rows; column c keeps v (beta on the diagonal) ----
  // v_c[r]: 0 above c and past m, 1 at c, sc P[r][c] below
  auto vc_of = [&](int k) {
    const int64_t r = rb + sl + PS_ * k;
    return csel(r > c && r < m, cmul(sc, vcol[sl + PS_ * k]), double2{r == c ? 1.0 : 0.0, 0});
  };
#pragma unroll
  for (int k = 0; k < PK; ++k) {
    const int64_t r = rb + sl + PS_ * k;
    const double2 v = vc_of(k);
    const double2 upd = csub(x[k], cmul(v, cw));
    x[k] = csel(j > c, upd, csel(j == c && r >= c, csel(r == c, double2{beta, 0}, v), x[k]));
  }
  if (j == c + 1)
#pragma unroll
    for (int k = 0; k < PK; ++k) vnext[sl + PS_ * k] = x[k];  // P'[r][c + 1]
  // ---- stores (columns c .. SBW - 1 change; rows past m are not written) ----
#pragma unroll
  for (int k = 0; k < PK; ++k) {
    const int64_t r = rb + sl + PS_ * k;
    double2 *dst = (r < m && j >= c) ? D.pb + r * SBW + j : D.sink + tid % SINK;
    *dst = x[k];
  }
#pragma unroll
  for (int k = 0; k < PK; ++k) {
    const int64_t r = rb + sl + PS_ * k;
    double2 *dst = (r == c + 1 && r < m) ? D.ptop + ((c + 1) & 1) * SBW + j : D.sink + tid % SINK;
    *dst = x[k];
  }
  __syncthreads();
  // ---- partial sums: Gram row of column c + 1, column c of V^dag V ----
  double2 ag = {0, 0}, as = {0, 0};
#pragma unroll
  for (int k = 0; k < PK; ++k) {
    const int64_t r = rb + sl + PS_ * k;
    // (a select, not a product with 0: vnext is not written after the last column)
    ag = csel(r < m && c + 1 < nref && r > c + 1, cadd(ag, cmulc(vnext[sl + PS_ * k], x[k])), ag);
    as = cadd(as, cmulc(x[k], vc_of(k)));  // conj(v_j[r]) v_c[r], used for j < c
  }
  red[sl][j] = ag;
  red2[sl][j] = as;
  __syncthreads();
  if (tid < 2 * SBW) {
    const int jj = tid % SBW;
    double2 s = tid < SBW ? red[0][jj] : red2[0][jj];
#pragma unroll
    for (int q = 1; q < PS_; ++q) s = cadd(s, tid < SBW ? red[q][jj] : red2[q][jj]);
    if (tid < SBW)
      D.grec[int64_t((c + 1) & 1) * nw * SBW + int64_t(wg) * SBW + jj] = s;
    else
      D.srec[(int64_t(wg) * SBW + c) * SBW + jj] = jj < c ? s : double2{0, 0};
  }
}

// T factor of the panel (forward, column by column: T[c][c] = tau_c,
// T[0:c, c] = -tau_c T[0:c, 0:c] (V^dag V)[0:c, c]) and the band columns of
// the panel: the diagonal block from A (final since the previous update), R
// from pb (beta_c on its diagonal), zero fill space.
template <typename TA>
__device__ __forceinline__ void b_sb_tmat(const Desc &D, int64_t j0, int nw) {
  typedef typename C2T<TA>::t CA;
  __shared__ double2 S[SBW][SBW + 1], T[SBW][SBW + 1], taus[SBW];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0;
  const int nref = (int)std::min<int64_t>(SBW, m);
  const int tid = threadIdx.x;
  // S[l][c] = sum over the records: one entry per thread (RNT = SBW^2),
  // sixteen loads in flight
  static_assert(RNT == SBW * SBW, "k_sb_tmat: one thread per entry of S");
  {
    const int e = tid, c = e / SBW, l = e % SBW;
    double2 s = {0, 0};
    if (l < c && c < nref) {
      for (int w0 = 0; w0 < nw; w0 += 16) {
        double2 v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          v[u] = D.srec[(int64_t(std::min(w0 + u, nw - 1)) * SBW + c) * SBW + l];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (w0 + u < nw) s = cadd(s, v[u]);
      }
    }
    S[l][c] = s;
    T[l][c] = (l == c && c < nref) ? D.sbsc[c] : double2{0, 0};
    if (tid < SBW) taus[tid] = D.sbsc[tid];
  }
  __syncthreads();
  // Row l of T needs only its own earlier entries and S: half-wave l holds
  // row l, lane k its entry T[l][k] in a register; column c is a sum over the
  // 32 lanes of the half-wave (xor shuffles), taken by lane c.  No barrier.
  {
    const int l = tid / SBW, k = tid % SBW;
    double2 tlk = T[l][k];  // tau on the diagonal, zero elsewhere
    for (int c = 1; c < nref; ++c) {
      double2 t = csel(k >= l && k < c, cmul(tlk, S[k][c]), double2{0, 0});
#pragma unroll
      for (int o = 1; o < SBW; o <<= 1) {
        t.x += __shfl_xor(t.x, o, 64);
        t.y += __shfl_xor(t.y, o, 64);
      }
      const double2 tc = taus[c];
      if (k == c && l < c) tlk = cmul(double2{-tc.x, -tc.y}, t);
    }
    D.sbt[tid] = tlk;
    // with refinement every panel's T is kept for the back-transformation
    if (D.rall) D.Tm[(j0 / SBW) * (SBW * SBW) + tid] = tlk;
  }
  const CA *A = reinterpret_cast<const CA *>(D.A);
  for (int e = tid; e < SBW * LDB; e += RNT) {
    const int c = e / LDB, d = e % LDB;
    const int64_t j = j0 + c, row = j + d;
    double2 val = {0, 0};
    if (d <= SBW && row < n) {
      if (row < p0) {
        val = to_d2(A[row * D.lda + j]);
      } else {
        const int64_t rp = row - p0;  // <= c
        if (rp < nref) val = rp == c ? D.sbsc[SBW + c] : D.pb[rp * SBW + c];
      }
    }
    D.band[j * LDB + d] = val;
  }
}

// band columns j0 .. n - 1 of the last diagonal block (no panel below it)
template <typename TA>
__device__ __forceinline__ void b_sb_bandtail(const Desc &D, int64_t j0) {
  typedef typename C2T<TA>::t CA;
  const CA *A = reinterpret_cast<const CA *>(D.A);
  const int64_t n = D.n;
  for (int64_t e = threadIdx.x; e < (n - j0) * LDB; e += ENT) {
    const int64_t j = j0 + e / LDB, d = e % LDB, row = j + d;
    D.band[j * LDB + d] = (d <= SBW && row < n) ? to_d2(A[row * D.lda + j]) : double2{0, 0};
  }
}

// V (column major, global rows) and U = V T in the storage type of A.  A
// workgroup takes 64 panel rows: pb rows are read whole and transposed
// through LDS; thread (row r, group g) forms U[r][8 g .. 8 g + 7] (T upper
// triangular), so every global access is coalesced.
template <typename TA>
__device__ __forceinline__ void b_sb_u(const Desc &D, int64_t j0, int wg) {
  typedef typename C2T<TA>::t CA;
  __shared__ double2 T[SBW][SBW + 1];
  __shared__ double2 Vs[64][SBW + 1];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0, rb = int64_t(wg) * 64;
  const int tid = threadIdx.x, rr = tid % 64, lg = tid / 64;
  constexpr int NE = 64 * SBW / ENT;
  double2 pv[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {  // entry e = (row e / SBW, column e % SBW)
    const int e = tid + ENT * i;
    const int64_t r = rb + e / SBW;
    pv[i] = D.pb[std::min<int64_t>(r, m - 1) * SBW + e % SBW];
  }
  for (int e = tid; e < SBW * SBW; e += ENT) T[e / SBW][e % SBW] = D.sbt[e];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = tid + ENT * i, q = e / SBW, l = e % SBW;
    const int64_t r = rb + q;
    Vs[q][l] = l < r ? pv[i] : (l == r ? double2{1, 0} : double2{0, 0});
  }
  __syncthreads();
  const int64_t r = rb + rr;
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = double2{0, 0};
#pragma unroll 4
  for (int l2 = 0; l2 < SBW; ++l2) {
    const double2 v = Vs[rr][l2];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], cmul(v, T[l2][8 * lg + q]));
  }
  if (r < m) {
    CA *U = reinterpret_cast<CA *>(D.u);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int l = 8 * lg + q;
      D.V[int64_t(l) * D.ldv + p0 + r] = Vs[rr][l];
      U[int64_t(l) * D.ldv + p0 + r] = CA{TA(acc[q].x), TA(acc[q].y)};
    }
    if (D.rall) {  // refinement: the panel's reflectors kept, packed by columns
      double2 *vp = D.vrow + g_sb_voff(n, j0 / SBW) * SBW + r;
#pragma unroll
      for (int q = 0; q < 8; ++q) vp[(8 * lg + q) * m] = Vs[rr][8 * lg + q];
    }
  }
}

// X = A22 U on MFMA, split over K: workgroup (row block rb, split sp) sums
// the columns sp Kc .. (sp + 1) Kc - 1 of A22 into xp[sp].  Complex product
// as a real GEMM: rows 2r / 2r + 1 of the A tile are (re, im) / (im, -re) of
// A's row r, the B tile holds (re, -im) of U, so C[2r][l] = Re X[r][l] and
// C[2r + 1][l] = Im X[r][l].  FP32 partial products are summed into FP64
// every 128 complex columns of K.  Slabs of 32 (FP32) or 16 (FP64) complex
// columns; the next slab is loaded into registers while the current one
// runs on the matrix cores.
template <typename TA>
__device__ __forceinline__ void b_sb_hemm(const Desc &D, int64_t j0, int wg) {
  typedef typename C2T<TA>::t CA;
  constexpr bool F32 = std::is_same<TA, float>::value;
  constexpr int BK = F32 ? 64 : 32, KC = BK / 2;  // real / complex K per slab
  constexpr int P = Pitch<TA, BK>::value, BM = 2 * SBHM, BN = SBW, MI = 4, NI = 1;
  constexpr int AL = SBHM * KC / ENT;  // complex A entries per thread and slab
  constexpr int BL = BN * KC / ENT;    // complex U entries per thread and slab
  constexpr int FLUSH = F32 ? 128 / KC : 1 << 30;  // slabs between FP64 sums (128 terms)
  constexpr int PT = BM + 16 / int(sizeof(TA));  // pitch of a K-major A slab
  constexpr int AS = BM * P > BK * PT ? BM * P : BK * PT;
  __shared__ __attribute__((aligned(16))) TA As[AS];
  __shared__ __attribute__((aligned(16))) TA Bs[BN * P];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0;
  const int rb = wg / SBNS, sp = wg % SBNS;
  const int64_t kc = g_sb_kc(m), k0 = int64_t(sp) * kc, k1 = std::min<int64_t>(m, k0 + kc);
  const int64_t r0 = int64_t(rb) * SBHM;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm0 = (wv >> 1) * (BM / 2), wn0 = (wv & 1) * (BN / 2);
  const CA *A = reinterpret_cast<const CA *>(D.A);
  const CA *U = reinterpret_cast<const CA *>(D.u);
  // thread -> A row ar, columns ak .. ak + AL - 1; U column bl, rows bk ..
  const int ar = tid / (KC / AL), ak = (tid % (KC / AL)) * AL;
  const int bl = tid / (KC / BL), bk = (tid % (KC / BL)) * BL;
  const bool arow_ok = r0 + ar < m;
  const CA *ap = A + (p0 + std::min<int64_t>(r0 + ar, m - 1)) * D.lda + p0;
  const CA *up = U + int64_t(bl) * D.ldv + p0;
  typename Mfma<TA>::acc_t acc[MI][NI];
  acc_zero<TA, MI, NI>(acc);
  double accd[MI][4];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int j = 0; j < 4; ++j) accd[mi][j] = 0;
  CA ra[AL], rbv[BL];
  // Only entries on or below the diagonal are read (the trailing update keeps
  // just the lower triangle up to date); an entry above it is the conjugate
  // of its mirror.  A slab wholly left of this row block's diagonal reads
  // rows (thread: row ar, columns ak ..); one wholly right of it reads the
  // mirror's rows (thread: column kt, rows rt .. rt + AL - 1) and is staged
  // K-major, as it comes; a slab across the diagonal reads entry by entry.
  // Whole slabs (a uniform condition) load 16-byte vectors unconditionally
  // (aligned: p0, the slab start and the thread offsets are multiples of 8
  // complex entries, lda of 16); only the last, partial slab of a split
  // loads entry by entry.  Rows past m were clamped to row m - 1 and are
  // zeroed when staged.
  typedef typename std::conditional<F32, float4, double2>::type V16;
  constexpr int PER = 16 / int(sizeof(CA));  // complex entries per 16-byte load
  const int kt = tid / (SBHM / AL), rt = (tid % (SBHM / AL)) * AL;
  static_assert(KC * (SBHM / AL) == ENT, "one mirror piece per thread");
  const CA *atp = A + p0 * D.lda + p0 + r0 + rt;  // + k lda: A[p0 + k][p0 + r0 + rt ..]
  auto side = [&](int64_t kk) { return kk + KC - 1 <= r0 ? 0 : (kk >= r0 + SBHM ? 1 : 2); };
  auto load = [&](int64_t kk) {
    const int sd = side(kk);
    if (sd == 0 && kk + KC <= k1) {
      const V16 *a16 = reinterpret_cast<const V16 *>(ap + kk + ak);
#pragma unroll
      for (int i = 0; i < AL / PER; ++i) {
        const V16 v = a16[i];
        memcpy(&ra[PER * i], &v, 16);
      }
    } else if (sd == 1 && kk + KC <= k1 && r0 + rt + AL <= m) {
      const V16 *a16 = reinterpret_cast<const V16 *>(atp + (kk + kt) * D.lda);
#pragma unroll
      for (int i = 0; i < AL / PER; ++i) {
        const V16 v = a16[i];
        memcpy(&ra[PER * i], &v, 16);
      }
#pragma unroll
      for (int i = 0; i < AL; ++i) ra[i].y = -ra[i].y;
    } else if (sd == 1) {
      const int64_t k = kk + kt;
#pragma unroll
      for (int i = 0; i < AL; ++i) {
        const CA v = (k < k1 && r0 + rt + i < m) ? atp[k * D.lda + i] : CA{0, 0};
        ra[i] = CA{v.x, -v.y};
      }
    } else {
      const int64_t r = r0 + ar;
#pragma unroll
      for (int i = 0; i < AL; ++i) {
        const int64_t k = kk + ak + i;
        CA v = {0, 0};
        if (k < k1 && r < m) {
          if (k <= r) {
            v = A[(p0 + r) * D.lda + p0 + k];
          } else {
            v = A[(p0 + k) * D.lda + p0 + r];
            v.y = -v.y;
          }
        }
        ra[i] = v;
      }
    }
    if (kk + KC <= k1) {
      const V16 *u16 = reinterpret_cast<const V16 *>(up + kk + bk);
#pragma unroll
      for (int i = 0; i < BL / PER; ++i) {
        const V16 v = u16[i];
        memcpy(&rbv[PER * i], &v, 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < BL; ++i) {
        const int64_t kx = kk + bk + i;
        rbv[i] = kx < k1 ? up[kx] : CA{0, 0};
      }
    }
  };
  if (k0 < k1) load(k0);
  int slab = 0;
  for (int64_t kk = k0; kk < k1; kk += KC, ++slab) {
    if (side(kk) == 1) {
#pragma unroll
      for (int i = 0; i < AL; ++i) {
        // real K rows 2 kt (re, im) and 2 kt + 1 (im, -re) of A rows rt + i
        const int rr = rt + i;
        const TA ax = ra[i].x, ay = ra[i].y;  // rows past m were loaded as 0
        *reinterpret_cast<CA *>(As + (2 * kt) * PT + 2 * rr) = CA{ax, ay};
        *reinterpret_cast<CA *>(As + (2 * kt + 1) * PT + 2 * rr) = CA{ay, -ax};
      }
    } else {
#pragma unroll
      for (int i = 0; i < AL; ++i) {
        const int kq = ak + i;
        const TA ax = arow_ok ? ra[i].x : TA(0), ay = arow_ok ? ra[i].y : TA(0);
        As[(2 * ar) * P + 2 * kq] = ax;
        As[(2 * ar) * P + 2 * kq + 1] = ay;
        As[(2 * ar + 1) * P + 2 * kq] = ay;
        As[(2 * ar + 1) * P + 2 * kq + 1] = -ax;
      }
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int kq = bk + i;
      Bs[bl * P + 2 * kq] = rbv[i].x;
      Bs[bl * P + 2 * kq + 1] = -rbv[i].y;
    }
    __syncthreads();
    if (kk + KC < k1) load(kk + KC);
    if (side(kk) == 1)
      mfma_slab_at<TA, MI, NI, BK, PT>(acc, As, Bs, wm0, wn0, lane);
    else
      mfma_slab<TA, MI, NI, BK>(acc, As, Bs, wm0, wn0, lane);
    __syncthreads();
    if (F32 && (slab + 1) % FLUSH == 0) {
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          accd[mi][j] += double(acc[mi][0][j]);
          acc[mi][0][j] = TA(0);
        }
    }
  }
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int j = 0; j < 4; ++j) accd[mi][j] += double(acc[mi][0][j]);
  const int r16 = lane & 15, g = lane >> 4;
  double2 *xo = D.xp + int64_t(sp) * SBW * D.ldv;
  const int l = wn0 + r16;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
    const int64_t a = r0 + (wm0 + 16 * mi + 4 * g) / 2;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (a + h < m) xo[int64_t(l) * D.ldv + p0 + a + h] = double2{accd[mi][2 * h], accd[mi][2 * h + 1]};
  }
}

// X = sum of the splits (kept in W), partial V^dag X of this workgroup's 64
// rows (one record per workgroup)
__device__ __forceinline__ void b_sb_xred(const Desc &D, int64_t j0, int wg) {
  __shared__ double2 Vs[64][SBW + 1], Xs[64][SBW + 1];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0;
  const int tid = threadIdx.x;
  const int yl = tid / 8, yq = 4 * (tid % 8);  // Y entries (yl, yq .. yq + 3)
  double2 y[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  {
    const int64_t rb = int64_t(wg) * 64;
    constexpr int NE = 64 * SBW / ENT;
    // every load first (rows clamped to m - 1), then the sums, then the
    // predicated stores of X
    double2 xs[NE][SBNS], vv[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + ENT * i, l = e / 64, rr = e % 64;
      const int64_t o = int64_t(l) * D.ldv + p0 + std::min<int64_t>(rb + rr, m - 1);
#pragma unroll
      for (int s = 0; s < SBNS; ++s) xs[i][s] = D.xp[int64_t(s) * SBW * D.ldv + o];
      vv[i] = D.V[o];
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + ENT * i, l = e / 64, rr = e % 64;
      const bool in = rb + rr < m;
      double2 x = xs[i][0];
#pragma unroll
      for (int s = 1; s < SBNS; ++s) x = cadd(x, xs[i][s]);
      x = csel(in, x, double2{0, 0});
      Xs[rr][l] = x;
      Vs[rr][l] = csel(in, vv[i], double2{0, 0});
      if (in) D.W[int64_t(l) * D.ldv + p0 + rb + rr] = x;
    }
    __syncthreads();
    for (int rr = 0; rr < 64; ++rr) {
      const double2 v = Vs[rr][yl];
#pragma unroll
      for (int q = 0; q < 4; ++q) y[q] = cadd(y[q], cmulc(v, Xs[rr][yq + q]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) D.yrec[(int64_t(wg) * SBW + yl) * SBW + yq + q] = y[q];
}

// Z = T^dag (sum of the partial V^dag X); one thread per entry (RNT = SBW^2)
__device__ __forceinline__ void b_sb_z(const Desc &D, int nw) {
  __shared__ double2 Ys[SBW][SBW + 1], Ts[SBW][SBW + 1];
  const int e = threadIdx.x;
  double2 y = {0, 0};
  for (int w0 = 0; w0 < nw; w0 += 16) {
    double2 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = D.yrec[int64_t(std::min(w0 + u, nw - 1)) * SBW * SBW + e];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (w0 + u < nw) y = cadd(y, v[u]);
  }
  Ys[e / SBW][e % SBW] = y;
  Ts[e / SBW][e % SBW] = D.sbt[e];
  __syncthreads();
  const int l = e / SBW, l2 = e % SBW;
  double2 z = {0, 0};
  for (int k = 0; k <= l; ++k) z = cadd(z, cmulc(Ts[k][l], Ys[k][l2]));  // T upper triangular
  D.sbz[e] = z;
}

// W = X - V Z / 2: a workgroup takes 64 panel rows, thread (row r, group g)
// the columns 8 g .. 8 g + 7 of row r
__device__ __forceinline__ void b_sb_w(const Desc &D, int64_t j0, int wg) {
  __shared__ double2 Zs[SBW][SBW + 1];
  __shared__ double2 Vs[64][SBW + 1];
  const int64_t n = D.n, p0 = j0 + SBW, m = n - p0, rb = int64_t(wg) * 64;
  const int tid = threadIdx.x, rr = tid % 64, lg = tid / 64;
  const int64_t r = rb + rr, rc = std::min<int64_t>(r, m - 1);
  double2 x[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) x[q] = D.W[int64_t(8 * lg + q) * D.ldv + p0 + rc];
#pragma unroll
  for (int q = 0; q < 8; ++q) Vs[rr][8 * lg + q] = D.V[int64_t(8 * lg + q) * D.ldv + p0 + rc];
  for (int e = tid; e < SBW * SBW; e += ENT) Zs[e / SBW][e % SBW] = D.sbz[e];
  __syncthreads();
#pragma unroll 4
  for (int l2 = 0; l2 < SBW; ++l2) {
    const double2 v = cscale(0.5, Vs[rr][l2]);
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = csub(x[q], cmul(v, Zs[l2][8 * lg + q]));
  }
  if (r < m)
#pragma unroll
    for (int q = 0; q < 8; ++q) D.W[int64_t(8 * lg + q) * D.ldv + p0 + r] = x[q];
}

// trailing update of the panel: A[p0:, p0:] -= V W^dag + W V^dag.  From HER_TRI_M
// trailing rows on only the tiles on or below the diagonal are updated (no
// mirror tiles): the later panels read A on or below its diagonal only.
template <typename TA>
__device__ __forceinline__ void b_sb_her2k(const Desc &D, int64_t p0, int wg) {
  constexpr int BN = HerTile<TA, 0>::BN;
  const int64_t t = cdiv(D.n - p0, BN);
  if (!her_tri(t, BN)) {
    b_her2k<TA, 0>(D.n, p0, SBW, D.V, D.W, D.ldv, (TA *)D.A, D.lda, wg % t, wg / t, false);
  } else {
    int64_t by = int64_t((sqrt(8.0 * double(wg) + 1.0) - 1.0) * 0.5);
    while (by * (by + 1) / 2 > wg) --by;
    while ((by + 1) * (by + 2) / 2 <= wg) ++by;
    const int64_t bx = wg - by * (by + 1) / 2;
    b_her2k<TA, 0>(D.n, p0, SBW, D.V, D.W, D.ldv, (TA *)D.A, D.lda, bx, by, false);
  }
}
template <typename TA>
inline int64_t sb_her2k_wgs(int64_t n, int64_t p0) {
  constexpr int BN = HerTile<TA, 0>::BN;
  const int64_t m = n - p0, t = cdiv(m, BN);
  return m > 0 ? (her_tri(t, BN) ? t * (t + 1) / 2 : t * t) : 0;
}

template <typename TA>
__global__ __launch_bounds__(ENT) void k_sb_pstart(Desc D, int64_t j0) {
  b_sb_pstart<TA>(D, j0, int(blockIdx.x));
}
__global__ __launch_bounds__(PCT) void k_sb_pcol(Desc D, int64_t j0, int c, int nw) {
  b_sb_pcol(D, j0, c, nw, int(blockIdx.x));
}
template <typename TA>
__global__ __launch_bounds__(RNT) void k_sb_tmat(Desc D, int64_t j0, int nw) {
  b_sb_tmat<TA>(D, j0, nw);
}
template <typename TA>
__global__ __launch_bounds__(ENT) void k_sb_bandtail(Desc D, int64_t j0) {
  b_sb_bandtail<TA>(D, j0);
}
template <typename TA>
__global__ __launch_bounds__(ENT) void k_sb_u(Desc D, int64_t j0) {
  b_sb_u<TA>(D, j0, int(blockIdx.x));
}
template <typename TA>
__global__ __launch_bounds__(ENT) void k_sb_hemm(Desc D, int64_t j0) {
  b_sb_hemm<TA>(D, j0, int(blockIdx.x));
}
__global__ __launch_bounds__(ENT) void k_sb_xred(Desc D, int64_t j0) {
  b_sb_xred(D, j0, int(blockIdx.x));
}
__global__ __launch_bounds__(RNT) void k_sb_z(Desc D, int nw) { b_sb_z(D, nw); }
__global__ __launch_bounds__(ENT) void k_sb_w(Desc D, int64_t j0) {
  b_sb_w(D, j0, int(blockIdx.x));
}
template <typename TA>
__global__ __launch_bounds__(ENT) void k_sb_her2k(Desc D, int64_t p0) {
  b_sb_her2k<TA>(D, p0, int(blockIdx.x));
}

// ---------------------------------------------------------------------------
// stage 2: bulge chasing, one task per workgroup
// ---------------------------------------------------------------------------
// Task (i, k) covers rows R_k = i + 1 + k SBW .. + L - 1:
//   k > 0: the block O = A[R_k, R_{k-1}] takes the previous reflector of the
//          sweep from the right; a new reflector annihilates its first column
//          below row 0 and is applied to O from the left;
//   k = 0: the new reflector annihilates column i below row i + 1 (e_i =
//          beta);
//   both: the two-sided update of the diagonal block D = A[R_k, R_k].
// Thread t holds entries (p, q) = (t % 32, g + BCG u), g = t / 32, u < BCU,
// of each block: a wave holds g = 2 w, 2 w + 1, so sums over q combine the
// two halves of a wave and then the waves in LDS; sums over p are taken
// from an LDS copy.  Loads are coalesced along p (the band is stored by
// columns); D's upper triangle comes from its lower one through LDS.
constexpr int BCT = 512;
constexpr int BCU = SBW * SBW / BCT;  // entries per thread and block
constexpr int BCG = BCT / SBW;        // row groups g (q = g + BCG u)
constexpr int BCR = SBW / BCG;        // rows p per group in the sums over p
// KEEP (refinement): every reflector is also stored for the back-transformation
template <bool KEEP>
__global__ __launch_bounds__(BCT) void k_sb_chase(Desc D, int64_t t, int64_t ihi) {
  __shared__ double2 Ms[SBW][SBW + 1];      // D in full, then O
  __shared__ double2 part[BCT / 64][SBW];   // per-wave sums over q
  __shared__ double2 c0s[SBW];              // column 0 of O after the right update
  __shared__ double2 zp[BCG][SBW];    // partial sums over p of conj(u) O
  __shared__ double xsum;
  const int64_t n = D.n, i = ihi - int64_t(blockIdx.x), k = t - 2 * i;
  const int64_t rk = i + 1 + k * SBW, rp = k > 0 ? rk - SBW : i;
  const int L = (int)std::min<int64_t>(SBW, n - rk);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, p = tid % SBW, g = tid / SBW;
  double2 *band = D.band;
  // ---- loads, all issued together from in-bounds addresses ----
  double2 o[BCU], uq[BCU], dl[BCU];
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    const int64_t ao = k > 0 ? (rp + q) * LDB + SBW + p - q : i * LDB + 1 + p;
    o[u] = band[ao];
    uq[u] = D.rfl[i * SBW + q];
    // lower triangle of D (q <= p), column by column
    dl[u] = band[std::min<int64_t>(rk + q, n - 1) * LDB + (p >= q ? p - q : 0)];
  }
  const double2 tprev = D.rtau[i];
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    o[u] = csel(p < L && (k > 0 || q == 0), o[u], double2{0, 0});
    const bool in = p < L && q <= p;
    dl[u] = csel(in, dl[u], double2{0, 0});
    if (q == p) dl[u].y = 0;
    if (q <= p) {  // the entry and its mirror; upper positions are the mirrors' owners'
      Ms[p][q] = dl[u];
      Ms[q][p] = cconj(dl[u]);
    }
  }
  // ---- k > 0: O <- O (I - tau u u^dag) ----
  if (k > 0) {
    double2 y = {0, 0};
#pragma unroll
    for (int u = 0; u < BCU; ++u) y = cadd(y, cmul(o[u], uq[u]));
    y.x += __shfl_xor(y.x, 32, 64);
    y.y += __shfl_xor(y.y, 32, 64);
    if (lane < SBW) part[wv][p] = y;
  }
  __syncthreads();  // Ms (D in full) and the partial sums of O u
  double2 dm[BCU];
#pragma unroll
  for (int u = 0; u < BCU; ++u) dm[u] = Ms[p][g + BCG * u];
  if (k > 0) {
    double2 y = part[0][p];
#pragma unroll
    for (int w = 1; w < BCT / 64; ++w) y = cadd(y, part[w][p]);
    const double2 ty = cmul(tprev, y);
#pragma unroll
    for (int u = 0; u < BCU; ++u) o[u] = csub(o[u], cmul(ty, cconj(uq[u])));
  }
  // ---- new reflector from column 0 (held by the threads with g = 0, u = 0) ----
  if (g == 0) c0s[p] = o[0];
  if (wv == 0) {
    // all 64 lanes take part in the sum (lanes 32 .. 63, g = 1, hold no
    // column-0 entries and add 0)
    double xs = (g == 0 && p >= 1 && p < L) ? o[0].x * o[0].x + o[0].y * o[0].y : 0.0;
    xs = wave_sum(xs);
    if (tid == 0) xsum = xs;
  }
  __syncthreads();  // c0s, xsum; the reads of Ms and part are done
  double beta;
  double2 tau, sc;
  householder(c0s[0], xsum, beta, tau, sc);
  // u = (1, sc O[1:L, 0]), read for this thread's row p and columns q
  const double2 up = csel(p == 0, double2{1, 0}, csel(p < L, cmul(sc, c0s[p]), double2{0, 0}));
  double2 uc[BCU];
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    uc[u] = csel(q == 0, double2{1, 0}, csel(q < L, cmul(sc, c0s[q]), double2{0, 0}));
  }
  if (k > 0) {
    // z[q] = sum_p conj(u[p]) O[p][q]; O -= conj(tau) u z^T (q >= 1)
#pragma unroll
    for (int u = 0; u < BCU; ++u) Ms[p][g + BCG * u] = o[u];
    __syncthreads();
    double2 z = {0, 0};  // column p of O over the rows BCR g .. BCR g + BCR - 1
#pragma unroll
    for (int a = 0; a < BCR; ++a) {
      const int pr = BCR * g + a;
      const double2 upr = csel(pr == 0, double2{1, 0}, csel(pr < L, cmul(sc, c0s[pr]), double2{0, 0}));
      z = cadd(z, cmulc(upr, Ms[pr][p]));
    }
    zp[g][p] = z;
    __syncthreads();
    const double2 cu = cmul(cconj(tau), up);
#pragma unroll
    for (int u = 0; u < BCU; ++u) {
      const int q = g + BCG * u;
      double2 zq = zp[0][q];
#pragma unroll
      for (int gg = 1; gg < BCG; ++gg) zq = cadd(zq, zp[gg][q]);
      o[u] = csel(q == 0, csel(p == 0, double2{beta, 0}, double2{0, 0}), csub(o[u], cmul(cu, zq)));
    }
  } else {
    o[0] = csel(p == 0, double2{beta, 0}, double2{0, 0});
    if (tid == 0) D.e[i] = beta;
  }
  // ---- D <- H^dag D H: y = D u, w = tau y - |tau|^2 (u^dag y) u / 2,
  //      D -= u w^dag + w u^dag ----
  double2 y = {0, 0};
#pragma unroll
  for (int u = 0; u < BCU; ++u) y = cadd(y, cmul(dm[u], uc[u]));
  y.x += __shfl_xor(y.x, 32, 64);
  y.y += __shfl_xor(y.y, 32, 64);
  if (lane < SBW) part[wv][p] = y;
  __syncthreads();
  double2 yp = part[0][p];
#pragma unroll
  for (int w = 1; w < BCT / 64; ++w) yp = cadd(yp, part[w][p]);
  // gamma = sum_p conj(u[p]) y[p] over the 32 lanes of a half wave (every
  // half wave holds all p)
  double gam = cmulc(up, yp).x;
#pragma unroll
  for (int o_ = 16; o_ > 0; o_ >>= 1) gam += __shfl_xor(gam, o_, 64);
  const double t2 = tau.x * tau.x + tau.y * tau.y;
  const double2 wp = csub(cmul(tau, yp), cscale(0.5 * t2 * gam, up));
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    double2 yq = part[0][q];
#pragma unroll
    for (int w = 1; w < BCT / 64; ++w) yq = cadd(yq, part[w][q]);
    const double2 wq = csub(cmul(tau, yq), cscale(0.5 * t2 * gam, uc[u]));
    dm[u] = csub(dm[u], cadd(cmul(up, cconj(wq)), cmul(wp, cconj(uc[u]))));
    if (q == p) dm[u].y = 0;
  }
  // ---- stores, all at the end and unconditional: entries without a place
  // go to the sink.  O (k > 0) rows past the block end lie past row n - 1
  // of their columns (padding that nothing reads); column i (k = 0) is
  // written by the threads with q = 0. ----
  double2 *sk = D.sink + tid % SINK;
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    double2 *dst = k > 0 ? band + (rp + q) * LDB + SBW + p - q : (q == 0 ? band + i * LDB + 1 + p : sk);
    *dst = o[u];
  }
#pragma unroll
  for (int u = 0; u < BCU; ++u) {
    const int q = g + BCG * u;
    double2 *dst = (q <= p && p < L) ? band + (rk + q) * LDB + p - q : sk;
    *dst = dm[u];
  }
  // ---- the reflector of the next step of this sweep ----
  if (g == 0) D.rfl[i * SBW + p] = up;
  if (tid == 0) D.rtau[i] = tau;
  if (KEEP && g == 0 && p < L)  // kept for the back-transformation; tau in place of u_0 = 1
    D.rall[g_bc_off(n, i) + k * SBW + p] = csel(p == 0, tau, up);
}

// d from the band's diagonal
__global__ __launch_bounds__(ENT) void k_sb_diag(Desc D) {
  const int64_t r = int64_t(blockIdx.x) * ENT + threadIdx.x;
  if (r < D.n) D.d[r] = D.band[r * LDB].x;
}

// ---------------------------------------------------------------------------
// back-transformation through the bulge chase (refinement): x = Q2 z for
// each eigenvector z of T, Q2 the product of the chase's reflectors
// H = I - tau u u^dag in the order they were made (each task turned D into
// H^dag D H).  The reflectors of one sweep act on disjoint row blocks, and a
// reflector of sweep i was made after every reflector of an earlier sweep
// that shares a row with it, so applying whole sweeps from the last to the
// first is the reverse order.  One workgroup per vector.  The stored entry of
// row 0 of a task holds its tau (u_0 = 1).  Within a sweep a row is read and
// written by one lane only; a barrier separates the sweeps.
//   k_bx_chase_lds  blocks of up to BXL - SBW rows: x in LDS (FP64); BXW lanes per
//                   task, BXQ consecutive rows per lane, u^dag x summed over
//                   the lane's rows and then over the task's lanes (DPP
//                   moves); the reflectors of the next sweep are loaded
//                   while the current one is applied (they do not depend on x)
//   k_bx_chase      larger blocks: x in global memory, SBW lanes per task
//                   (one row each), BXU tasks per group with their loads in
//                   flight together
// ---------------------------------------------------------------------------

// cross-lane moves within groups of eight lanes (DPP, no LDS round trip):
// quad_perm [1,0,3,2] (lane ^ 1), [2,3,0,1] (lane ^ 2), [0,0,0,0] (lane 0 of
// the quad) and row_half_mirror (lane i <-> 7 - i of each eight)
constexpr int DPP_X1 = 0xB1, DPP_X2 = 0x4E, DPP_Q0 = 0x00, DPP_HM = 0x141;
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
// sum over the eight lanes of a group, on every lane: the quad sums by two
// exchanges, then the mirrored quad's sum
__device__ __forceinline__ double sum8(double v) {
  v += dppd<DPP_X1>(v);
  v += dppd<DPP_X2>(v);
  return v + dppd<DPP_HM>(v);
}
// the value of lane 0 of the group of eight, on every lane (pl: lane in the group)
__device__ __forceinline__ double bcast8(double v, int pl) {
  const double q = dppd<DPP_Q0>(v);
  const double m = dppd<DPP_HM>(q);
  return pl < 4 ? q : m;
}
static_assert(BXW == 8, "k_bx_chase_lds: tasks of eight lanes");

__global__ __launch_bounds__(BXT) void k_bx_chase_lds(Desc D) {
  __shared__ double2 xs[BXL];
  const int n = (int)D.n;  // <= BXL: every index below fits in 32 bits
  const int64_t l = blockIdx.x;
  const int tid = threadIdx.x, pl = tid % BXW, grp = tid / BXW;
  const double *z = D.Z + l * n;
  double2 *x = D.X + l * n;
  // rows n .. n + SBW - 1 (n <= BXL - SBW) are zero padding: the lanes of the
  // last task of a sweep past row n - 1 read and write there with u = 0
  for (int r = tid; r < n + SBW; r += BXT) xs[r] = double2{r < n ? z[r] : 0.0, 0.0};
  // stored entries of a sweep, this lane's rows: two sets, the one of the
  // sweep being applied and the one being loaded for the next sweep
  double2 wa[BXRL][BXQ], wb[BXRL][BXQ];
#define BX_FETCH(W, I)                                                           \
  {                                                                              \
    const int i_ = (I), nt_ = (int)g_bc_kmax(n, i_) + 1;                          \
    const double2 *r_ = D.rall + (int)g_bc_off(n, i_);                                \
    _Pragma("unroll") for (int j = 0; j < BXRL; ++j) {                           \
      const int k = grp + BXGL * j, r = i_ + 1 + k * SBW + BXQ * pl;         \
      _Pragma("unroll") for (int q = 0; q < BXQ; ++q)                            \
        W[j][q] = r_[k < nt_ && r + q < n ? r + q - i_ - 1 : 0];                 \
    }                                                                            \
  }
  // sweep I with the entries in WC, the next sweep's loaded into WN; the
  // barrier covers the LDS writes only, so those loads stay in flight across it
#define BX_SWEEP(I, WC, WN)                                                      \
  {                                                                              \
    const int sw_ = (I), nt = (int)g_bc_kmax(n, sw_) + 1;                             \
    BX_FETCH(WN, sw_ > 0 ? sw_ - 1 : 0)                                              \
    __asm__ volatile("" ::: "memory"); /* the loads are issued here */           \
    _Pragma("unroll") for (int j = 0; j < BXRL; ++j) {                           \
      const int k = grp + BXGL * j;                                          \
      if (k < nt) { /* the same for the lanes of a task */                       \
        const int r0 = sw_ + 1 + k * SBW + BXQ * pl;                           \
        const double2 tau = {bcast8(WC[j][0].x, pl), bcast8(WC[j][0].y, pl)};   \
        double2 u[BXQ], xv[BXQ], y = {0, 0};                                     \
        _Pragma("unroll") for (int q = 0; q < BXQ; ++q) {                        \
          const bool in = r0 + q < n;                                            \
          u[q] = csel(in, csel(pl == 0 && q == 0, double2{1, 0}, WC[j][q]), double2{0, 0}); \
          xv[q] = xs[r0 + q];                                                    \
          y = cadd(y, cmulc(u[q], xv[q]));                                       \
        }                                                                        \
        y.x = sum8(y.x);                                                         \
        y.y = sum8(y.y);                                                         \
        const double2 f = cmul(tau, y);                                          \
        _Pragma("unroll") for (int q = 0; q < BXQ; ++q)                          \
          xs[r0 + q] = csub(xv[q], cmul(f, u[q]));                               \
      }                                                                          \
    }                                                                            \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");              \
    __builtin_amdgcn_s_barrier();                                                \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");              \
  }
  BX_FETCH(wa, n - 2)
  __syncthreads();  // xs complete
  for (int i = n - 2; i >= 0; i -= 2) {
    BX_SWEEP(i, wa, wb)
    if (i >= 1) BX_SWEEP(i - 1, wb, wa)
  }
#undef BX_SWEEP
#undef BX_FETCH
  for (int r = tid; r < n; r += BXT) x[r] = xs[r];
}

// one reflector on the SBW lanes of a group (lane p: row rk + p), for
// k_bx_chase: x -= tau u (u^dag x); w is the stored entry (tau on lane 0),
// in says whether the lane has a row
__device__ __forceinline__ double2 bx_apply(double2 w, double2 xv, bool in, int p) {
  const int base = (threadIdx.x & 63) & ~(SBW - 1);
  const double2 tau = {__shfl(w.x, base, 64), __shfl(w.y, base, 64)};
  const double2 u = csel(in, csel(p == 0, double2{1, 0}, w), double2{0, 0});
  double2 y = cmulc(u, xv);
#pragma unroll
  for (int o = 1; o < SBW; o <<= 1) {
    y.x += __shfl_xor(y.x, o, 64);
    y.y += __shfl_xor(y.y, o, 64);
  }
  return csub(xv, cmul(cmul(tau, y), u));
}

__global__ __launch_bounds__(BXC) void k_bx_chase(Desc D) {
  const int64_t n = D.n, l = blockIdx.x;
  const int tid = threadIdx.x, p = tid % SBW, grp = tid / SBW;
  const double *z = D.Z + l * n;
  double2 *x = D.X + l * n;
  for (int64_t r = tid; r < n; r += BXC) x[r] = double2{z[r], 0.0};
  __syncthreads();
  for (int64_t i = n - 2; i >= 0; --i) {
    const int64_t nt = g_bc_kmax(n, i) + 1;  // tasks of sweep i
    const double2 *ri = D.rall + g_bc_off(n, i);
    for (int64_t k0 = 0; k0 < nt; k0 += BXG * BXU) {
      double2 w[BXU], xv[BXU];
      int64_t row[BXU];
      bool in[BXU];
#pragma unroll
      for (int j = 0; j < BXU; ++j) {  // every load from an in-bounds address
        const int64_t k = k0 + grp + BXG * j, r = i + 1 + k * SBW + p;
        in[j] = k < nt && r < n;
        row[j] = in[j] ? r : i + 1;
        w[j] = ri[k < nt ? row[j] - i - 1 : 0];
        xv[j] = x[row[j]];
      }
#pragma unroll
      for (int j = 0; j < BXU; ++j) xv[j] = bx_apply(w[j], xv[j], in[j], p);
#pragma unroll
      for (int j = 0; j < BXU; ++j)
        if (in[j]) x[row[j]] = xv[j];
    }
    __syncthreads();
  }
}
