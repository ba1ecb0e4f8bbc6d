// Host-only check of the block eigensolver's workspace layout and launch
// geometry (no GPU).  Built with g++ and AddressSanitizer from the same
// geometry header as the kernels (eigh_geometry.h); it lays out one block's
// workspace in host memory, replays the single-block launch sequence (the
// order of launches and the form of k_colA per column, as the library issues
// them) and, for every launch, visits the index ranges each kernel writes and
// reads, as given by its indexing:
//   k_col0      col[j0..n), record wg of the alternating partial-sum buffer
//   k_colA      parta[wg], bred[16 wg + 0..15] (wg < 4), tau/scl[m0], d/e[jn];
//               row forms: y[r], V[ir][r] for its rows; tile forms: the tile
//               (bi, bj) of workgroup wg, ys[bj][rows] and ys[bi][columns],
//               V[ir][rows] on the diagonal
//   k_colB      ys[0..nbt)[rows] (tile forms), parta[0..npa), records of its
//               workgroup in the other buffer, W[ir][rows], col[rows]
//   k_her2k     the A entries of every tile, V and W columns 0..nbk
//   k_tail, the tridiagonal and refinement kernels: their buffers whole;
//   two-stage reduction: the panel rows, records, band columns and X splits
//   of every stage-1 launch, and the band, reflector and tridiagonal entries
//   of every bulge-chasing task.
// Every index is asserted to lie inside its region of the layout, and the
// byte is touched, so an index past the region or past the workspace stops
// the check (assertion or AddressSanitizer report).  Regions must not overlap.
//
//   g++ -std=c++17 -O1 -fsanitize=address,undefined -I paper_2603_24860_amd/csrc \
//       tests/eigh_layout_check.cpp -o eigh_layout_check
//   ./eigh_layout_check n a_fp64 K [n a_fp64 K ...]     (K = -1 - k: two-stage reduction, k refined)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "eigh_geometry.h"

using namespace bse;

namespace {

struct Region {
  const char *name;
  char *p;
  size_t elem;
  int64_t count;
};

struct Check {
  std::vector<Region> regs;
  int64_t touches = 0;
  char *base = nullptr;
  size_t bytes = 0;

  void add(const char *name, const void *p, size_t elem, int64_t count) {
    regs.push_back(Region{name, (char *)p, elem, count});
  }
  const Region &reg(const char *name) const {
    for (const Region &r : regs)
      if (!std::strcmp(r.name, name)) return r;
    std::fprintf(stderr, "no region %s\n", name);
    std::abort();
  }
  void at(const char *name, int64_t i, const char *who) {
    const Region &r = reg(name);
    if (i < 0 || i >= r.count) {
      std::fprintf(stderr, "%s: index %lld outside %s[0..%lld)\n", who, (long long)i, name,
                   (long long)r.count);
      std::exit(1);
    }
    volatile char *b = r.p + size_t(i) * r.elem;
    b[0] = b[0];
    b[r.elem - 1] = b[r.elem - 1];
    ++touches;
  }
  void range(const char *name, int64_t lo, int64_t hi, const char *who) {  // [lo, hi)
    if (hi > lo) {
      at(name, lo, who);
      at(name, hi - 1, who);
    }
  }
  void layout_ok() const {
    for (size_t i = 0; i < regs.size(); ++i) {
      const Region &a = regs[i];
      if (a.count == 0) continue;
      const char *a1 = a.p + a.elem * size_t(a.count);
      if (a.p < base || a1 > base + bytes) {
        std::fprintf(stderr, "region %s outside the workspace\n", a.name);
        std::exit(1);
      }
      for (size_t j = i + 1; j < regs.size(); ++j) {
        const Region &b = regs[j];
        if (b.count == 0) continue;
        const char *b1 = b.p + b.elem * size_t(b.count);
        if (a.p < b1 && b.p < a1) {
          std::fprintf(stderr, "regions %s and %s overlap\n", a.name, b.name);
          std::exit(1);
        }
      }
    }
  }
};

// tile (bi, bj), bi >= bj, of workgroup wg in row-major lower-triangle order
void tri_of(int64_t wg, int64_t &bi, int64_t &bj) {
  bi = int64_t((std::sqrt(8.0 * double(wg) + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= wg) ++bi;
  while (bi > 0 && bi * (bi + 1) / 2 > wg) --bi;
  bj = wg - bi * (bi + 1) / 2;
}

// the two-stage reduction (stage 1 panels, bulge chasing, band diagonal);
// the copy-in, the initial reflection and the tridiagonal step are the
// one-stage ones and are replayed by the caller
int run_two_stage(Check &C, const Desc &D, int64_t n, bool a64) {
  const size_t elu = a64 ? 16 : 8;
  const int64_t nwmax = g_sb_nw(n);
  C.add("pb", D.pb, 16, n * SBW);
  C.add("grec", D.grec, 16, 2 * nwmax * SBW);
  C.add("srec", D.srec, 16, nwmax * SBW * SBW);
  C.add("sbt", D.sbt, 16, SBW * SBW);
  C.add("sbz", D.sbz, 16, SBW * SBW);
  C.add("sbsc", D.sbsc, 16, 2 * SBW);
  C.add("ptop", D.ptop, 16, 2 * SBW);
  C.add("u", D.u, elu, SBW * D.ldv);
  C.add("xp", D.xp, 16, int64_t(SBNS) * SBW * D.ldv);
  C.add("yrec", D.yrec, 16, g_sb_nx(n) * SBW * SBW);
  C.add("band", D.band, 16, n * LDB);
  C.add("rfl", D.rfl, 16, n * SBW);
  C.add("rtau", D.rtau, 16, n);
  C.add("sink", D.sink, 16, SINK);
  const int64_t K = D.K;
  if (K > 0) {
    C.add("rall", D.rall, 16, std::max<int64_t>(g_bc_off(n, n - 1), 1));
    C.add("vrow", D.vrow, 16, std::max<int64_t>(g_sb_voff(n, g_sb_npan(n)), 1) * SBW);
    C.add("bxw", D.bxw, 16, cdiv(n, BPR) * K * SBW);
    if (D.Vall) return 1;  // the two-stage path keeps its reflectors by rows only
  }
  C.layout_ok();
  int64_t j0 = 0;
  for (; j0 + SBW < n; j0 += SBW) {
    const int64_t p0 = j0 + SBW, m = n - p0, nw = g_sb_nw(m);
    const int nref = (int)std::min<int64_t>(SBW, m);
    if (n - j0 < SBW + 1) return 1;  // a factored panel is always SBW wide
    // k_sb_pstart / k_sb_pcol: rows wg SBR .. + SBR (clamped to m - 1), all SBW columns
    for (int64_t wg = 0; wg < nw; ++wg) {
      const int64_t r0 = wg * SBR, r1 = std::min<int64_t>(r0 + SBR, m) - 1;
      if (r0 < m) {
        C.at("A", (p0 + r0) * D.lda + j0, "k_sb_pstart");
        C.at("A", (p0 + r1) * D.lda + j0 + SBW - 1, "k_sb_pstart");
        C.range("pb", r0 * SBW, r1 * SBW + SBW, "k_sb_pstart/pcol");
      } else {
        C.range("pb", (m - 1) * SBW, m * SBW, "k_sb_pcol clamped");
      }
      C.range("grec", wg * SBW, wg * SBW + SBW, "k_sb_pstart");
      if (wg == 0) C.range("ptop", 0, SBW, "k_sb_pstart top");
      for (int c = 0; c < nref; ++c) {
        C.range("grec", ((c + 1) & 1) * nw * SBW + wg * SBW, ((c + 1) & 1) * nw * SBW + wg * SBW + SBW,
                "k_sb_pcol out");
        C.range("srec", (wg * SBW + c) * SBW, (wg * SBW + c) * SBW + SBW, "k_sb_pcol srec");
      }
    }
    for (int c = 0; c < nref; ++c) {
      C.range("grec", (c & 1) * nw * SBW, (c & 1) * nw * SBW + nw * SBW, "k_sb_pcol in");
      C.range("ptop", (c & 1) * SBW, (c & 1) * SBW + SBW, "k_sb_pcol top");
      if (c + 1 < m) C.range("ptop", ((c + 1) & 1) * SBW, ((c + 1) & 1) * SBW + SBW, "k_sb_pcol next top");
      C.at("sbsc", c, "k_sb_pcol");
      C.at("sbsc", SBW + c, "k_sb_pcol");
    }
    // k_sb_tmat
    C.range("srec", 0, (nw - 1) * SBW * SBW + SBW * SBW, "k_sb_tmat");
    C.range("sbt", 0, SBW * SBW, "k_sb_tmat");
    if (K > 0) {
      C.range("Tm", (j0 / SBW) * SBW * SBW, (j0 / SBW + 1) * SBW * SBW, "k_sb_tmat T kept");
      // k_sb_u: panel rows 0 .. m, all SBW entries, row-major from g_sb_voff
      if (g_sb_voff(n, j0 / SBW + 1) - g_sb_voff(n, j0 / SBW) != m) return 1;
      C.range("vrow", g_sb_voff(n, j0 / SBW) * SBW, (g_sb_voff(n, j0 / SBW) + m) * SBW,
              "k_sb_u rows kept");
    }
    for (int c = 0; c < SBW; ++c)
      for (int d = 0; d < LDB; ++d) {
        const int64_t j = j0 + c, row = j + d;
        C.at("band", j * LDB + d, "k_sb_tmat band");
        if (d <= SBW && row < n) {
          if (row < p0) C.at("A", row * D.lda + j, "k_sb_tmat A");
          else if (row - p0 < nref) C.at("pb", (row - p0) * SBW + c, "k_sb_tmat R");
        }
      }
    // k_sb_u, k_sb_xred, k_sb_w: rows 0 .. m of V, W, U, the splits of X
    for (int l = 0; l < SBW; ++l) {
      C.range("V", int64_t(l) * D.ldv + p0, int64_t(l) * D.ldv + n, "k_sb_u V");
      C.range("W", int64_t(l) * D.ldv + p0, int64_t(l) * D.ldv + n, "k_sb_xred/w W");
      C.range("u", int64_t(l) * D.ldv + p0, int64_t(l) * D.ldv + n, "k_sb_u U");
      for (int sp = 0; sp < SBNS; ++sp)
        C.range("xp", (int64_t(sp) * SBW + l) * D.ldv + p0, (int64_t(sp) * SBW + l) * D.ldv + n,
                "k_sb_hemm/xred xp");
    }
    C.range("pb", 0, m * SBW, "k_sb_u pb");
    C.range("yrec", 0, g_sb_nx(m) * SBW * SBW, "k_sb_xred/z");
    C.range("sbz", 0, SBW * SBW, "k_sb_z/w");
    // k_sb_hemm: A rows p0 + min(r0 + ar, m - 1), columns p0 + [k0, k1)
    const int64_t kc = g_sb_kc(m);
    for (int64_t wg = 0; wg < g_sb_hemm_wgs(m); ++wg) {
      const int64_t rb = wg / SBNS, sp = wg % SBNS, r0 = rb * SBHM;
      const int64_t k0 = sp * kc, k1 = std::min<int64_t>(m, k0 + kc);
      const int64_t ra = std::min<int64_t>(r0, m - 1), rz = std::min<int64_t>(r0 + SBHM - 1, m - 1);
      if (k0 < k1) {
        C.at("A", (p0 + ra) * D.lda + p0 + k0, "k_sb_hemm A");
        C.at("A", (p0 + rz) * D.lda + p0 + k1 - 1, "k_sb_hemm A");
        C.range("u", p0 + k0, p0 + k1, "k_sb_hemm U");
        C.range("u", int64_t(SBW - 1) * D.ldv + p0 + k0, int64_t(SBW - 1) * D.ldv + p0 + k1,
                "k_sb_hemm U");
      }
      // entries above the diagonal come from their mirrors A[p0 + k][p0 + r], r < m
      if (k0 < k1 && k1 > r0 + 1 && r0 < m) {
        const int64_t kf = std::max<int64_t>(k0, r0 + 1);
        C.at("A", (p0 + kf) * D.lda + p0 + ra, "k_sb_hemm mirror");
        C.at("A", (p0 + k1 - 1) * D.lda + p0 + rz, "k_sb_hemm mirror");
      }
      for (int64_t a = r0; a < std::min<int64_t>(r0 + SBHM, m); a += SBHM - 1)
        for (int l = 0; l < SBW; l += SBW - 1)
          C.at("xp", (sp * SBW + l) * D.ldv + p0 + a, "k_sb_hemm out");
    }
    // k_her2k from p0, tile shape 0
    {
      const int BN = HerTile<float, 0>::BN, BM = HerTile<float, 0>::BM;
      const int64_t t = cdiv(n - p0, int64_t(BN));
      const int64_t gh = her_tri(t, BN) ? t * (t + 1) / 2 : t * t;
      for (int64_t wg = 0; wg < gh; ++wg) {
        int64_t bx, by;
        if (!her_tri(t, BN)) {
          bx = wg % t;
          by = wg / t;
        } else {
          tri_of(wg, by, bx);
        }
        const int64_t a0 = p0 + by * (BM / 2), b0 = p0 + bx * BN;
        if (a0 >= n || b0 >= n) continue;
        const int64_t a1 = std::min<int64_t>(a0 + BM / 2, n) - 1;
        const int64_t b1 = std::min<int64_t>(b0 + BN, n) - 1;
        C.at("A", a0 * D.lda + b0, "k_sb_her2k");
        C.at("A", a1 * D.lda + b1, "k_sb_her2k");
        C.at("A", b1 * D.lda + a1, "k_sb_her2k mirror");
      }
    }
  }
  // k_sb_bandtail: columns j0 .. n
  for (int64_t j = j0; j < n; ++j)
    for (int d = 0; d < LDB; ++d) {
      C.at("band", j * LDB + d, "k_sb_bandtail");
      if (d <= SBW && j + d < n) C.at("A", (j + d) * D.lda + j, "k_sb_bandtail A");
    }
  // k_sb_chase: every task of every launch
  int64_t tasks = 0;
  for (int64_t t = 0; t <= g_bc_tmax(n); ++t) {
    const int64_t lo = g_bc_ilo(n, t), hi = g_bc_ihi(n, t);
    for (int64_t i = lo; i <= hi; ++i) {
      const int64_t k = t - 2 * i, rk = i + 1 + k * SBW;
      if (k < 0 || k > g_bc_kmax(n, i) || rk >= n) {
        std::fprintf(stderr, "task (%lld, %lld) of launch %lld\n", (long long)i, (long long)k,
                     (long long)t);
        return 1;
      }
      const int L = (int)std::min<int64_t>(SBW, n - rk);
      if (k > 0) {
        const int64_t rp = rk - SBW;
        for (int q = 0; q < SBW; q += SBW - 1)
          for (int p = 0; p < L; p += std::max(1, L - 1)) {
            const int64_t d = SBW + p - q;
            if (d < 1 || d >= LDB) return 1;
            C.at("band", (rp + q) * LDB + d, "k_sb_chase O");
          }
        C.at("rtau", i, "k_sb_chase");
      } else {
        C.range("band", i * LDB + 1, i * LDB + 1 + L, "k_sb_chase column");
        C.at("e", i, "k_sb_chase");
      }
      // loads issued for every lane before masking: O over all 32 rows (or
      // column i to offset SBW), D clamped to the last column
      if (k > 0) {
        const int64_t rp = rk - SBW;
        C.at("band", rp * LDB + SBW + SBW - 1, "k_sb_chase O load");
        C.at("band", (rp + SBW - 1) * LDB + 1, "k_sb_chase O load");
      } else {
        C.at("band", i * LDB + SBW, "k_sb_chase column load");
      }
      C.at("band", std::min<int64_t>(rk + SBW - 1, n - 1) * LDB + SBW - 1, "k_sb_chase D load");
      C.range("rfl", i * SBW, i * SBW + SBW, "k_sb_chase");
      if (K > 0) {  // the reflector kept: rows rk .. rk + L of sweep i, packed
        if (rk - i - 1 != k * SBW) return 1;
        C.range("rall", g_bc_off(n, i) + k * SBW, g_bc_off(n, i) + k * SBW + L, "k_sb_chase keep");
        if (g_bc_off(n, i) + k * SBW + L > g_bc_off(n, i) + (n - 1 - i)) return 1;  // own sweep
      }
      C.at("band", rk * LDB, "k_sb_chase D");
      C.at("band", (rk + L - 1) * LDB, "k_sb_chase D");
      C.at("band", rk * LDB + L - 1, "k_sb_chase D");
      ++tasks;
    }
  }
  int64_t want = 0;
  for (int64_t i = 0; i + 1 < n; ++i) want += g_bc_kmax(n, i) + 1;
  if (tasks != want) {
    std::fprintf(stderr, "%lld chase tasks launched, %lld in the sweeps\n", (long long)tasks,
                 (long long)want);
    return 1;
  }
  C.range("band", 0, n * LDB, "k_sb_diag");
  C.range("sink", 0, SINK, "masked stores (thread index modulo SINK)");
  if (K > 0) {
    // k_bx_chase / k_bx_chase_lds: every task of every sweep (its rows, the
    // entry of its row 0 with tau), loads of masked lanes from the sweep's
    // first entry; the LDS form's x covers rows 0 .. n + SBW <= BXL
    for (int64_t i = n - 2; i >= 0; --i) {
      const int64_t nt = g_bc_kmax(n, i) + 1;
      if (n <= BXL - SBW) {  // the LDS form: its rounds cover the tasks, its rows fit with padding
        if (nt > int64_t(BXGL) * BXRL) return 1;
        if (i + 1 + (nt - 1) * SBW + SBW > BXL) return 1;
      }
      for (int64_t k = 0; k < nt; ++k) {
        const int64_t r0 = i + 1 + k * SBW, r1 = std::min<int64_t>(r0 + SBW, n);
        C.range("rall", g_bc_off(n, i) + (r0 - i - 1), g_bc_off(n, i) + (r1 - i - 1), "k_bx_chase u");
        if (g_bc_off(n, i) + (r1 - i - 1) > g_bc_off(n, i + 1)) return 1;  // inside its sweep
        C.range("X", r0, r1, "k_bx_chase x");
        C.range("X", (K - 1) * n + r0, (K - 1) * n + r1, "k_bx_chase x");
      }
      C.at("rall", g_bc_off(n, i), "k_bx_chase masked lanes");
    }
    C.range("Z", 0, K * n, "k_bx_chase z");
    // k_bp_part / k_bp_apply: panel p, grid (cdiv(m, BPR), cdiv(K, BPV)); rows
    // rb .. min(rb + BPR, m) of every column of the panel and of the group's
    // vectors (clamped to K - 1), the partial sums of every block
    for (int64_t p = g_sb_npan(n) - 1; p >= 0; --p) {
      const int64_t pj = p * NBK, p0 = pj + SBW, m = n - p0, nb = cdiv(m, BPR);
      if (m < 1 || nb > cdiv(n, BPR)) return 1;
      const int64_t o = g_sb_voff(n, p) * SBW;
      for (int64_t b = 0; b < nb; ++b) {
        const int64_t rb = b * BPR, re = std::min<int64_t>(rb + BPR, m);
        for (int c = 0; c < SBW; c += SBW - 1) C.range("vrow", o + c * m + rb, o + c * m + re, "k_bp V");
        for (int64_t g = 0; g < cdiv(K, BPV); ++g)
          for (int v = 0; v < BPV; ++v) {
            const int64_t l = std::min<int64_t>(g * BPV + v, K - 1);
            C.range("X", l * n + p0 + rb, l * n + p0 + re, "k_bp x");
            C.range("bxw", (b * K + l) * SBW, (b * K + l) * SBW + SBW, "k_bp partial");
          }
      }
      C.range("Tm", p * NBK * NBK, (p + 1) * NBK * NBK, "k_bp_apply T");
    }
    C.range("X", 0, K * n, "k_bx_q0");
    C.range("vbuf", 0, n, "k_bx_q0");
  }
  return 0;
}

int run(int64_t n, bool a64, int64_t K) {
  const size_t el = a64 ? 16 : 8;
  const bool two = K < 0;  // K = -1 - k: the two-stage reduction with k refined
  if (two) K = -1 - K;
  const size_t need = ws_layout(n, a64, nullptr, nullptr, K, two);
  std::vector<char> buf(need);
  Desc D{};
  ws_layout(n, a64, &D, buf.data(), K, two);
  Check C;
  C.base = buf.data();
  C.bytes = need;
  const int64_t R = g_records(n), P2 = g_nwg(n);
  const bool tiles = n - 1 > TILE_M;
  const int64_t slots = tiles ? g_yslots(n) : 0;
  C.add("A", D.A, el, n * D.lda);
  C.add("V", D.V, 16, D.ldv * NBK);
  C.add("W", D.W, 16, D.ldv * NBK);
  C.add("col", D.col, 16, n);
  C.add("y", D.y, 16, n);
  C.add("ys", D.ys, 16, slots * D.ldys);
  C.add("wraw", D.wraw, 16, n);
  C.add("vbuf", D.vbuf, 16, n);
  C.add("partb0", D.partb0, 16, R * PS);
  C.add("partb1", D.partb1, 16, R * PS);
  C.add("parta", D.parta, 16, std::max<int64_t>(std::max<int64_t>(n, 1), slots * (slots + 1) / 2));
  C.add("bred", D.bred, 16, 2 * NBK);
  C.add("part2", D.part2, 16, P2);
  C.add("part3", D.part3, 8, P2);
  C.add("scl", D.scl, 16, n + 1);
  C.add("tau", D.tau, 16, n + 1);
  C.add("d", D.d, 8, n);
  C.add("e", D.e, 8, n);
  C.add("e2", D.e2, 8, n);
  C.add("tsc", D.tsc, 8, 8);
  C.add("bgrid", D.bgrid, 4, NGRID);
  C.add("beta0", D.beta0, 8, 1);
  C.add("status", D.status, 4, 4);
  if (K > 0) {
    C.add("Vall", D.Vall, 16, D.Vall ? n * D.ldv : 0);
    C.add("Z", D.Z, 8, K * n);
    C.add("X", D.X, 16, K * n);
    C.add("rqp", D.rqp, 16, K * cdiv(n, HXR));
    C.add("scr", D.scr, 8, K * 6 * CMAX * n);
    C.add("wref", D.wref, 8, K);
    C.add("Tm", D.Tm, 16, std::max<int64_t>(cdiv(n - 1, NBK), 1) * NBK * NBK);
    C.add("clo", D.clo, 4, n);
  }
  C.layout_ok();
  if (D.ldys != n || D.lda < n || D.ldv < n || D.lda % 16 || D.ldv % 64) {
    std::fprintf(stderr, "leading dimensions\n");
    return 1;
  }
  // ---- copy-in and the initial reflection ----
  C.range("A", 0, (n - 1) * D.lda + n, "k_copy_in");
  C.range("part3", 0, kind_wgs<float>(K_LOADB, n, 0, 4), "k_load_b");
  C.range("col", 0, n, "k_load_b");
  C.range("y", 0, n, "k_hemv0");
  C.range("vbuf", 0, n, "k_hemv0");
  C.range("part2", 0, kind_wgs<float>(K_W0, n, 0, 4), "k_w0");
  C.range("wraw", 0, n, "k_w0");
  C.at("tau", 0, "k_hemv0");
  C.at("beta0", 0, "k_hemv0");
  if (two) {
    if (run_two_stage(C, D, n, a64)) {
      std::fprintf(stderr, "two-stage launch sequence out of bounds\n");
      return 1;
    }
  }
  // ---- blocked columns ----
  int cur = 0;
  for (int64_t j0 = 0; j0 < (two ? 0 : n); j0 += NBK) {
    if (j0 == g_tail0(n)) {  // k_tail: rows and columns j0..n of A, the tridiagonal
      C.range("A", j0 * D.lda + j0, (n - 1) * D.lda + n, "k_tail");
      C.range("d", j0, n, "k_tail");
      C.range("e", j0, n, "k_tail");
      C.range("tau", j0, n + 1, "k_tail");
      C.range("scl", j0, n + 1, "k_tail");
      if (K > 0) C.range("Vall", j0 * D.ldv, n * D.ldv, "k_tail");
      break;
    }
    const int nbk = g_nbk(n, j0);
    const char *Vn = K > 0 ? "Vall" : "V";
    const int64_t voff = K > 0 ? j0 * D.ldv : 0;
    {  // k_col0
      const int64_t g = kind_wgs<float>(K_COL0, n, j0, 4);
      C.range("col", j0, n, "k_col0");
      for (int64_t wg = 0; wg < g; ++wg) C.at(cur ? "partb1" : "partb0", wg * PS, "k_col0");
    }
    for (int i = 0; i < nbk; ++i) {
      const int64_t jn = j0 + i, m = n - jn - 1, m0 = jn + 1;
      const int wpr = single_wpr(m) == 4 ? 4 : (m > TILE_M ? tile_wpr(m) : 0);
      const int np = g_np_in(n, jn);
      if (np > PMAX) {
        std::fprintf(stderr, "k_colA reads %d records > PMAX\n", np);
        return 1;
      }
      const char *pin = cur ? "partb1" : "partb0";
      C.range(pin, 0, int64_t(np - 1) * PS + 1 + 2 * NBK, "k_colA records");
      const int64_t ga = wpr < 0 ? g_tiles(n, m0, tile_of(wpr)) : g_colA_wgs(m, wpr);
      if (ga != kind_wgs<float>(K_COLA, n, jn, wpr)) return 1;
      for (int64_t wg = 0; wg < std::min<int64_t>(ga, 4); ++wg)
        C.range("bred", 16 * wg, 16 * wg + 16, "k_colA");
      C.range("parta", 0, ga, "k_colA");
      C.at("d", jn, "k_colA");
      if (m > 0) {
        C.at("e", jn, "k_colA");
        C.at("tau", m0, "k_colA");
        C.at("scl", m0, "k_colA");
      }
      int64_t nbt = 0;
      if (wpr < 0) {
        const int T = tile_of(wpr);
        const int64_t base = g_tbase(m0);
        nbt = g_tblocks(n, m0, T);
        if (nbt > slots) {
          std::fprintf(stderr, "column %lld: %lld tile blocks > %lld slots\n", (long long)jn,
                       (long long)nbt, (long long)slots);
          return 1;
        }
        for (int64_t wg = 0; wg < ga; ++wg) {
          int64_t bi, bj;
          tri_of(wg, bi, bj);
          if (bi >= nbt || bj > bi) {
            std::fprintf(stderr, "tile %lld of %lld\n", (long long)wg, (long long)ga);
            return 1;
          }
          const int64_t r0 = base + bi * T, c0 = base + bj * T;
          // rows r0 .. r0 + T (clamped into [m0, n)); columns up to lda
          const int64_t rlo = std::min(std::max(r0, m0), n - 1);
          const int64_t rhi = std::min(std::max(r0 + T - 1, m0), n - 1);
          const int64_t chi = std::min<int64_t>(c0 + T - 1, D.lda - 1);
          C.at("A", rlo * D.lda + c0, "k_colA tile");
          C.at("A", rhi * D.lda + chi, "k_colA tile");
          // thread t < T stores row r0 + t and column c0 + t when they lie in [m0, n)
          const int64_t ra = std::max(r0, m0), rb = std::min(r0 + T, n);
          const int64_t ca = std::max(c0, m0), cb = std::min(c0 + T, n);
          C.range("ys", bj * D.ldys + ra, bj * D.ldys + rb, "k_colA tile rows");
          if (bi == bj) C.range(Vn, voff + int64_t(i) * D.ldv + ra, voff + int64_t(i) * D.ldv + rb,
                                "k_colA tile V");
          else C.range("ys", bi * D.ldys + ca, bi * D.ldys + cb, "k_colA tile cols");
        }
      } else {
        C.range("y", m0, n, "k_colA");
        C.range(Vn, voff + int64_t(i) * D.ldv + m0, voff + int64_t(i) * D.ldv + n, "k_colA V");
      }
      if (m <= 0) break;
      // k_colB: rows jx .. n in workgroups of RB
      const int64_t jx = jn + 1, gb = cdiv(m, RB);
      const int64_t npa = wpr < 0 ? g_tiles(n, m0, tile_of(wpr)) : g_colA_wgs(m, wpr);
      C.range("parta", 0, npa, "k_colB");
      if (nbt > 0)
        for (int64_t k = 0; k < nbt; ++k) C.range("ys", k * D.ldys + jx, k * D.ldys + n, "k_colB");
      C.range(Vn, voff, voff + int64_t(NBK - 1) * D.ldv + n, "k_colB V");
      C.range("W", int64_t(i) * D.ldv + jx, int64_t(i) * D.ldv + n, "k_colB W");
      C.range("col", jx, n, "k_colB");
      C.at("tau", jx, "k_colB");
      C.at("scl", jx, "k_colB");
      if (g_more(n, jn)) {
        const char *pout = cur ? "partb0" : "partb1";
        for (int64_t wg = 0; wg < gb; ++wg) C.range(pout, wg * PS, wg * PS + PS, "k_colB");
        if (g_np_in(n, jn + 1) != gb) {
          std::fprintf(stderr, "column %lld: k_colB writes %lld records, the next k_colA reads "
                       "%d\n", (long long)jn, (long long)gb, g_np_in(n, jn + 1));
          return 1;
        }
      }
      cur ^= 1;
    }
    // k_her2k: tiles of BM/2 x BN complex entries from c0, both tile shapes
    const int64_t c0 = j0 + nbk;
    for (int ht = 0; ht < 2; ++ht) {
      const int64_t gh = a64 ? kind_wgs<double>(K_HER2K, n, j0, 4, ht)
                             : kind_wgs<float>(K_HER2K, n, j0, 4, ht);
      if (gh <= 0) continue;
      const int BN = ht ? HerTile<float, 1>::BN : HerTile<float, 0>::BN;
      const int BM = ht ? HerTile<float, 1>::BM : HerTile<float, 0>::BM;
      const int64_t t = cdiv(n - c0, int64_t(BN));
      for (int64_t wg = 0; wg < gh; ++wg) {
        int64_t bx, by;
        if (!her_tri(t, BN)) {
          bx = wg % t;
          by = wg / t;
        } else {
          tri_of(wg, by, bx);
        }
        const int64_t a0 = c0 + by * (BM / 2), b0 = c0 + bx * BN;
        if (a0 >= n || b0 >= n) continue;
        const int64_t a1 = std::min<int64_t>(a0 + BM / 2, n) - 1;
        const int64_t b1 = std::min<int64_t>(b0 + BN, n) - 1;
        C.at("A", a0 * D.lda + b0, "k_her2k");
        C.at("A", a1 * D.lda + b1, "k_her2k");
        C.at("A", b1 * D.lda + a1, "k_her2k mirror");
      }
      C.range(Vn, voff, voff + int64_t(nbk - 1) * D.ldv + n, "k_her2k V");
      C.range("W", 0, int64_t(nbk - 1) * D.ldv + n, "k_her2k W");
    }
  }
  // ---- tridiagonal step ----
  C.range("d", 0, n, "k_tri_prep");
  C.range("e2", 0, n, "k_tri_prep");
  C.range("tsc", 0, 8, "k_tri_prep");
  C.range("status", 0, 4, "k_tri_prep");
  C.range("bgrid", 0, NGRID, "k_bisect_grid");
  if (K > 0) {
    C.range("clo", 0, n, "k_weights (clusters), k_invit, k_rq_fin");
    C.range("Z", 0, K * n, "k_invit");
    C.range("scr", 0, K * 6 * CMAX * n, "k_invit");
    if (!two) C.range("Tm", 0, std::max<int64_t>(cdiv(n - 1, NBK), 1) * NBK * NBK, "k_bx_tmat");
    C.range("X", 0, K * n, "k_backxf");
    C.range("rqp", 0, K * cdiv(n, HXR), "k_hx_part");
    C.range("wref", 0, K, "k_rq_fin");
  }
  std::printf("n = %lld %s K = %lld%s: workspace %zu B, %zu regions, %lld accesses in bounds\n",
              (long long)n, a64 ? "FP64" : "FP32", (long long)K, two ? " two-stage" : "", need,
              C.regs.size(), (long long)C.touches);
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 4 || (argc - 1) % 3) {
    std::fprintf(stderr, "usage: %s n a_fp64 K [n a_fp64 K ...]\n", argv[0]);
    return 2;
  }
  for (int a = 1; a + 2 < argc; a += 3) {
    const int r = run(std::atoll(argv[a]), std::atoi(argv[a + 1]) != 0, std::atoll(argv[a + 2]));
    if (r) return r;
  }
  return 0;
}
