// Host side of the library: point groups, orbit tables and the per-orbit
// symmetry-adapted bases.  All integer work is exact; the bases are FP64.
//
// Paper: Sec. III.C.1 (operations act on k as A k folded into the zone,
// Eq. (sk)); Sec. III.C.2 (pairs related by one operation share their
// interaction elements); Sec. III.C.4 (projector Eq. (projection) applied to
// unit vectors orbit by orbit, then orthonormalised; U is sparse with at most
// |S| d_max^2 non-zeros per vector).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "bse_internal.h"

namespace bse {

static thread_local std::string t_err;

int32_t fail(int32_t st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return st;
}

// ---------------------------------------------------------------------------
// Oh: 48 signed permutation matrices; classes of O from the proper part.
// Character table of O over (E, 8C3, 3C2, 6C4, 6C2'); u irreps carry det(R).
// ---------------------------------------------------------------------------
static void mat3_mul(const double *a, const double *b, double *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      c[3 * i + j] = s;
    }
}

static double det3(const double *m) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

static Group make_oh() {
  Group g;
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<int> cls;  // 0 E, 1 C3, 2 C2, 3 C4, 4 C2'
  std::vector<int> det;
  for (int p = 0; p < 6; ++p)
    for (int sg = 0; sg < 8; ++sg) {
      int32_t m[9] = {0};
      for (int i = 0; i < 3; ++i) m[3 * i + perms[p][i]] = (sg >> (2 - i)) & 1 ? -1 : 1;
      double r[9];
      for (int i = 0; i < 9; ++i) r[i] = m[i];
      int d = (int)std::lround(det3(r));
      int tr = 0, offdiag = 0;
      for (int i = 0; i < 3; ++i) tr += d * m[4 * i];
      for (int i = 0; i < 9; ++i)
        if (i % 4 != 0 && m[i] != 0) offdiag = 1;
      int c = tr == 3 ? 0 : tr == 0 ? 1 : tr == 1 ? 3 : (offdiag ? 4 : 2);
      g.kmat.insert(g.kmat.end(), m, m + 9);
      g.rcart.insert(g.rcart.end(), r, r + 9);
      cls.push_back(c);
      det.push_back(d);
    }
  g.nops = 48;
  struct Row { const char *nm; int dim; int chi[5]; };
  static const Row tab[5] = {{"A1", 1, {1, 1, 1, 1, 1}},  {"A2", 1, {1, 1, 1, -1, -1}},
                             {"E", 2, {2, -1, 2, 0, 0}},  {"T1", 3, {3, 0, -1, 1, -1}},
                             {"T2", 3, {3, 0, -1, -1, 1}}};
  for (int par = 0; par < 2; ++par)
    for (const Row &r : tab) {
      Group::Irrep ir;
      ir.name = std::string(r.nm) + (par ? "u" : "g");
      ir.dim = r.dim;
      for (int s = 0; s < g.nops; ++s) ir.chi.push_back(double(r.chi[cls[s]] * (par ? det[s] : 1)));
      g.irreps.push_back(ir);
    }
  return g;
}

// ---------------------------------------------------------------------------
// D6h on a hexagonal lattice a1 = (1,0), a2 = (-1/2, sqrt3/2).  Proper ops:
// rotations about z by m*60 deg and two-fold rotations about in-plane axes
// every 30 deg; improper ops are their products with the inversion.  The
// reduced-k action is B^-1 R B with B = [b1 b2], b1 = (1, 1/sqrt3),
// b2 = (0, 2/sqrt3).  Classes of D6: E, C6, C3, C2, C2' (axes at 0, 60, 120
// deg, i.e. along a1, a1+a2, a2) and C2'' (30, 90, 150 deg).
// ---------------------------------------------------------------------------
static Group make_d6h() {
  Group g;
  const double PI = 3.14159265358979323846;
  std::vector<std::vector<double>> prop;
  std::vector<int> cls;  // 0 E, 1 C6, 2 C3, 3 C2, 4 C2', 5 C2''
  for (int m = 0; m < 6; ++m) {
    double t = m * PI / 3, c = std::cos(t), s = std::sin(t);
    prop.push_back({c, -s, 0, s, c, 0, 0, 0, 1});
    static const int rc[6] = {0, 1, 2, 3, 2, 1};
    cls.push_back(rc[m]);
  }
  for (int j = 0; j < 6; ++j) {
    double phi = j * PI / 6, c2 = std::cos(2 * phi), s2 = std::sin(2 * phi);
    // rotation by pi about (cos phi, sin phi, 0): in-plane reflection across
    // the axis, z -> -z
    prop.push_back({c2, s2, 0, s2, -c2, 0, 0, 0, -1});
    cls.push_back(j % 2 == 0 ? 4 : 5);
  }
  const double s3 = std::sqrt(3.0);
  const double B[4] = {1.0, 0.0, 1.0 / s3, 2.0 / s3};     // columns b1, b2
  const double Binv[4] = {1.0, 0.0, -0.5, s3 / 2.0};       // inverse of B
  std::vector<int> det;
  for (int inv = 0; inv < 2; ++inv)
    for (size_t o = 0; o < prop.size(); ++o) {
      double r[9];
      for (int i = 0; i < 9; ++i) r[i] = inv ? -prop[o][i] : prop[o][i];
      // M2 = Binv * R2 * B
      double t[4], m2[4];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) t[2 * i + j] = r[3 * i] * B[j] + r[3 * i + 1] * B[2 + j];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) m2[2 * i + j] = Binv[2 * i] * t[j] + Binv[2 * i + 1] * t[2 + j];
      int32_t m[9] = {0};
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) m[3 * i + j] = (int32_t)std::lround(m2[2 * i + j]);
      m[8] = (int32_t)std::lround(r[8]);
      g.kmat.insert(g.kmat.end(), m, m + 9);
      g.rcart.insert(g.rcart.end(), r, r + 9);
      det.push_back(inv ? -1 : 1);
    }
  g.nops = 24;
  struct Row { const char *nm; int dim; int chi[6]; };
  static const Row tab[6] = {{"A1", 1, {1, 1, 1, 1, 1, 1}},   {"A2", 1, {1, 1, 1, 1, -1, -1}},
                             {"B1", 1, {1, -1, 1, -1, 1, -1}}, {"B2", 1, {1, -1, 1, -1, -1, 1}},
                             {"E1", 2, {2, 1, -1, -2, 0, 0}},  {"E2", 2, {2, -1, -1, 2, 0, 0}}};
  for (int par = 0; par < 2; ++par)
    for (const Row &rw : tab) {
      Group::Irrep ir;
      ir.name = std::string(rw.nm) + (par ? "u" : "g");
      ir.dim = rw.dim;
      for (int s = 0; s < g.nops; ++s)
        ir.chi.push_back(double(rw.chi[cls[s % 12]] * (par ? det[s] : 1)));
      g.irreps.push_back(ir);
    }
  return g;
}

const Group *get_group(int32_t group) {
  static std::once_flag once;
  static Group oh, d6h;
  std::call_once(once, [] {
    oh = make_oh();
    d6h = make_d6h();
  });
  if (group == BSE_GROUP_OH) return &oh;
  if (group == BSE_GROUP_D6H) return &d6h;
  return nullptr;
}

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
static int32_t check_grid(const Group *g, const int32_t *grid3, Grid &gr) {
  if (!g) return fail(BSE_EINVAL, "unknown group id");
  if (!grid3) return fail(BSE_EINVAL, "grid is NULL");
  gr = Grid{grid3[0], grid3[1], grid3[2]};
  if (gr.n1 < 1 || gr.n2 < 1 || gr.n3 < 1) return fail(BSE_ESHAPE, "grid sizes must be >= 1");
  // the group must map the grid onto itself: the k matrices need equal sizes
  // along directions they mix
  for (int s = 0; s < g->nops; ++s)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (g->kmat[9 * s + 3 * i + j] != 0 && grid3[i] != grid3[j])
          return fail(BSE_ESHAPE, "grid %dx%dx%d is not invariant under the group", grid3[0],
                      grid3[1], grid3[2]);
  if (gr.nk() * gr.nk() >= (int64_t(1) << 31))
    return fail(BSE_ESHAPE, "nk^2 must fit in int32 (nk = %lld)", (long long)gr.nk());
  return BSE_OK;
}

static void build_kperm(const Group *g, const Grid &gr, std::vector<int32_t> &kp) {
  const int64_t nk = gr.nk();
  kp.resize(size_t(g->nops) * nk);
  const int n[3] = {gr.n1, gr.n2, gr.n3};
  for (int s = 0; s < g->nops; ++s) {
    const int32_t *m = &g->kmat[9 * s];
    for (int a = 0; a < gr.n1; ++a)
      for (int b = 0; b < gr.n2; ++b)
        for (int c = 0; c < gr.n3; ++c) {
          int k[3] = {a, b, c}, o[3];
          for (int i = 0; i < 3; ++i) {
            int64_t v = int64_t(m[3 * i]) * k[0] + int64_t(m[3 * i + 1]) * k[1] +
                        int64_t(m[3 * i + 2]) * k[2];
            v %= n[i];
            if (v < 0) v += n[i];
            o[i] = int(v);
          }
          kp[size_t(s) * nk + (int64_t(a) * gr.n2 + b) * gr.n3 + c] =
              int32_t((int64_t(o[0]) * gr.n2 + o[1]) * gr.n3 + o[2]);
        }
  }
}

struct Tables {
  int64_t nk = 0;
  int nops = 0;
  std::vector<int32_t> kperm, korb, korb_rep, porb, porb_rep, pidx, cls_rep;
  std::vector<uint8_t> pconj, cls_selfswap;
};

static void build_tables(const Group *g, const Grid &gr, Tables &t, bool pairs) {
  t.nk = gr.nk();
  t.nops = g->nops;
  const int64_t nk = t.nk;
  build_kperm(g, gr, t.kperm);
  // k orbits: representative = smallest image
  std::vector<int32_t> rep(nk);
  for (int64_t k = 0; k < nk; ++k) {
    int32_t m = int32_t(k);
    for (int s = 0; s < t.nops; ++s) m = std::min(m, t.kperm[size_t(s) * nk + k]);
    rep[k] = m;
  }
  std::vector<int32_t> id(nk, -1);
  t.korb_rep.clear();
  for (int64_t k = 0; k < nk; ++k)
    if (rep[k] == k) {
      id[k] = int32_t(t.korb_rep.size());
      t.korb_rep.push_back(int32_t(k));
    }
  t.korb.resize(nk);
  for (int64_t k = 0; k < nk; ++k) t.korb[k] = id[rep[k]];
  if (!pairs) return;
  // pair orbits under the diagonal action
  const int64_t np = nk * nk;
  std::vector<int32_t> prep(np);
  for (int64_t k = 0; k < nk; ++k)
    for (int64_t k2 = 0; k2 < nk; ++k2) {
      int64_t m = k * nk + k2;
      for (int s = 0; s < t.nops; ++s) {
        int64_t v = int64_t(t.kperm[size_t(s) * nk + k]) * nk + t.kperm[size_t(s) * nk + k2];
        if (v < m) m = v;
      }
      prep[k * nk + k2] = int32_t(m);
    }
  std::vector<int32_t> pid(np, -1);
  t.porb_rep.clear();
  for (int64_t p = 0; p < np; ++p)
    if (prep[p] == p) {
      pid[p] = int32_t(t.porb_rep.size());
      t.porb_rep.push_back(int32_t(p));
    }
  t.porb.resize(np);
  for (int64_t p = 0; p < np; ++p) t.porb[p] = pid[prep[p]];
  // swap partners and storage classes
  const int64_t nporb = int64_t(t.porb_rep.size());
  std::vector<int32_t> swp(nporb), cls(nporb, -1);
  for (int64_t o = 0; o < nporb; ++o) {
    int64_t p = t.porb_rep[o], k = p / nk, k2 = p % nk;
    swp[o] = t.porb[k2 * nk + k];
  }
  t.cls_rep.clear();
  t.cls_selfswap.clear();
  for (int64_t o = 0; o < nporb; ++o)
    if (o <= swp[o]) {
      cls[o] = int32_t(t.cls_rep.size());
      t.cls_rep.push_back(t.porb_rep[o]);
      t.cls_selfswap.push_back(uint8_t(o == swp[o]));
    }
  t.pidx.resize(np);
  t.pconj.resize(np);
  for (int64_t p = 0; p < np; ++p) {
    int32_t o = t.porb[p];
    int32_t owner = std::min<int32_t>(o, swp[o]);
    t.pidx[p] = cls[owner];
    t.pconj[p] = uint8_t(o > swp[o]);
  }
}

// ---------------------------------------------------------------------------
// per-orbit symmetry-adapted basis
// ---------------------------------------------------------------------------
struct BlockBasis {
  int64_t n = 0, nub = 0;
  std::vector<int32_t> mem_off, members, orb_dim;
  std::vector<int64_t> orb_off, ub_off;
  std::vector<double> ub;
};

// Cartesian rows spanned by a vector irrep: its characters are the trace of
// an invariant sub-block of the rotation matrices (T1u of Oh: x, y, z; E1u of
// D6h: x, y; A2u of D6h: z).  Returns false for the other irreps.
static bool vector_rows(const Group *g, int irrep, std::vector<int> &rows) {
  const Group::Irrep &ir = g->irreps[irrep];
  const int sets[7][3] = {{0, 1, 2}, {0, 1, -1}, {0, 2, -1}, {1, 2, -1},
                          {0, -1, -1}, {1, -1, -1}, {2, -1, -1}};
  for (const auto &st : sets) {
    std::vector<int> S;
    for (int i = 0; i < 3; ++i)
      if (st[i] >= 0) S.push_back(st[i]);
    if (int(S.size()) != ir.dim) continue;
    bool ok = true;
    for (int s = 0; s < g->nops && ok; ++s) {
      const double *R = &g->rcart[size_t(s) * 9];
      double tr = 0;
      for (int i : S) tr += R[i * 3 + i];
      if (std::fabs(tr - ir.chi[s]) > 1e-12) ok = false;
      for (int i : S)  // invariance: no coupling to rows outside S
        for (int j = 0; j < 3 && ok; ++j)
          if (std::find(S.begin(), S.end(), j) == S.end() && std::fabs(R[i * 3 + j]) > 1e-12)
            ok = false;
    }
    if (ok) {
      rows = S;
      return true;
    }
  }
  return false;
}

// weights w[s] of the projector P = d/|G| sum_s w[s] Gamma(s): the characters
// (isotypic block, Eq. (projection)) or, for partner row p >= 0 of a vector
// irrep, the diagonal irrep-matrix element Gamma(s)_pp = (R_s)_ii
static int32_t projector_weights(const Group *g, int irrep, int partner,
                                 std::vector<double> &w) {
  if (irrep < 0 || irrep >= int(g->irreps.size())) return fail(BSE_EINVAL, "irrep out of range");
  const Group::Irrep &ir = g->irreps[irrep];
  if (partner < 0) {
    w = ir.chi;
    return BSE_OK;
  }
  std::vector<int> rows;
  if (!vector_rows(g, irrep, rows))
    return fail(BSE_EUNSUPPORTED, "partner blocks need a vector irrep (%s is not one)",
                ir.name.c_str());
  if (partner >= ir.dim) return fail(BSE_EINVAL, "partner row %d >= dim %d", partner, ir.dim);
  const int i = rows[partner];
  w.resize(g->nops);
  for (int s = 0; s < g->nops; ++s) w[s] = g->rcart[size_t(s) * 9 + i * 3 + i];
  return BSE_OK;
}

static int32_t build_basis(const Group *g, const Grid &gr, int irrep, int nv, int nc,
                           BlockBasis &bb, int partner = -1) {
  if (irrep < 0 || irrep >= int(g->irreps.size())) return fail(BSE_EINVAL, "irrep out of range");
  if (nv < 1 || nc < 1) return fail(BSE_ESHAPE, "nv, nc must be >= 1");
  std::vector<double> wts;
  int32_t st = projector_weights(g, irrep, partner, wts);
  if (st) return st;
  Tables t;
  build_tables(g, gr, t, false);
  const int64_t nk = t.nk;
  const int nkorb = int(t.korb_rep.size());
  const Group::Irrep &ir = g->irreps[irrep];
  const double scale = double(ir.dim) / g->nops;
  bb = BlockBasis();
  bb.mem_off.assign(nkorb + 1, 0);
  for (int64_t k = 0; k < nk; ++k) bb.mem_off[t.korb[k] + 1]++;
  for (int o = 0; o < nkorb; ++o) bb.mem_off[o + 1] += bb.mem_off[o];
  bb.members.assign(nk, 0);
  std::vector<int32_t> fill(bb.mem_off.begin(), bb.mem_off.end() - 1), pos(nk);
  for (int64_t k = 0; k < nk; ++k) {
    int o = t.korb[k];
    pos[k] = fill[o] - bb.mem_off[o];
    bb.members[fill[o]++] = int32_t(k);
  }
  bb.orb_off.assign(nkorb, 0);
  bb.orb_dim.assign(nkorb, 0);
  bb.ub_off.assign(nkorb + 1, 0);
  const int64_t nb = int64_t(nv) * nc;
  for (int o = 0; o < nkorb; ++o) {
    const int L = bb.mem_off[o + 1] - bb.mem_off[o];
    const int32_t *mem = &bb.members[bb.mem_off[o]];
    // projector restricted to the orbit: P[i][j] = d/|G| sum_s w(s) [s m_j = m_i]
    std::vector<double> P(size_t(L) * L, 0.0);
    for (int s = 0; s < g->nops; ++s)
      for (int j = 0; j < L; ++j) {
        int32_t img = t.kperm[size_t(s) * nk + mem[j]];
        P[size_t(pos[img]) * L + j] += wts[s];
      }
    double tr = 0;
    for (int i = 0; i < L; ++i) tr += P[size_t(i) * L + i] * scale;
    const int r = int(std::lround(tr));
    if (std::fabs(tr - r) > 1e-9 || r < 0 || r > L)
      return fail(BSE_EINVAL, "projector trace %.12f on orbit %d is not an integer", tr, o);
    // Gram-Schmidt with column pivoting over the columns of P (the range of an
    // orthogonal projector is spanned by its columns)
    std::vector<double> cols(size_t(L) * L);  // column j stored contiguously
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) cols[size_t(j) * L + i] = P[size_t(i) * L + j] * scale;
    std::vector<double> U(size_t(L) * r, 0.0);
    std::vector<char> used(L, 0);
    for (int q = 0; q < r; ++q) {
      int best = -1;
      double bn = 0;
      for (int j = 0; j < L; ++j) {
        if (used[j]) continue;
        double s = 0;
        for (int i = 0; i < L; ++i) s += cols[size_t(j) * L + i] * cols[size_t(j) * L + i];
        if (s > bn) { bn = s; best = j; }
      }
      if (best < 0 || bn < 1e-20) return fail(BSE_EINVAL, "basis rank deficit on orbit %d", o);
      used[best] = 1;
      double *u = &cols[size_t(best) * L];
      const double inv = 1.0 / std::sqrt(bn);
      for (int i = 0; i < L; ++i) U[size_t(i) * r + q] = u[i] * inv;
      for (int j = 0; j < L; ++j) {  // orthogonalise the rest (twice)
        if (used[j]) continue;
        double *c = &cols[size_t(j) * L];
        for (int pass = 0; pass < 2; ++pass) {
          double dt = 0;
          for (int i = 0; i < L; ++i) dt += U[size_t(i) * r + q] * c[i];
          for (int i = 0; i < L; ++i) c[i] -= dt * U[size_t(i) * r + q];
        }
      }
    }
    for (int j = 0; j < L; ++j) {  // the remaining columns must lie in the span
      if (used[j]) continue;
      double s = 0;
      for (int i = 0; i < L; ++i) s += cols[size_t(j) * L + i] * cols[size_t(j) * L + i];
      if (s > 1e-16) return fail(BSE_EINVAL, "projector range exceeds rank on orbit %d", o);
    }
    bb.orb_off[o] = bb.n;
    bb.orb_dim[o] = r;
    bb.ub_off[o + 1] = bb.ub_off[o] + int64_t(L) * r;
    bb.ub.insert(bb.ub.end(), U.begin(), U.end());
    bb.n += int64_t(r) * nb;
  }
  bb.nub = bb.ub_off[nkorb];
  return BSE_OK;
}

}  // namespace bse

// ===========================================================================
// C ABI
// ===========================================================================
using namespace bse;

extern "C" const char *bse_last_error(void) { return t_err.c_str(); }
extern "C" const char *bse_version(void) { return "bse-mi355x 0.1 (gfx950)"; }

extern "C" int32_t bse_group_order(int32_t group) {
  const Group *g = get_group(group);
  return g ? g->nops : fail(BSE_EINVAL, "unknown group id %d", group);
}

extern "C" int32_t bse_group_nirreps(int32_t group) {
  const Group *g = get_group(group);
  return g ? int32_t(g->irreps.size()) : fail(BSE_EINVAL, "unknown group id %d", group);
}

extern "C" int32_t bse_group_ops(int32_t group, int32_t *h_kmat, double *h_rcart) {
  const Group *g = get_group(group);
  if (!g) return fail(BSE_EINVAL, "unknown group id %d", group);
  if (h_kmat) std::memcpy(h_kmat, g->kmat.data(), g->kmat.size() * sizeof(int32_t));
  if (h_rcart) std::memcpy(h_rcart, g->rcart.data(), g->rcart.size() * sizeof(double));
  return BSE_OK;
}

extern "C" int32_t bse_group_irrep(int32_t group, int32_t irrep, char *h_name8, int32_t *h_dim,
                                   double *h_chi) {
  const Group *g = get_group(group);
  if (!g) return fail(BSE_EINVAL, "unknown group id %d", group);
  if (irrep < 0 || irrep >= int(g->irreps.size())) return fail(BSE_EINVAL, "irrep out of range");
  const Group::Irrep &ir = g->irreps[irrep];
  if (h_name8) {
    std::memset(h_name8, 0, 8);
    std::strncpy(h_name8, ir.name.c_str(), 7);
  }
  if (h_dim) *h_dim = ir.dim;
  if (h_chi) std::memcpy(h_chi, ir.chi.data(), ir.chi.size() * sizeof(double));
  return BSE_OK;
}

extern "C" int32_t bse_dims_get(int32_t group, const int32_t *h_grid3, bse_dims *h_out) {
  const Group *g = get_group(group);
  Grid gr;
  int32_t st = check_grid(g, h_grid3, gr);
  if (st) return st;
  if (!h_out) return fail(BSE_EINVAL, "out is NULL");
  Tables t;
  build_tables(g, gr, t, true);
  h_out->grid[0] = gr.n1; h_out->grid[1] = gr.n2; h_out->grid[2] = gr.n3;
  h_out->nk = int32_t(t.nk);
  h_out->nops = g->nops;
  h_out->nkorb = int32_t(t.korb_rep.size());
  h_out->nporb = int32_t(t.porb_rep.size());
  h_out->ncls = int32_t(t.cls_rep.size());
  return BSE_OK;
}

extern "C" int32_t bse_tables_build(int32_t group, const int32_t *h_grid3, const bse_tables *o) {
  const Group *g = get_group(group);
  Grid gr;
  int32_t st = check_grid(g, h_grid3, gr);
  if (st) return st;
  if (!o) return fail(BSE_EINVAL, "out is NULL");
  Tables t;
  build_tables(g, gr, t, true);
  auto cp = [](void *dst, const void *src, size_t bytes) {
    if (dst) std::memcpy(dst, src, bytes);
  };
  cp(o->kperm, t.kperm.data(), t.kperm.size() * 4);
  cp(o->korb, t.korb.data(), t.korb.size() * 4);
  cp(o->korb_rep, t.korb_rep.data(), t.korb_rep.size() * 4);
  cp(o->porb, t.porb.data(), t.porb.size() * 4);
  cp(o->porb_rep, t.porb_rep.data(), t.porb_rep.size() * 4);
  cp(o->pidx, t.pidx.data(), t.pidx.size() * 4);
  cp(o->pconj, t.pconj.data(), t.pconj.size());
  cp(o->cls_rep, t.cls_rep.data(), t.cls_rep.size() * 4);
  cp(o->cls_selfswap, t.cls_selfswap.data(), t.cls_selfswap.size());
  return BSE_OK;
}

namespace {
int32_t dims_impl(int32_t group, const int32_t *h_grid3, int32_t irrep, int32_t partner,
                  int32_t nv, int32_t nc, bse_block_dims *h_out) {
  const Group *g = get_group(group);
  Grid gr;
  int32_t st = check_grid(g, h_grid3, gr);
  if (st) return st;
  if (!h_out) return fail(BSE_EINVAL, "out is NULL");
  BlockBasis bb;
  st = build_basis(g, gr, irrep, nv, nc, bb, partner);
  if (st) return st;
  h_out->n = bb.n;
  h_out->nmem = int32_t(gr.nk());
  h_out->nub = bb.nub;
  return BSE_OK;
}

int32_t basis_impl(int32_t group, const int32_t *h_grid3, int32_t irrep, int32_t partner,
                   int32_t nv, int32_t nc, int32_t *h_mem_off, int32_t *h_members,
                   int64_t *h_orb_off, int32_t *h_orb_dim, int64_t *h_ub_off, double *h_ubasis) {
  const Group *g = get_group(group);
  Grid gr;
  int32_t st = check_grid(g, h_grid3, gr);
  if (st) return st;
  BlockBasis bb;
  st = build_basis(g, gr, irrep, nv, nc, bb, partner);
  if (st) return st;
  auto cp = [](void *dst, const void *src, size_t bytes) {
    if (dst) std::memcpy(dst, src, bytes);
  };
  cp(h_mem_off, bb.mem_off.data(), bb.mem_off.size() * 4);
  cp(h_members, bb.members.data(), bb.members.size() * 4);
  cp(h_orb_off, bb.orb_off.data(), bb.orb_off.size() * 8);
  cp(h_orb_dim, bb.orb_dim.data(), bb.orb_dim.size() * 4);
  cp(h_ub_off, bb.ub_off.data(), bb.ub_off.size() * 8);
  cp(h_ubasis, bb.ub.data(), bb.ub.size() * 8);
  return BSE_OK;
}
}  // namespace

extern "C" int32_t bse_block_dims_get(int32_t group, const int32_t *h_grid3, int32_t irrep,
                                      int32_t nv, int32_t nc, bse_block_dims *h_out) {
  return dims_impl(group, h_grid3, irrep, -1, nv, nc, h_out);
}

extern "C" int32_t bse_block_basis(int32_t group, const int32_t *h_grid3, int32_t irrep,
                                   int32_t nv, int32_t nc, int32_t *h_mem_off, int32_t *h_members,
                                   int64_t *h_orb_off, int32_t *h_orb_dim, int64_t *h_ub_off,
                                   double *h_ubasis) {
  return basis_impl(group, h_grid3, irrep, -1, nv, nc, h_mem_off, h_members, h_orb_off,
                    h_orb_dim, h_ub_off, h_ubasis);
}

extern "C" int32_t bse_partner_block_dims_get(int32_t group, const int32_t *h_grid3,
                                              int32_t irrep, int32_t partner, int32_t nv,
                                              int32_t nc, bse_block_dims *h_out) {
  if (partner < 0) return fail(BSE_EINVAL, "partner row must be >= 0");
  return dims_impl(group, h_grid3, irrep, partner, nv, nc, h_out);
}

extern "C" int32_t bse_partner_block_basis(int32_t group, const int32_t *h_grid3, int32_t irrep,
                                           int32_t partner, int32_t nv, int32_t nc,
                                           int32_t *h_mem_off, int32_t *h_members,
                                           int64_t *h_orb_off, int32_t *h_orb_dim,
                                           int64_t *h_ub_off, double *h_ubasis) {
  if (partner < 0) return fail(BSE_EINVAL, "partner row must be >= 0");
  return basis_impl(group, h_grid3, irrep, partner, nv, nc, h_mem_off, h_members, h_orb_off,
                    h_orb_dim, h_ub_off, h_ubasis);
}
