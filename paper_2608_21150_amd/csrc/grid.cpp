// Host grid layer: validation, optional space-filling-curve renumbering, canonical
// connectivity, orientation signs and stencil coefficients.
//
// Neighbour access on the icosahedral grid goes through index lookup tables
// (paper, Section 4.2.1); the grid is the RnBk construction of Section 5.1.
// Canonical orders (they are readings; the paper fixes none):
//   e2v[e]     ordered so that (x_v1 - x_v0) . t_e > 0, t_e = x_e x n_e
//   c2e[c]     input order if it runs counter-clockwise seen from outside,
//              else slots 1 and 2 swapped; c2e[c][i] joins c2v[i], c2v[i+1]
//   c2v[c][i]  common vertex of c2e[c][i-1] and c2e[c][i]
//   c2e2c      cell across c2e[c][i]; s = +1 where c is the edge's first cell
//   v2e[v]     counter-clockwise from the smallest incident edge id, -1 pad
//   v2c[v][i]  cell between v2e[v][i] and v2e[v][i+1]
//   e2c2e[e]   other edges of c0 then of c1, in c2e order
//   e2c2v[e]   v0, v1, vertex of c0 off e, vertex of c1 off e
// Space-filling-curve renumbering: cells by (triangle-tree key, id), edges
// by (min new cell, max new cell, id), vertices by (min new id of their
// cells, id).  The key descends a recursive subdivision of a fixed
// icosahedron (poles on the z axis, rings at z = +-1/sqrt 5, longitudes 72 i
// and 72 i + 36 degrees): the face whose smallest great-circle side test is
// largest, then 16 levels of 4-way splits at normalised edge midpoints
// (corner children first, the middle child otherwise), two bits per level.
// Runs of 4^j consecutive keys are spherical triangles: a 64-cell block of
// a subdivided icosahedral grid is one compact patch.
// This file is compiled without floating-point contraction so that the
// floating-point decisions above (orientation tests, the tree's side tests)
// are taken exactly as written.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace dc {

namespace {

struct V3 {
  double x, y, z;
};
inline V3 ld(const std::vector<double>& a, int i) { return {a[3 * i], a[3 * i + 1], a[3 * i + 2]}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// a . (b x c), summed in this order
inline double det3(V3 a, V3 b, V3 c) {
  return (a.x * (b.y * c.z - b.z * c.y) + a.y * (b.z * c.x - b.x * c.z)) + a.z * (b.x * c.y - b.y * c.x);
}
inline V3 mid(V3 p, V3 q) {
  const V3 s = add(p, q);
  const double n = std::sqrt((s.x * s.x + s.y * s.y) + s.z * s.z);
  return {s.x / n, s.y / n, s.z / n};
}

constexpr int kTreeLevels = 16;

uint64_t tree_key(V3 x) {
  const double s5 = std::sqrt(5.0);
  const double c1 = (s5 - 1.0) / 2.0, s1 = std::sqrt(10.0 + 2.0 * s5) / 2.0;  // 2 cos 72, 2 sin 72
  const double c2 = (s5 + 1.0) / 2.0, s2 = std::sqrt(10.0 - 2.0 * s5) / 2.0;  // 2 cos 36, 2 sin 36
  const double raw[12][3] = {{0.0, 0.0, s5},  {2.0, 0.0, 1.0},  {c1, s1, 1.0},    {-c2, s2, 1.0},
                             {-c2, -s2, 1.0}, {c1, -s1, 1.0},   {c2, s2, -1.0},   {-c1, s1, -1.0},
                             {-2.0, 0.0, -1.0}, {-c1, -s1, -1.0}, {c2, -s2, -1.0}, {0.0, 0.0, -s5}};
  static const int faces[20][3] = {{0, 1, 2},  {1, 6, 2},  {2, 6, 7},  {11, 7, 6}, {0, 2, 3},
                                   {2, 7, 3},  {3, 7, 8},  {11, 8, 7}, {0, 3, 4},  {3, 8, 4},
                                   {4, 8, 9},  {11, 9, 8}, {0, 4, 5},  {4, 9, 5},  {5, 9, 10},
                                   {11, 10, 9}, {0, 5, 1}, {5, 10, 1}, {1, 10, 6}, {11, 6, 10}};
  V3 v[12];
  for (int i = 0; i < 12; ++i) v[i] = {raw[i][0] / s5, raw[i][1] / s5, raw[i][2] / s5};
  int face = 0;
  double best = -INFINITY;
  for (int f = 0; f < 20; ++f) {
    const V3 a = v[faces[f][0]], b = v[faces[f][1]], c = v[faces[f][2]];
    const double m = std::min(std::min(det3(x, b, c), det3(a, x, c)), det3(a, b, x));
    if (m > best) {
      best = m;
      face = f;
    }
  }
  V3 a = v[faces[face][0]], b = v[faces[face][1]], c = v[faces[face][2]];
  uint64_t key = (uint64_t)face;
  for (int l = 0; l < kTreeLevels; ++l) {
    const V3 ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
    int ch;
    if (det3(x, ab, ca) > 0) {
      ch = 0;
      b = ab;
      c = ca;
    } else if (det3(x, bc, ab) > 0) {
      ch = 1;
      a = ab;
      c = bc;
    } else if (det3(x, ca, bc) > 0) {
      ch = 2;
      a = ca;
      b = bc;
    } else {
      ch = 3;
      a = ab;
      b = bc;
      c = ca;
    }
    key = key * 4 + (uint64_t)ch;
  }
  return key;
}

bool finite_pos(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(std::isfinite(a[i]) && a[i] > 0.0)) return false;
  return true;
}
bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

void lsq_vertex_weights(const HostGrid& g, int v, double w[3][6]) {
  // V = P (N P)^+ vn: least-squares fit of the normal winds of the incident
  // edges by a vector tangent to the sphere at the vertex.
  V3 x = ld(g.xv, v);
  V3 ax = std::fabs(x.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
  V3 e1 = cross(ax, x);
  e1 = scl(e1, 1.0 / norm(e1));
  V3 e2 = cross(x, e1);
  double np[6][2] = {};
  for (int s = 0; s < 6; ++s) {
    int e = g.v2e[6 * v + s];
    if (e < 0) continue;
    V3 n = ld(g.nrm, e);
    np[s][0] = dot(n, e1);
    np[s][1] = dot(n, e2);
  }
  double a = 0, b = 0, c = 0;  // G = (NP)^T (NP) = [[a b][b c]]
  for (int s = 0; s < 6; ++s) {
    a += np[s][0] * np[s][0];
    b += np[s][0] * np[s][1];
    c += np[s][1] * np[s][1];
  }
  const double det = a * c - b * b;
  const double i00 = c / det, i01 = -b / det, i11 = a / det;
  for (int s = 0; s < 6; ++s) {
    const double p0 = i00 * np[s][0] + i01 * np[s][1];
    const double p1 = i01 * np[s][0] + i11 * np[s][1];
    w[0][s] = e1.x * p0 + e2.x * p1;
    w[1][s] = e1.y * p0 + e2.y * p1;
    w[2][s] = e1.z * p0 + e2.z * p1;
  }
}

namespace {

// orthonormal pair spanning the tangent plane at the unit vector x
void plane_basis(V3 x, V3* e1, V3* e2) {
  const V3 ax = std::fabs(x.y) < 0.9 ? V3{0, 1, 0} : V3{0, 0, 1};
  V3 a = cross(x, ax);
  *e1 = scl(a, 1.0 / norm(a));
  *e2 = cross(x, *e1);
}

// Solve the n x n system M y = b in place (row-major M, n <= 8) by Gaussian
// elimination with partial pivoting; false if a pivot vanishes.
bool solve_small(double* M, double* b, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[i * n + k]) > std::fabs(M[piv * n + k])) piv = i;
    if (!(std::fabs(M[piv * n + k]) > 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(M[k * n + j], M[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = M[i * n + k] / M[k * n + k];
      for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double acc = b[k];
    for (int j = k + 1; j < n; ++j) acc -= M[k * n + j] * b[j];
    b[k] = acc / M[k * n + k];
  }
  return true;
}

}  // namespace

// Tangential wind by radial-basis-function vector reconstruction (the
// interpolation of ICON's discretisation, Section 4.1): over the stencil
// {e, e2c2e[e][0..3]} a field sum_j a_j phi(|x - x_j|) n_j + c, with c a
// constant vector in the tangent plane at x_e, matches the normal winds at
// the stencil's midpoints, its coefficients being orthogonal to the
// constants (sum_j a_j n_j . b = 0 for the plane's two directions b);
// vt_e = t_e . v(x_e).  phi(r) = 1 / sqrt(1 + (r / eps)^2), eps = 0.5 l_e,
// positions in metres.  vt_e is linear in the five winds: its weights are
// the first five entries of the solution of the (symmetric) system with
// the evaluation functional as right-hand side.  Slot-major [5][es].
bool build_rbf_vt(HostGrid* g) {
  const int ne = g->ne, es = g->es;
  const double R = g->radius;
  g->k_vt_rbf.assign(5 * (size_t)es, 0.0);
  for (int e = 0; e < ne; ++e) {
    int st[5] = {e, g->e2c2e[4 * e], g->e2c2e[4 * e + 1], g->e2c2e[4 * e + 2], g->e2c2e[4 * e + 3]};
    V3 x[5], n[5];
    for (int i = 0; i < 5; ++i) {
      x[i] = scl(ld(g->xe, st[i]), R);
      n[i] = ld(g->nrm, st[i]);
    }
    const double eps = 0.5 * g->l[e];
    auto phi = [&](double r) { return 1.0 / std::sqrt(1.0 + (r / eps) * (r / eps)); };
    V3 b1, b2;
    plane_basis(ld(g->xe, e), &b1, &b2);
    const V3 t = ld(g->tan, e);
    double M[49] = {}, rhs[7];
    for (int i = 0; i < 5; ++i) {
      for (int j = 0; j < 5; ++j) M[i * 7 + j] = phi(norm(sub(x[i], x[j]))) * dot(n[i], n[j]);
      M[i * 7 + 5] = M[5 * 7 + i] = dot(n[i], b1);
      M[i * 7 + 6] = M[6 * 7 + i] = dot(n[i], b2);
      rhs[i] = phi(norm(sub(x[0], x[i]))) * dot(n[i], t);
    }
    rhs[5] = dot(t, b1);
    rhs[6] = dot(t, b2);
    if (!solve_small(M, rhs, 7)) return false;
    // k_vt's slot order: self, then e2c2e[0..3]
    for (int i = 0; i < 5; ++i) g->k_vt_rbf[i * es + e] = rhs[i];
  }
  return true;
}

// Second-order upwind (Miura) edge values of cell scalars (Section 4.1):
// q_e = q_up + grad q_up . (x* - R x_up), x* = R x_e - dtau (vn n_e + vt t_e)
// the departure point of the edge midpoint, up the upwind cell (c0 when
// vn >= 0), grad the least-squares gradient over the three neighbour cells
// in the tangent plane at x_up, grad q = sum_i W_i (q_i - q_up).  Per side
// s (0: c0 upwind, 1: c1) and neighbour i the table holds
// a_i = W_i . (R x_e - R x_up), b_i = W_i . n_e, c_i = W_i . t_e, so that
// q_e = q_up + sum_i (a_i - dtau (vn b_i + vt c_i)) (q_i - q_up);
// slot 9 s + 3 m + i (m: a, b, c), [18][es].
void build_miura(HostGrid* g) {
  const int nc = g->nc, ne = g->ne, es = g->es;
  const double R = g->radius;
  // gradient weights of every cell: W = [e1 e2] (D^T D)^-1 D^T, D the 3 x 2
  // plane coordinates of the neighbour offsets
  std::vector<double> W(9 * (size_t)nc);
  for (int c = 0; c < nc; ++c) {
    const V3 xc = ld(g->xc, c);
    V3 e1, e2;
    plane_basis(xc, &e1, &e2);
    double D[3][2];
    for (int i = 0; i < 3; ++i) {
      const V3 d = scl(sub(ld(g->xc, g->c2e2c[3 * c + i]), xc), R);
      D[i][0] = dot(d, e1);
      D[i][1] = dot(d, e2);
    }
    double a = 0, b = 0, cc = 0;
    for (int i = 0; i < 3; ++i) {
      a += D[i][0] * D[i][0];
      b += D[i][0] * D[i][1];
      cc += D[i][1] * D[i][1];
    }
    const double det = a * cc - b * b;
    for (int i = 0; i < 3; ++i) {
      const double p0 = (cc * D[i][0] - b * D[i][1]) / det;
      const double p1 = (a * D[i][1] - b * D[i][0]) / det;
      const V3 w = add(scl(e1, p0), scl(e2, p1));
      W[9 * c + 3 * i + 0] = w.x;
      W[9 * c + 3 * i + 1] = w.y;
      W[9 * c + 3 * i + 2] = w.z;
    }
  }
  g->k_miura.assign(18 * (size_t)es, 0.0);
  for (int e = 0; e < ne; ++e) {
    const V3 xe = scl(ld(g->xe, e), R), n = ld(g->nrm, e), t = ld(g->tan, e);
    for (int s = 0; s < 2; ++s) {
      const int c = g->e2c[2 * e + s];
      const V3 off = sub(xe, scl(ld(g->xc, c), R));
      for (int i = 0; i < 3; ++i) {
        const V3 w{W[9 * c + 3 * i], W[9 * c + 3 * i + 1], W[9 * c + 3 * i + 2]};
        g->k_miura[(9 * s + 0 + i) * es + e] = dot(w, off);
        g->k_miura[(9 * s + 3 + i) * es + e] = dot(w, n);
        g->k_miura[(9 * s + 6 + i) * es + e] = dot(w, t);
      }
    }
  }
}

// Tiles of the fused edge pass (layout in internal.h).  Staged order: the
// tile's own edges in id order, then R1, R2 and the remaining edges around
// the tile's vertices, each in order of first appearance.
void build_edge_tiles(HostGrid* g) {
  using T = EdgeTiles;
  const int ne = g->ne, nt = (ne + T::kTileE - 1) / T::kTileE;
  g->et_ok = 0;
  g->et_ntile = nt;
  g->et_n.assign(4 * (size_t)nt, 0);
  g->et_x.assign((size_t)T::XM * nt, 0);
  g->et_vx.assign((size_t)T::VM * nt, 0);
  g->et_nb.assign((size_t)4 * T::XV * nt, 0);
  g->et_vl.assign((size_t)6 * T::VM * nt, 0);
  g->et_ev.assign((size_t)2 * T::kTileE * nt, 0);
  std::vector<int> pos(ne, -1), vpos(g->nv, -1);
  std::vector<int> ext, vert;
  const int vs = g->vs;
  for (int t = 0; t < nt; ++t) {
    const int e0 = t * T::kTileE, e1 = std::min(ne, e0 + T::kTileE);
    ext.clear();
    vert.clear();
    auto add = [&](int e) {
      if (pos[e] < 0) {
        pos[e] = (int)ext.size();
        ext.push_back(e);
      }
    };
    for (int e = e0; e < e1; ++e) add(e);
    const int n_own = e1 - e0;
    for (int i = 0; i < n_own; ++i)
      for (int s = 0; s < 4; ++s) add(g->e2c2e[4 * ext[i] + s]);
    const int n_vt = (int)ext.size();
    for (int i = n_own; i < n_vt; ++i)
      for (int s = 0; s < 4; ++s) add(g->e2c2e[4 * ext[i] + s]);
    for (int i = 0; i < n_own; ++i)
      for (int s = 0; s < 2; ++s) {
        const int v = g->e2v[2 * ext[i] + s];
        if (vpos[v] < 0) {
          vpos[v] = (int)vert.size();
          vert.push_back(v);
        }
      }
    for (int v : vert)
      for (int s = 0; s < 6; ++s) add(g->t_v2e[s * vs + v]);
    const int n_ext = (int)ext.size(), n_v = (int)vert.size();
    const bool fits = n_ext <= T::XM && n_vt <= T::XV && n_v <= T::VM;
    if (fits) {
      const size_t tt = t;
      g->et_n[4 * tt + 0] = n_own;
      g->et_n[4 * tt + 1] = n_vt;
      g->et_n[4 * tt + 2] = n_ext;
      g->et_n[4 * tt + 3] = n_v;
      for (int p = 0; p < T::XM; ++p) g->et_x[tt * T::XM + p] = ext[p < n_ext ? p : 0];
      for (int l = 0; l < n_vt; ++l)
        for (int s = 0; s < 4; ++s) g->et_nb[(tt * 4 + s) * T::XV + l] = (uint16_t)pos[g->e2c2e[4 * ext[l] + s]];
      for (int v = 0; v < n_v; ++v) {
        g->et_vx[tt * T::VM + v] = vert[v];
        for (int s = 0; s < 6; ++s) g->et_vl[(tt * 6 + s) * T::VM + v] = (uint16_t)pos[g->t_v2e[s * vs + vert[v]]];
      }
      for (int i = 0; i < n_own; ++i)
        for (int s = 0; s < 2; ++s) g->et_ev[(tt * 2 + s) * T::kTileE + i] = (uint16_t)vpos[g->e2v[2 * ext[i] + s]];
    }
    for (int e : ext) pos[e] = -1;
    for (int v : vert) vpos[v] = -1;
    if (!fits) {
      std::vector<int32_t>().swap(g->et_n);
      std::vector<int32_t>().swap(g->et_x);
      std::vector<int32_t>().swap(g->et_vx);
      std::vector<uint16_t>().swap(g->et_nb);
      std::vector<uint16_t>().swap(g->et_vl);
      std::vector<uint16_t>().swap(g->et_ev);
      return;
    }
  }
  g->et_ok = 1;
}

int build_host_grid(const dc_grid_desc* D, HostGrid* g, std::string* err) {
  auto fail = [&](int code, const std::string& m) {
    *err = m;
    return code;
  };
  if (!D) return fail(DC_EINVAL, "grid description is NULL");
  const int nc = D->n_cells, ne = D->n_edges, nv = D->n_verts, K = D->n_lev;
  if (nc <= 0 || ne <= 0 || nv <= 0 || K < 1) return fail(DC_EINVAL, "entity counts must be > 0 and n_lev >= 1");
  if (nc > (1 << 28) || ne > (1 << 28) || nv > (1 << 28)) return fail(DC_EINVAL, "grid too large");
  if (K > 129) return fail(DC_EINVAL, "n_lev must be <= 129 (8 column chunks of at most 16 levels)");
  if (!D->e2c || !D->c2e || !D->e2v || !D->c2e2c || !D->vert_xyz || !D->cell_xyz || !D->edge_xyz ||
      !D->edge_length || !D->dual_edge_length || !D->cell_area || !D->dual_area || !D->edge_normal_xyz ||
      !D->z_half || !D->exner_ref_full || !D->theta_ref_full || !D->theta_ref_half || !D->dexner_dz_ref_half)
    return fail(DC_EINVAL, "a grid description pointer is NULL");
  if (!(D->radius > 0.0) || !std::isfinite(D->radius)) return fail(DC_EINVAL, "radius must be > 0");
  if (D->sfc_reorder != 0 && D->sfc_reorder != 1) return fail(DC_EINVAL, "sfc_reorder must be 0 or 1");

  // ---- validation of the given tables (original numbering) ----
  for (int i = 0; i < 2 * ne; ++i)
    if (D->e2c[i] < 0 || D->e2c[i] >= nc) return fail(DC_EGRID, "e2c index out of range");
  for (int i = 0; i < 2 * ne; ++i)
    if (D->e2v[i] < 0 || D->e2v[i] >= nv) return fail(DC_EGRID, "e2v index out of range");
  for (int i = 0; i < 3 * nc; ++i)
    if (D->c2e[i] < 0 || D->c2e[i] >= ne) return fail(DC_EGRID, "c2e index out of range");
  for (int i = 0; i < 3 * nc; ++i)
    if (D->c2e2c[i] < 0 || D->c2e2c[i] >= nc) return fail(DC_EGRID, "c2e2c index out of range");
  if ((long long)nv - ne + nc != 2) return fail(DC_EGRID, "Euler characteristic V - E + C != 2");
  for (int e = 0; e < ne; ++e) {
    if (D->e2c[2 * e] == D->e2c[2 * e + 1]) return fail(DC_EGRID, "edge with identical cells");
    if (D->e2v[2 * e] == D->e2v[2 * e + 1]) return fail(DC_EGRID, "edge with identical vertices");
  }
  {
    std::vector<int> cnt(ne, 0);
    for (int c = 0; c < nc; ++c)
      for (int i = 0; i < 3; ++i) {
        const int e = D->c2e[3 * c + i];
        if (D->e2c[2 * e] != c && D->e2c[2 * e + 1] != c) return fail(DC_EGRID, "c2e and e2c disagree");
        cnt[e]++;
      }
    for (int e = 0; e < ne; ++e)
      if (cnt[e] != 2) return fail(DC_EGRID, "an edge is not in exactly two cells");
    for (int c = 0; c < nc; ++c) {
      int across[3], given[3];
      for (int i = 0; i < 3; ++i) {
        const int e = D->c2e[3 * c + i];
        across[i] = D->e2c[2 * e] == c ? D->e2c[2 * e + 1] : D->e2c[2 * e];
        given[i] = D->c2e2c[3 * c + i];
      }
      std::sort(across, across + 3);
      std::sort(given, given + 3);
      if (!std::equal(across, across + 3, given)) return fail(DC_EGRID, "c2e2c disagrees with c2e/e2c");
      // the three edges must close a triangle: 3 distinct vertices, each on 2 edges
      int vs[6];
      for (int i = 0; i < 3; ++i) {
        const int e = D->c2e[3 * c + i];
        vs[2 * i] = D->e2v[2 * e];
        vs[2 * i + 1] = D->e2v[2 * e + 1];
      }
      std::sort(vs, vs + 6);
      if (!(vs[0] == vs[1] && vs[2] == vs[3] && vs[4] == vs[5] && vs[1] != vs[2] && vs[3] != vs[4]))
        return fail(DC_EGRID, "the edges of a cell do not form a triangle");
    }
  }
  if (!finite_pos(D->edge_length, ne) || !finite_pos(D->dual_edge_length, ne) || !finite_pos(D->cell_area, nc) ||
      !finite_pos(D->dual_area, nv))
    return fail(DC_EGRID, "lengths and areas must be finite and > 0");
  if (!finite_all(D->vert_xyz, 3 * (size_t)nv) || !finite_all(D->cell_xyz, 3 * (size_t)nc) ||
      !finite_all(D->edge_xyz, 3 * (size_t)ne) || !finite_all(D->edge_normal_xyz, 3 * (size_t)ne))
    return fail(DC_EGRID, "positions and normals must be finite");
  for (int e = 0; e < ne; ++e) {
    V3 n{D->edge_normal_xyz[3 * e], D->edge_normal_xyz[3 * e + 1], D->edge_normal_xyz[3 * e + 2]};
    const int c0 = D->e2c[2 * e], c1 = D->e2c[2 * e + 1];
    V3 x0{D->cell_xyz[3 * c0], D->cell_xyz[3 * c0 + 1], D->cell_xyz[3 * c0 + 2]};
    V3 x1{D->cell_xyz[3 * c1], D->cell_xyz[3 * c1 + 1], D->cell_xyz[3 * c1 + 2]};
    if (!(dot(n, sub(x1, x0)) > 0.0)) return fail(DC_EGRID, "edge normal does not point from e2c[0] to e2c[1]");
  }
  if (!finite_all(D->z_half, K + 1)) return fail(DC_EGRID, "z_half must be finite");
  for (int k = 0; k < K; ++k)
    if (!(D->z_half[k] > D->z_half[k + 1])) return fail(DC_EGRID, "z_half must decrease strictly (level 0 = top)");
  if (!finite_pos(D->exner_ref_full, K) || !finite_pos(D->theta_ref_full, K) || !finite_pos(D->theta_ref_half, K + 1) ||
      !finite_all(D->dexner_dz_ref_half, K + 1))
    return fail(DC_EGRID, "reference profiles must be finite (and positive for Exner and theta)");

  g->nc = nc;
  g->ne = ne;
  g->nv = nv;
  g->K = K;
  g->radius = D->radius;
  g->mean_area = 4.0 * M_PI * D->radius * D->radius / nc;

  // ---- optional space-filling-curve renumbering (permutations internal -> original) ----
  std::vector<int32_t> pc(nc), pe(ne), pv(nv);
  std::iota(pc.begin(), pc.end(), 0);
  std::iota(pe.begin(), pe.end(), 0);
  std::iota(pv.begin(), pv.end(), 0);
  if (D->sfc_reorder) {
    std::vector<uint64_t> key(nc);
    for (int c = 0; c < nc; ++c) key[c] = tree_key({D->cell_xyz[3 * c], D->cell_xyz[3 * c + 1], D->cell_xyz[3 * c + 2]});
    std::stable_sort(pc.begin(), pc.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int32_t> oc(nc);
    for (int i = 0; i < nc; ++i) oc[pc[i]] = i;
    std::vector<int32_t> lo(ne), hi(ne);
    for (int e = 0; e < ne; ++e) {
      const int a = oc[D->e2c[2 * e]], b = oc[D->e2c[2 * e + 1]];
      lo[e] = std::min(a, b);
      hi[e] = std::max(a, b);
    }
    std::stable_sort(pe.begin(), pe.end(), [&](int a, int b) { return lo[a] != lo[b] ? lo[a] < lo[b] : hi[a] < hi[b]; });
    std::vector<int32_t> vmin(nv, INT32_MAX);
    for (int c = 0; c < nc; ++c)
      for (int i = 0; i < 3; ++i) {
        const int e = D->c2e[3 * c + i];
        for (int j = 0; j < 2; ++j) {
          const int v = D->e2v[2 * e + j];
          vmin[v] = std::min(vmin[v], oc[c]);
        }
      }
    std::stable_sort(pv.begin(), pv.end(), [&](int a, int b) { return vmin[a] < vmin[b]; });
  }
  std::vector<int32_t> oc(nc), oe(ne), ov(nv);
  for (int i = 0; i < nc; ++i) oc[pc[i]] = i;
  for (int i = 0; i < ne; ++i) oe[pe[i]] = i;
  for (int i = 0; i < nv; ++i) ov[pv[i]] = i;
  g->perm_c = pc;
  g->perm_e = pe;
  g->perm_v = pv;

  // renumbered inputs and geometry
  std::vector<int32_t> e2c(2 * ne), e2v_in(2 * ne), c2e_in(3 * nc);
  for (int e = 0; e < ne; ++e)
    for (int j = 0; j < 2; ++j) {
      e2c[2 * e + j] = oc[D->e2c[2 * pe[e] + j]];
      e2v_in[2 * e + j] = ov[D->e2v[2 * pe[e] + j]];
    }
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 3; ++i) c2e_in[3 * c + i] = oe[D->c2e[3 * pc[c] + i]];
  g->xv.resize(3 * nv);
  g->xe.resize(3 * ne);
  g->xc.resize(3 * nc);
  g->nrm.resize(3 * ne);
  g->tan.resize(3 * ne);
  g->l.resize(ne);
  g->d.resize(ne);
  g->ac.resize(nc);
  g->av.resize(nv);
  for (int v = 0; v < nv; ++v) {
    for (int j = 0; j < 3; ++j) g->xv[3 * v + j] = D->vert_xyz[3 * pv[v] + j];
    g->av[v] = D->dual_area[pv[v]];
  }
  for (int c = 0; c < nc; ++c) {
    for (int j = 0; j < 3; ++j) g->xc[3 * c + j] = D->cell_xyz[3 * pc[c] + j];
    g->ac[c] = D->cell_area[pc[c]];
  }
  for (int e = 0; e < ne; ++e) {
    for (int j = 0; j < 3; ++j) {
      g->xe[3 * e + j] = D->edge_xyz[3 * pe[e] + j];
      g->nrm[3 * e + j] = D->edge_normal_xyz[3 * pe[e] + j];
    }
    g->l[e] = D->edge_length[pe[e]];
    g->d[e] = D->dual_edge_length[pe[e]];
  }

  // ---- canonical tables ----
  g->e2c = e2c;
  g->e2v.resize(2 * ne);
  for (int e = 0; e < ne; ++e) {
    V3 t = cross(ld(g->xe, e), ld(g->nrm, e));
    g->tan[3 * e] = t.x;
    g->tan[3 * e + 1] = t.y;
    g->tan[3 * e + 2] = t.z;
    const int a = e2v_in[2 * e], b = e2v_in[2 * e + 1];
    const double along = dot(sub(ld(g->xv, b), ld(g->xv, a)), t);
    g->e2v[2 * e] = along > 0 ? a : b;
    g->e2v[2 * e + 1] = along > 0 ? b : a;
  }
  auto common = [&](int ea, int eb) {
    const int a0 = g->e2v[2 * ea], a1 = g->e2v[2 * ea + 1];
    return (a0 == g->e2v[2 * eb] || a0 == g->e2v[2 * eb + 1]) ? a0 : a1;
  };
  g->c2e.resize(3 * nc);
  g->c2v.resize(3 * nc);
  g->c2e2c.resize(3 * nc);
  g->sgn_c.resize(3 * nc);
  for (int c = 0; c < nc; ++c) {
    int ce[3] = {c2e_in[3 * c], c2e_in[3 * c + 1], c2e_in[3 * c + 2]};
    int cv[3];
    for (int i = 0; i < 3; ++i) cv[i] = common(ce[(i + 2) % 3], ce[i]);
    V3 a = ld(g->xv, cv[0]), b = ld(g->xv, cv[1]), cc = ld(g->xv, cv[2]);
    if (!(dot(cross(sub(b, a), sub(cc, a)), ld(g->xc, c)) > 0)) {
      std::swap(ce[1], ce[2]);
      for (int i = 0; i < 3; ++i) cv[i] = common(ce[(i + 2) % 3], ce[i]);
    }
    for (int i = 0; i < 3; ++i) {
      g->c2e[3 * c + i] = ce[i];
      g->c2v[3 * c + i] = cv[i];
      const bool first = e2c[2 * ce[i]] == c;
      g->c2e2c[3 * c + i] = first ? e2c[2 * ce[i] + 1] : e2c[2 * ce[i]];
      g->sgn_c[3 * c + i] = first ? 1 : -1;
    }
  }
  // counter-clockwise walk around each vertex
  std::vector<int32_t> nxt_e(2 * ne, -1), nxt_c(2 * ne, -1);
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 3; ++i) {
      const int v = g->c2v[3 * c + i];
      const int ef = g->c2e[3 * c + i];
      const int side = g->e2v[2 * ef] != v ? 1 : 0;
      nxt_e[2 * ef + side] = g->c2e[3 * c + (i + 2) % 3];
      nxt_c[2 * ef + side] = c;
    }
  std::vector<int32_t> emin(nv, INT32_MAX);
  for (int e = 0; e < ne; ++e)
    for (int j = 0; j < 2; ++j) emin[g->e2v[2 * e + j]] = std::min(emin[g->e2v[2 * e + j]], e);
  g->v2e.assign(6 * (size_t)nv, -1);
  g->v2c.assign(6 * (size_t)nv, -1);
  g->sgn_v.assign(6 * (size_t)nv, 0);
  for (int v = 0; v < nv; ++v) {
    int cur = emin[v];
    if (cur == INT32_MAX) return fail(DC_EGRID, "vertex without edges");
    bool closed = false;
    for (int i = 0; i < 6; ++i) {
      g->v2e[6 * v + i] = cur;
      g->sgn_v[6 * v + i] = g->e2v[2 * cur + 1] == v ? 1 : -1;
      const int side = g->e2v[2 * cur] != v ? 1 : 0;
      const int nx = nxt_e[2 * cur + side];
      g->v2c[6 * v + i] = nxt_c[2 * cur + side];
      if (nx < 0) return fail(DC_EGRID, "open vertex fan (inconsistent orientation)");
      cur = nx;
      if (cur == emin[v]) {
        closed = true;
        if (i < 2) return fail(DC_EGRID, "vertex with fewer than 3 edges");
        break;
      }
    }
    if (!closed) return fail(DC_EGRID, "a vertex has more than 6 edges");
  }
  g->e2c2e.resize(4 * ne);
  g->e2c2v.resize(4 * ne);
  for (int e = 0; e < ne; ++e) {
    g->e2c2v[4 * e] = g->e2v[2 * e];
    g->e2c2v[4 * e + 1] = g->e2v[2 * e + 1];
    for (int side = 0; side < 2; ++side) {
      const int c = e2c[2 * e + side];
      int m = 0;
      for (int i = 0; i < 3; ++i) {
        const int x = g->c2e[3 * c + i];
        if (x != e) g->e2c2e[4 * e + 2 * side + (m++)] = x;
        const int vv = g->c2v[3 * c + i];
        if (vv != g->e2v[2 * e] && vv != g->e2v[2 * e + 1]) g->e2c2v[4 * e + 2 + side] = vv;
      }
      if (m != 2) return fail(DC_EGRID, "edge not found in its cell");
    }
  }

  // ---- vertical column ----
  g->z_half.assign(D->z_half, D->z_half + K + 1);
  g->ex_ref.assign(D->exner_ref_full, D->exner_ref_full + K);
  g->th_ref.assign(D->theta_ref_full, D->theta_ref_full + K);
  g->th_ref_ic.assign(D->theta_ref_half, D->theta_ref_half + K + 1);
  g->dex_ref_ic.assign(D->dexner_dz_ref_half, D->dexner_dz_ref_half + K + 1);
  const int K1 = K + 1;
  g->vert.assign((size_t)VT_COUNT * K1, 0.0);
  std::vector<double> zf(K);
  for (int j = 0; j < K; ++j) zf[j] = 0.5 * (g->z_half[j] + g->z_half[j + 1]);
  for (int j = 0; j < K; ++j) {
    const double dz = g->z_half[j] - g->z_half[j + 1];
    g->vert[VT_DZF * K1 + j] = dz;
    g->vert[VT_IDZF * K1 + j] = 1.0 / dz;
    g->vert[VT_EXREF * K1 + j] = g->ex_ref[j];
    g->vert[VT_THREF * K1 + j] = g->th_ref[j];
  }
  for (int k = 0; k <= K; ++k) {
    g->vert[VT_THREFIC * K1 + k] = g->th_ref_ic[k];
    g->vert[VT_DEXREFIC * K1 + k] = g->dex_ref_ic[k];
    if (k >= 1 && k <= K - 1) {
      g->vert[VT_IDZH * K1 + k] = 1.0 / (zf[k - 1] - zf[k]);
      g->vert[VT_IDZC2 * K1 + k] = 1.0 / (g->z_half[k - 1] - g->z_half[k + 1]);
    }
  }

  // ---- stencil coefficients (slot-major, padded) ----
  const int cs = pad_to(nc, kPad), es = pad_to(ne, kPad), vs = pad_to(nv, kPad);
  g->cs = cs;
  g->es = es;
  g->vs = vs;
  const double R = g->radius;
  g->t_c2e.assign(3 * (size_t)cs, 0);
  g->t_c2e2c.assign(3 * (size_t)cs, 0);
  g->k_div.assign(3 * (size_t)cs, 0.0);
  g->k_lap.assign(3 * (size_t)cs, 0.0);
  g->k_area.assign(cs, 0.0);
  for (int c = 0; c < nc; ++c) {
    g->k_area[c] = g->ac[c];
    for (int i = 0; i < 3; ++i) {
      const int e = g->c2e[3 * c + i];
      g->t_c2e[i * cs + c] = e;
      g->t_c2e2c[i * cs + c] = g->c2e2c[3 * c + i];
      g->k_div[i * cs + c] = g->sgn_c[3 * c + i] * g->l[e] / g->ac[c];
      g->k_lap[i * cs + c] = g->l[e] / (g->d[e] * g->ac[c]);
    }
  }
  g->t_e2c.assign(2 * (size_t)es, 0);
  g->t_e2v.assign(2 * (size_t)es, 0);
  g->t_e2c2e.assign(4 * (size_t)es, 0);
  g->t_e2c2v.assign(4 * (size_t)es, 0);
  g->k_vt.assign(5 * (size_t)es, 0.0);
  g->k_invd.assign(es, 0.0);
  g->k_invl.assign(es, 0.0);
  g->k_f.assign(es, 0.0);
  g->k_ae.assign(es, 0.0);
  g->k_invlr.assign(es, 0.0);
  g->k_nrm.assign(3 * (size_t)es, 0.0);
  g->k_tan.assign(3 * (size_t)es, 0.0);
  for (int e = 0; e < ne; ++e) {
    for (int j = 0; j < 2; ++j) {
      g->t_e2c[j * es + e] = e2c[2 * e + j];
      g->t_e2v[j * es + e] = g->e2v[2 * e + j];
    }
    for (int j = 0; j < 4; ++j) {
      g->t_e2c2e[j * es + e] = g->e2c2e[4 * e + j];
      g->t_e2c2v[j * es + e] = g->e2c2v[4 * e + j];
    }
    const V3 t = ld(g->tan, e);
    // Perot: vt_e = 1/2 (V_c0 + V_c1) . t_e, V_c = (1/A_c) sum_i s l F (x_ei - x_c) R
    double self = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int c = e2c[2 * e + side];
      int m = 0;
      for (int i = 0; i < 3; ++i) {
        const int x = g->c2e[3 * c + i];
        const double coef = 0.5 * (g->sgn_c[3 * c + i] * g->l[x] / g->ac[c]) * R * dot(sub(ld(g->xe, x), ld(g->xc, c)), t);
        if (x == e)
          self += coef;
        else
          g->k_vt[(1 + 2 * side + (m++)) * es + e] = coef;
      }
    }
    g->k_vt[e] = self;
    g->k_invd[e] = 1.0 / g->d[e];
    g->k_invl[e] = 1.0 / g->l[e];
    g->k_f[e] = 0.0;  // set per state (depends on omega)
    g->k_ae[e] = 0.5 * g->l[e] * g->d[e];
    const V3 x2 = ld(g->xv, g->e2c2v[4 * e + 2]), x3 = ld(g->xv, g->e2c2v[4 * e + 3]);
    g->k_invlr[e] = 1.0 / (R * std::atan2(norm(cross(x2, x3)), dot(x2, x3)));
    for (int j = 0; j < 3; ++j) {
      g->k_nrm[j * es + e] = g->nrm[3 * e + j];
      g->k_tan[j * es + e] = g->tan[3 * e + j];
    }
  }
  g->t_v2e.assign(6 * (size_t)vs, 0);
  g->k_curl.assign(6 * (size_t)vs, 0.0);
  g->k_lsq.assign(18 * (size_t)vs, 0.0);
  for (int v = 0; v < nv; ++v) {
    double w[3][6];
    lsq_vertex_weights(*g, v, w);
    for (int s = 0; s < 6; ++s) {
      const int e = g->v2e[6 * v + s];
      g->t_v2e[s * vs + v] = e >= 0 ? e : g->v2e[6 * v];
      g->k_curl[s * vs + v] = e >= 0 ? g->sgn_v[6 * v + s] * g->d[e] / g->av[v] : 0.0;
      for (int j = 0; j < 3; ++j) g->k_lsq[(j * 6 + s) * vs + v] = e >= 0 ? w[j][s] : 0.0;
    }
  }
  build_edge_tiles(g);
  return DC_OK;
}

}  // namespace dc
