// Host-side setup: macro-primitive graph, per-cell stencils, keys, coarse
// operator.  Runs once per mesh; everything per level is derived in closed
// form from the unit-scale data built here.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hytet_impl.hpp"

namespace ht {

static int offset_index(int di, int dj, int dk) {
  for (int d = 0; d < kNumOffsets; ++d) {
    int a, b, c;
    stencil_offset(d, a, b, c);
    if (a == di && b == dj && c == dk) return d;
  }
  return -1;
}

static double det3(const double E[3][3]) {
  return E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
         E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
         E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
}

// Class-partial stencils and lumped masses of one cell at unit scale
// (micro-tet edge vectors J (o_r - o_0), i.e. level 0 spacing).  At level l
// every entry is divided by 2^l (stiffness) or 8^l (mass): the micro-cells of
// a level are the unit shapes scaled by 2^-l.
static void compute_cell_stencils(const double X[4][3], Cell& cell) {
  std::memset(cell.stencil_unit, 0, sizeof(cell.stencil_unit));
  std::memset(cell.mass_unit, 0, sizeof(cell.mass_unit));
  double J[3][3];  // J[row][col], column c = X_{c+1} - X_0
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) J[r][c] = X[c + 1][r] - X[0][r];
  for (int t = 0; t < 6; ++t) {
    const int(*o)[3] = kShapeOffsets[t];
    double E[3][3];  // rows: physical edge vectors e_r = J (o_r - o_0)
    for (int r = 0; r < 3; ++r)
      for (int a = 0; a < 3; ++a) {
        double v = 0;
        for (int c = 0; c < 3; ++c) v += J[a][c] * (o[r + 1][c] - o[0][c]);
        E[r][a] = v;
      }
    const double det = det3(E);
    const double vol = std::fabs(det) / 6.0;
    // inverse of E by cofactors; grad(lambda_q) = column q-1 of inv(E)
    double inv[3][3];
    inv[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
    inv[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
    inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    inv[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
    inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    inv[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
    inv[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
    inv[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
    inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    double G[4][3];
    for (int q = 1; q < 4; ++q)
      for (int a = 0; a < 3; ++a) G[q][a] = inv[a][q - 1];
    for (int a = 0; a < 3; ++a) G[0][a] = -(G[1][a] + G[2][a] + G[3][a]);
    double K[4][4];
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 4; ++r)
        K[q][r] = vol * (G[q][0] * G[r][0] + G[q][1] * G[r][1] +
                         G[q][2] * G[r][2]);
    {
      static const int kPairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
      for (int p = 0; p < 6; ++p) cell.shape_k[t][p] = K[kPairs[p][0]][kPairs[p][1]];
    }
    // Accumulate into every boundary class: the micro-cell with the point in
    // role q is inside the closure iff none of its vertices crosses a face
    // on which the point lies (offsets have components in {-1,0,1}, so only
    // the faces through the point can be crossed).
    for (int cls = 0; cls < 15; ++cls) {
      for (int q = 0; q < 4; ++q) {
        bool inside = true;
        for (int r = 0; r < 4 && inside; ++r) {
          const int ei = o[r][0] - o[q][0], ej = o[r][1] - o[q][1],
                    ek = o[r][2] - o[q][2];
          if ((cls & 1) && ei < 0) inside = false;
          if ((cls & 2) && ej < 0) inside = false;
          if ((cls & 4) && ek < 0) inside = false;
          if ((cls & 8) && ei + ej + ek > 0) inside = false;
        }
        if (!inside) continue;
        for (int r = 0; r < 4; ++r) {
          const int d = offset_index(o[r][0] - o[q][0], o[r][1] - o[q][1],
                                     o[r][2] - o[q][2]);
          cell.stencil_unit[cls][d] += K[q][r];
        }
        cell.mass_unit[cls] += vol / 4.0;
      }
    }
  }
  cell.volume = std::fabs(det3(J)) / 6.0;
}

// Class bits of the points of the primitive spanned by the local vertices
// `span` (others have zero weight): bit b is set iff local vertex
// face_vertex(b) is not in the span.
static int class_of_span(unsigned span_mask) {
  int cls = 0;
  for (int b = 0; b < 4; ++b)
    if (!(span_mask & (1u << face_vertex(b)))) cls |= 1 << b;
  return cls;
}

void build_mesh(Mesh& m, const double* xyz, int64_t nv, const int64_t* cells,
                int64_t nc, int min_level, int max_level) {
  if (min_level < 0 || max_level < min_level || max_level > 10)
    throw Error{HT_ERR_LEVEL, "levels must satisfy 0 <= min <= max <= 10"};
  if (nv < 4 || nc < 1 || !xyz || !cells)
    throw Error{HT_ERR_ARG, "need nv >= 4, nc >= 1 and non-null arrays"};
  m.nv = nv;
  m.nc = nc;
  m.min_level = min_level;
  m.max_level = max_level;
  m.xyz.assign(xyz, xyz + 3 * nv);
  m.cells.resize(nc);
  for (int64_t c = 0; c < nc; ++c) {
    Cell& cell = m.cells[c];
    double X[4][3];
    for (int q = 0; q < 4; ++q) {
      const int64_t g = cells[4 * c + q];
      if (g < 0 || g >= nv)
        throw Error{HT_ERR_MESH, "cell " + std::to_string(c) +
                                     " has an out-of-range vertex id"};
      cell.gv[q] = g;
      for (int a = 0; a < 3; ++a) X[q][a] = xyz[3 * g + a];
    }
    for (int q = 0; q < 4; ++q)
      for (int r = q + 1; r < 4; ++r)
        if (cell.gv[q] == cell.gv[r])
          throw Error{HT_ERR_MESH,
                      "cell " + std::to_string(c) + " repeats a vertex"};
    double J[3][3], hmax = 0;
    for (int r = 0; r < 3; ++r)
      for (int a = 0; a < 3; ++a) J[r][a] = X[r + 1][a] - X[0][a];
    for (int q = 0; q < 4; ++q)
      for (int r = q + 1; r < 4; ++r) {
        double l2 = 0;
        for (int a = 0; a < 3; ++a) l2 += (X[q][a] - X[r][a]) * (X[q][a] - X[r][a]);
        hmax = std::max(hmax, std::sqrt(l2));
      }
    if (!(std::fabs(det3(J)) > 1e-12 * hmax * hmax * hmax))
      throw Error{HT_ERR_MESH,
                  "cell " + std::to_string(c) + " is degenerate (zero volume)"};
    compute_cell_stencils(X, cell);
  }

  // ---- macro-primitive graph: faces, edges, vertices deduplicated by their
  // sorted global vertex ids.
  std::map<std::array<int64_t, 3>, int32_t> fmap, emap, vmap;
  std::vector<Prim> faces, edges, verts;
  auto add = [&](std::map<std::array<int64_t, 3>, int32_t>& mp,
                 std::vector<Prim>& list, int dim, int64_t c,
                 std::vector<int> lvs) {
    std::sort(lvs.begin(), lvs.end(), [&](int a, int b) {
      return m.cells[c].gv[a] < m.cells[c].gv[b];
    });
    std::array<int64_t, 3> key{-1, -1, -1};
    unsigned span = 0;
    Incidence inc;
    inc.cell = (int32_t)c;
    inc.lv[0] = inc.lv[1] = inc.lv[2] = -1;
    for (size_t s = 0; s < lvs.size(); ++s) {
      key[s] = m.cells[c].gv[lvs[s]];
      inc.lv[s] = (int8_t)lvs[s];
      span |= 1u << lvs[s];
    }
    inc.cls = (int8_t)class_of_span(span);
    auto it = mp.find(key);
    int32_t id;
    if (it == mp.end()) {
      id = (int32_t)list.size();
      mp.emplace(key, id);
      Prim p;
      p.dim = dim;
      p.gv = key;
      list.push_back(p);
    } else {
      id = it->second;
    }
    list[id].inc.push_back(inc);
    return id;
  };
  std::vector<std::array<int32_t, 16>> local_prim(nc);
  for (int64_t c = 0; c < nc; ++c) {
    auto& lp = local_prim[c];
    lp.fill(-1);
    for (int q = 0; q < 4; ++q) {  // face opposite local vertex q
      std::vector<int> lv;
      for (int r = 0; r < 4; ++r)
        if (r != q) lv.push_back(r);
      int32_t id = add(fmap, faces, 2, c, lv);
      lp[class_of_span(0xFu & ~(1u << q))] = id;
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        int32_t id = add(emap, edges, 1, c, {a, b});
        lp[class_of_span((1u << a) | (1u << b))] = id;
      }
    for (int q = 0; q < 4; ++q) {
      int32_t id = add(vmap, verts, 0, c, {q});
      lp[class_of_span(1u << q)] = id;
    }
  }
  for (auto& f : faces)
    if (f.inc.size() > 2)
      throw Error{HT_ERR_MESH, "a face is shared by more than two cells"};
  // boundary: faces with one cell, and their edges and vertices
  for (auto& f : faces) {
    if (f.inc.size() != 1) continue;
    f.boundary = true;
    const int64_t* g = f.gv.data();
    const int64_t pairs[3][2] = {{g[0], g[1]}, {g[0], g[2]}, {g[1], g[2]}};
    for (auto& pr : pairs) edges[emap.at({pr[0], pr[1], -1})].boundary = true;
    for (int s = 0; s < 3; ++s) verts[vmap.at({g[s], -1, -1})].boundary = true;
  }
  m.n_faces = (int64_t)faces.size();
  m.n_edges = (int64_t)edges.size();
  m.n_verts = (int64_t)verts.size();
  m.prims.clear();
  m.prims.reserve(faces.size() + edges.size() + verts.size());
  for (auto* list : {&faces, &edges, &verts})
    for (auto& p : *list) m.prims.push_back(std::move(p));
  const int32_t eoff = (int32_t)m.n_faces, voff = (int32_t)(m.n_faces + m.n_edges);
  for (int64_t c = 0; c < nc; ++c) {
    for (int k = 0; k < 16; ++k) {
      int32_t id = local_prim[c][k];
      if (id >= 0) {
        const int nb = __builtin_popcount(k);
        id += nb == 1 ? 0 : (nb == 2 ? eoff : voff);
      }
      m.cells[c].cls_prim[k] = id;
    }
  }
  for (auto& p : m.prims) {
    p.diag_unit = 0;
    p.mass_unit = 0;
    for (auto& inc : p.inc) {
      p.diag_unit += m.cells[inc.cell].stencil_unit[inc.cls][0];
      p.mass_unit += m.cells[inc.cell].mass_unit[inc.cls];
    }
  }
  m.cls.assign(nc * 16, ClassInfo{});
  for (int64_t c = 0; c < nc; ++c) {
    for (int k = 0; k < 16; ++k) {
      ClassInfo& ci = m.cls[16 * c + k];
      ci.prim = -1;
      ci.flags = 0;
      ci.inv_diag_unit = 0;
      ci.mass_unit = 0;
      if (k == 15) continue;
      ci.flags = kClsValid;
      if (k == 0) {
        ci.flags |= kClsOwner;
        ci.inv_diag_unit = 1.0 / m.cells[c].stencil_unit[0][0];
        ci.mass_unit = m.cells[c].mass_unit[0];
        continue;
      }
      const int32_t pid = m.cells[c].cls_prim[k];
      const Prim& p = m.prims[pid];
      ci.prim = pid;
      if (p.inc[0].cell == c) ci.flags |= kClsOwner;
      if (p.boundary) ci.flags |= kClsDirichlet;
      ci.inv_diag_unit = p.boundary ? 0.0 : 1.0 / p.diag_unit;
      ci.mass_unit = p.mass_unit;
    }
  }
  set_problems(m, {0, nc}, {max_level});
}

// Problem partition of the cells.  Faces, edges and vertices are numbered
// in order of first appearance over the cells, so each problem's primitives
// form a contiguous run of each kind as long as problems are disjoint; this
// is checked here.
void set_problems(Mesh& m, const std::vector<int64_t>& cell_begin,
                  const std::vector<int>& finest_level) {
  const int P = (int)cell_begin.size() - 1;
  if (P < 1 || cell_begin.front() != 0 || cell_begin.back() != m.nc ||
      (int)finest_level.size() != P)
    throw Error{HT_ERR_ARG, "bad problem partition"};
  std::vector<int32_t> prob_of_cell(m.nc);
  for (int p = 0; p < P; ++p) {
    if (cell_begin[p + 1] <= cell_begin[p])
      throw Error{HT_ERR_ARG, "every problem needs at least one cell"};
    if (p > 0 && finest_level[p] > finest_level[p - 1])
      throw Error{HT_ERR_ARG, "problems must be sorted by finest level, descending"};
    for (int64_t c = cell_begin[p]; c < cell_begin[p + 1]; ++c) prob_of_cell[c] = p;
  }
  m.nprob = P;
  m.pcell = cell_begin;
  auto ranges = [&](int64_t first, int64_t count, std::vector<int64_t>& out) {
    out.assign(P + 1, 0);
    int cur = 0;
    for (int64_t q = 0; q < count; ++q) {
      const Prim& pr = m.prims[first + q];
      const int p = prob_of_cell[pr.inc[0].cell];
      for (const Incidence& I : pr.inc)
        if (prob_of_cell[I.cell] != p)
          throw Error{HT_ERR_MESH, "problems of a batch share a primitive"};
      if (p < cur) throw Error{HT_ERR_MESH, "primitives of a problem are not contiguous"};
      while (cur < p) out[++cur] = q;
    }
    while (cur < P) out[++cur] = count;
  };
  ranges(0, m.n_faces, m.pface);
  ranges(m.n_faces, m.n_edges, m.pedge);
  ranges(m.n_faces + m.n_edges, m.n_verts, m.pvert);
  m.act_cells.assign(m.max_level + 1, 0);
  for (int l = 0; l <= m.max_level; ++l) {
    int p1 = 0;
    while (p1 < P && finest_level[p1] >= l) ++p1;
    m.act_cells[l] = cell_begin[p1];
  }
}

Range problem_range(const Mesh& m, int p0, int p1) {
  Range r;
  r.c0 = m.pcell[p0]; r.c1 = m.pcell[p1];
  r.f0 = m.pface[p0]; r.f1 = m.pface[p1];
  r.e0 = m.pedge[p0]; r.e1 = m.pedge[p1];
  r.v0 = m.pvert[p0]; r.v1 = m.pvert[p1];
  return r;
}

void level_scaled_stencils(const Mesh& m, int level, std::vector<double>& w) {
  const double s = std::ldexp(1.0, -level);
  w.resize(m.nc * 16 * 15);
  for (int64_t c = 0; c < m.nc; ++c)
    for (int k = 0; k < 16; ++k)
      for (int d = 0; d < 15; ++d)
        w[(c * 16 + k) * 15 + d] = m.cells[c].stencil_unit[k][d] * s;
}

// -------------------------------------------------------- slot decoding --
// Inverse of slot_in_cell; returns false for padding slots.
static bool decode_offset(const CellLayout& L, int64_t off, int& i, int& j,
                          int& k) {
  const int n = L.n;
  auto decode2 = [](int64_t w, int64_t o, int& jj, int& kk) {
    int64_t base = 0;
    for (kk = 0; kk < w; ++kk) {
      const int64_t row = w - kk;
      if (o < base + row) { jj = (int)(o - base); return; }
      base += row;
    }
  };
  if (off < L.m_size) {
    const int64_t w = n - 1;
    int64_t base = 0;
    for (k = 0; k < w; ++k) {
      const int64_t plane = n_tri(w - k);
      if (off < base + plane) break;
      base += plane;
    }
    int64_t o = off - base;
    for (j = 0; j < w - k; ++j) {
      const int64_t row = w - k - j;
      if (o < row) break;
      o -= row;
    }
    i = (int)o + 1;
    return true;
  }
  if (off >= L.off_s0 && off < L.off_s0 + L.s0_size) {
    decode2(n + 1, off - L.off_s0, j, k);
    i = 0;
    return true;
  }
  if (off >= L.off_s1 && off < L.off_s1 + L.s1_size) {
    decode2(n, off - L.off_s1, j, k);
    i = n - j - k;
    return true;
  }
  return false;
}

void slot_key(const Mesh& m, int level, int64_t slot, int64_t key[8],
              uint8_t* flags) {
  const CellLayout L = make_layout(level);
  const int64_t c = slot / L.stride;
  int i, j, k;
  for (int p = 0; p < 4; ++p) { key[2 * p] = -1; key[2 * p + 1] = 0; }
  if (c >= m.nc || !decode_offset(L, slot % L.stride, i, j, k)) {
    if (flags) *flags = HT_SLOT_PAD;
    return;
  }
  const Cell& cell = m.cells[c];
  const int64_t w[4] = {L.n - i - j - k, i, j, k};
  int order[4] = {0, 1, 2, 3};
  std::sort(order, order + 4, [&](int a, int b) { return cell.gv[a] < cell.gv[b]; });
  int p = 0;
  for (int s = 0; s < 4; ++s)
    if (w[order[s]] > 0) {
      key[2 * p] = cell.gv[order[s]];
      key[2 * p + 1] = w[order[s]];
      ++p;
    }
  if (flags) {
    const int cls = point_class(L.n, i, j, k);
    const ClassInfo& ci = m.cls[16 * c + cls];
    uint8_t f = (ci.flags & kClsOwner) ? HT_SLOT_OWNER : HT_SLOT_GHOST;
    if (ci.flags & kClsDirichlet) f |= HT_SLOT_DIRICHLET;
    *flags = f;
  }
}

void slot_coords(const Mesh& m, int level, int64_t slot, double out[3]) {
  int64_t key[8];
  slot_key(m, level, slot, key, nullptr);
  const double inv_n = std::ldexp(1.0, -level);
  out[0] = out[1] = out[2] = 0.0;
  if (key[0] < 0) return;
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int p = 0; p < 4; ++p)
      if (key[2 * p] >= 0) s += (double)key[2 * p + 1] * m.xyz[3 * key[2 * p] + a];
    out[a] = s * inv_n;
  }
}

// ------------------------------------------------------- coarse solver --
// Dense Cholesky factorisation A = L L^T in place (lower triangle), then the
// inverse A^-1 = L^-T L^-1.  O(N^3) once per mesh and coarse level.
static void cholesky_inverse(std::vector<double>& A, int64_t N) {
  for (int64_t j = 0; j < N; ++j) {
    double d = A[j * N + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * N + k] * A[j * N + k];
    if (!(d > 0)) throw Error{HT_ERR_MESH, "coarse matrix is not SPD"};
    d = std::sqrt(d);
    A[j * N + j] = d;
    parallel_for(N - j - 1, [&](int64_t lo, int64_t hi) {
      for (int64_t i = j + 1 + lo; i < j + 1 + hi; ++i) {
        double s = A[i * N + j];
        const double* ri = &A[i * N];
        const double* rj = &A[j * N];
        for (int64_t k = 0; k < j; ++k) s -= ri[k] * rj[k];
        A[i * N + j] = s / d;
      }
    }, 64);
  }
  // Linv (lower) by columns: solve L x = e_c.
  std::vector<double> Li(N * N, 0.0);  // Li[r*N + c]
  // columns interleaved over threads for balance (column c costs ~(N-c)^2)
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t t = lo; t < hi; ++t) {
      const int64_t c = (t % 2 == 0) ? t / 2 : N - 1 - t / 2;
      Li[c * N + c] = 1.0 / A[c * N + c];
      for (int64_t r = c + 1; r < N; ++r) {
        double s = 0.0;
        for (int64_t k = c; k < r; ++k) s -= A[r * N + k] * Li[k * N + c];
        Li[r * N + c] = s / A[r * N + r];
      }
    }
  }, 8);
  // A^-1 = Li^T Li: (A^-1)[a][b] = sum_{r >= max(a,b)} Li[r][a] Li[r][b]
  std::vector<double> LiT(N * N, 0.0);  // LiT[a*N + r] = Li[r][a]
  for (int64_t a = 0; a < N; ++a)
    for (int64_t r = a; r < N; ++r) LiT[a * N + r] = Li[r * N + a];
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t t = lo; t < hi; ++t) {
      const int64_t a = (t % 2 == 0) ? t / 2 : N - 1 - t / 2;
      for (int64_t b = a; b < N; ++b) {
        double s = 0.0;
        const double* pa = &LiT[a * N];
        const double* pb = &LiT[b * N];
        for (int64_t r = b; r < N; ++r) s += pa[r] * pb[r];
        A[a * N + b] = s;
        A[b * N + a] = s;
      }
    }
  }, 8);
}

void build_coarse_solver(Mesh& m, int level, CoarseSolver& cs) {
  const CellLayout L = make_layout(level);
  const int n = L.n;
  const int64_t nslot = m.nc * L.stride;
  // DoF numbering: owner copies of non-Dirichlet micro-vertices, in slot order.
  std::vector<int64_t> dof_of_slot(nslot, -1);
  std::map<std::array<int64_t, 8>, int64_t> dof_of_key;
  std::vector<std::array<int64_t, 8>> keys(nslot);
  std::vector<uint8_t> flags(nslot);
  for (int64_t s = 0; s < nslot; ++s) {
    slot_key(m, level, s, keys[s].data(), &flags[s]);
    if ((flags[s] & HT_SLOT_OWNER) && !(flags[s] & HT_SLOT_DIRICHLET)) {
      const int64_t id = (int64_t)cs.owner_slot.size();
      dof_of_key[keys[s]] = id;
      cs.owner_slot.push_back(s);
    }
  }
  const int64_t N = (int64_t)cs.owner_slot.size();
  std::vector<std::vector<int64_t>> copies(N);
  for (int64_t s = 0; s < nslot; ++s) {
    if (flags[s] & (HT_SLOT_PAD | HT_SLOT_DIRICHLET)) continue;
    const int64_t id = dof_of_key.at(keys[s]);
    dof_of_slot[s] = id;
    copies[id].push_back(s);
  }
  // blocks: the DoFs of one problem are contiguous (owner copies lie in the
  // problem's own cells, which are contiguous in slot order)
  cs.blk_dof.assign(1, 0);
  cs.row_blk.assign(N, 0);
  for (int p = 0; p < m.nprob; ++p) {
    int64_t d1 = cs.blk_dof.back();
    while (d1 < N && cs.owner_slot[d1] < m.pcell[p + 1] * L.stride) ++d1;
    for (int64_t d = cs.blk_dof.back(); d < d1; ++d) cs.row_blk[d] = p;
    cs.blk_dof.push_back(d1);
  }
  cs.blk_inv.assign(m.nprob, 0);
  int64_t inv_size = 0;
  for (int p = 0; p < m.nprob; ++p) {
    const int64_t nb = cs.blk_dof[p + 1] - cs.blk_dof[p];
    cs.blk_inv[p] = inv_size;
    inv_size += nb * nb;
  }
  cs.copy_ptr.assign(N + 1, 0);
  for (int64_t d = 0; d < N; ++d) cs.copy_ptr[d + 1] = cs.copy_ptr[d] + copies[d].size();
  cs.copy_slot.clear();
  for (auto& v : copies) cs.copy_slot.insert(cs.copy_slot.end(), v.begin(), v.end());
  // Rows: each copy contributes its cell's class-partial stencil.
  std::vector<double> A(inv_size, 0.0);
  const double scale = std::ldexp(1.0, -level);
  for (int64_t c = 0; c < m.nc; ++c) {
    for (int k = 0; k <= n; ++k)
      for (int j = 0; j <= n - k; ++j)
        for (int i = 0; i <= n - k - j; ++i) {
          const int64_t s = c * L.stride + slot_in_cell(L, i, j, k);
          const int64_t row = dof_of_slot[s];
          if (row < 0) continue;
          const int cls = point_class(n, i, j, k);
          for (int d = 0; d < 15; ++d) {
            const double w = m.cells[c].stencil_unit[cls][d] * scale;
            if (w == 0.0) continue;
            int di, dj, dk;
            stencil_offset(d, di, dj, dk);
            const int ii = i + di, jj = j + dj, kk = k + dk;
            if (ii < 0 || jj < 0 || kk < 0 || ii + jj + kk > n) continue;
            const int64_t col = dof_of_slot[c * L.stride + slot_in_cell(L, ii, jj, kk)];
            if (col < 0) continue;  // Dirichlet neighbour: not an unknown
            const int b = cs.row_blk[row];
            const int64_t d0 = cs.blk_dof[b], nb = cs.blk_dof[b + 1] - d0;
            A[cs.blk_inv[b] + (row - d0) * nb + (col - d0)] += w;
          }
        }
  }
  for (int p = 0; p < m.nprob; ++p) {
    const int64_t nb = cs.blk_dof[p + 1] - cs.blk_dof[p];
    if (nb == 0) continue;
    std::vector<double> blk(A.begin() + cs.blk_inv[p], A.begin() + cs.blk_inv[p] + nb * nb);
    cholesky_inverse(blk, nb);
    std::copy(blk.begin(), blk.end(), A.begin() + cs.blk_inv[p]);
  }
  cs.inv.swap(A);
  cs.ndof = N;
  cs.level = level;
}

Mesh::~Mesh() {}

}  // namespace ht
