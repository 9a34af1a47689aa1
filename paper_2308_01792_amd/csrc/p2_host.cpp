// Host side of the P2 operator: the element matrices of the six micro-cell
// shapes of a cell and the class-partial stencils built from them.
#include <cmath>
#include <cstring>

#include "p2.hpp"

namespace ht {

// P2 element matrix of one micro-cell from the products
// G[a][b] = |T| grad(lambda_a) . grad(lambda_b) (Section 5.2.1 element
// matrix; basis lambda_q (2 lambda_q - 1) at vertex q and 4 lambda_q lambda_r
// at edge (q, r)).  With the integrals of lambda_a lambda_b over T,
// |T| (1 + delta_ab) / 20, and of lambda_a, |T| / 4:
//   vertex a, vertex b: G[a][b] (4 (1 + delta_ab) / 5 - 1)
//   vertex a, edge bc:  4 (G[a][c] c_ab + G[a][b] c_ac),
//                       c_xy = (1 + delta_xy) / 5 - 1 / 4
//   edge ab, edge cd:   16 (G[b][d] m_ac + G[b][c] m_ad + G[a][d] m_bc
//                       + G[a][c] m_bd), m_xy = (1 + delta_xy) / 20
static void p2_element_matrix(const double G[4][4], double K[10][10]) {
  auto dl = [](int x, int y) { return x == y ? 1.0 : 0.0; };
  auto cc = [&](int x, int y) { return (1.0 + dl(x, y)) / 5.0 - 0.25; };
  auto mm = [&](int x, int y) { return (1.0 + dl(x, y)) / 20.0; };
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) K[a][b] = G[a][b] * (0.8 * (1.0 + dl(a, b)) - 1.0);
  for (int a = 0; a < 4; ++a)
    for (int e = 0; e < 6; ++e) {
      const int b = kP2EdgeNodes[e][0], c = kP2EdgeNodes[e][1];
      const double v = 4.0 * (G[a][c] * cc(a, b) + G[a][b] * cc(a, c));
      K[a][4 + e] = v;
      K[4 + e][a] = v;
    }
  for (int e = 0; e < 6; ++e)
    for (int f = 0; f < 6; ++f) {
      const int a = kP2EdgeNodes[e][0], b = kP2EdgeNodes[e][1];
      const int c = kP2EdgeNodes[f][0], d = kP2EdgeNodes[f][1];
      K[4 + e][4 + f] = 16.0 * (G[b][d] * mm(a, c) + G[b][c] * mm(a, d) +
                                G[a][d] * mm(b, c) + G[a][c] * mm(b, d));
    }
}

// Gradient products of shape s at unit scale (edge vectors J (o_r - o_0)).
static void shape_gradient_products(const double X[4][3], int s, double G[4][4]) {
  double Jm[3][3];  // column c = X_{c+1} - X_0
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Jm[r][c] = X[c + 1][r] - X[0][r];
  const int(*o)[3] = kShapeOffsets[s];
  double E[3][3];  // rows: physical edge vectors
  for (int r = 0; r < 3; ++r)
    for (int a = 0; a < 3; ++a) {
      double v = 0;
      for (int c = 0; c < 3; ++c) v += Jm[a][c] * (o[r + 1][c] - o[0][c]);
      E[r][a] = v;
    }
  const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                     E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                     E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  const double vol = std::fabs(det) / 6.0;
  // grad(lambda_q), q >= 1: column q - 1 of inv(E) (cofactors / det)
  double inv[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      inv[r][c] = (E[r1][c1] * E[r2][c2] - E[r1][c2] * E[r2][c1]) / det;
    }
  double g[4][3];
  for (int q = 1; q < 4; ++q)
    for (int a = 0; a < 3; ++a) g[q][a] = inv[a][q - 1];
  for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q)
      G[p][q] = vol * (g[p][0] * g[q][0] + g[p][1] * g[q][1] + g[p][2] * g[q][2]);
}

static int p2_offset_index(int p, const int d[3]) {
  for (int t = 0; t < kP2Off.len[p]; ++t)
    if (kP2Off.d[p][t][0] == d[0] && kP2Off.d[p][t][1] == d[1] && kP2Off.d[p][t][2] == d[2])
      return t;
  return -1;
}

void p2_cell_weights(const double X[4][3], double* w) {
  double K[6][10][10];
  for (int s = 0; s < 6; ++s) {
    double G[4][4];
    shape_gradient_products(X, s, G);
    p2_element_matrix(G, K[s]);
  }
  std::memset(w, 0, sizeof(double) * kP2PerCell);
  for (int p = 0; p < kP2Parities; ++p)
    p2_for_each_cell(p, [&](int s, int role, const int (&rel)[10][3]) {
      // A micro-cell around a point lies inside the cell unless it crosses
      // one of the cell faces through the point (its nodes are within one
      // coarse step of the point's micro-vertex or micro-edge).
      for (int cls = 0; cls < kNumClasses; ++cls) {
        bool inside = true;
        for (int q = 0; q < 10 && inside; ++q) {
          if ((cls & 1) && rel[q][0] < 0) inside = false;
          if ((cls & 2) && rel[q][1] < 0) inside = false;
          if ((cls & 4) && rel[q][2] < 0) inside = false;
          if ((cls & 8) && rel[q][0] + rel[q][1] + rel[q][2] > 0) inside = false;
        }
        if (!inside) continue;
        double* row = w + (p * kNumClasses + cls) * kP2MaxOffsets;
        for (int q = 0; q < 10; ++q) row[p2_offset_index(p, rel[q])] += K[s][role][q];
      }
    });
}

}  // namespace ht
