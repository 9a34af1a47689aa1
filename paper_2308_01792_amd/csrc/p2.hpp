// P2 (quadratic Lagrange) operator on regularly refined cells: the stencil
// offsets of its node classes, kernel arguments and launchers.
//
// The P2 space of level l has one DoF per micro-vertex and one per micro-edge
// (the vertex subgroup and the seven edge subgroups of the paper's subgroup
// table, composed as in Section 5.1).  Those nodes are exactly the micro-
// vertices of level l + 1: a vertex (i, j, k) of level l sits at (2i, 2j, 2k)
// of the finer lattice and the midpoint of an edge at the sum of its two
// endpoints.  A P2 vector of level l is therefore stored in the closure layout
// of level l + 1, and the parity of a point's fine index names its DoF kind:
// all even is a vertex DoF, the seven other parities are the seven edge
// directions x, y, z, xy, xz, yz, xyz (index.hpp order).
//
// On a straight cell every micro-cell of one shape has the same element
// matrix, so the operator is a stencil per (parity, boundary class) of the
// fine point: the sum, over the micro-cells of level l that have the point as
// a node and lie inside the cell, of the element-matrix row of that node.
#pragma once
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include "index.hpp"

namespace ht {

enum { kP2Parities = 8, kP2MaxOffsets = 65 };
constexpr int kP2EdgeNodes[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// Fine-lattice coordinates of the ten P2 nodes (vertices, then the edges in
// kP2EdgeNodes order) of the micro-cell of shape s with base point a.
constexpr void p2_nodes(const int a[3], int s, int out[10][3]) {
  for (int q = 0; q < 4; ++q)
    for (int d = 0; d < 3; ++d) out[q][d] = 2 * (a[d] + kShapeOffsets[s][q][d]);
  for (int e = 0; e < 6; ++e)
    for (int d = 0; d < 3; ++d)
      out[4 + e][d] = 2 * a[d] + kShapeOffsets[s][kP2EdgeNodes[e][0]][d] +
                      kShapeOffsets[s][kP2EdgeNodes[e][1]][d];
}

// The micro-cells around the fine point f = (p & 1, p >> 1 & 1, p >> 2 & 1)
// of parity p: a node of the cell with base a has fine coordinates in
// 2 a + [0, 2]^3, so the bases a in [-1, 0]^3 are all candidates.
template <typename F>
constexpr void p2_for_each_cell(int p, F&& f) {
  const int fp[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
  for (int a0 = -1; a0 <= 0; ++a0)
    for (int a1 = -1; a1 <= 0; ++a1)
      for (int a2 = -1; a2 <= 0; ++a2)
        for (int s = 0; s < 6; ++s) {
          const int a[3] = {a0, a1, a2};
          int nd[10][3] = {};
          p2_nodes(a, s, nd);
          int role = -1;
          for (int q = 0; q < 10; ++q)
            if (nd[q][0] == fp[0] && nd[q][1] == fp[1] && nd[q][2] == fp[2]) role = q;
          if (role < 0) continue;
          int rel[10][3] = {};
          for (int q = 0; q < 10; ++q)
            for (int d = 0; d < 3; ++d) rel[q][d] = nd[q][d] - fp[d];
          f(s, role, rel);
        }
}

// Stencil offsets of every parity: the union of the node offsets of the
// micro-cells around a point, sorted by (dk, dj, di).
struct P2Offsets {
  int len[kP2Parities];
  signed char d[kP2Parities][kP2MaxOffsets][3];
};

constexpr P2Offsets make_p2_offsets() {
  P2Offsets t{};
  for (int p = 0; p < kP2Parities; ++p) {
    int len = 0;
    signed char (&d)[kP2MaxOffsets][3] = t.d[p];
    p2_for_each_cell(p, [&](int, int, const int (&rel)[10][3]) {
      for (int q = 0; q < 10; ++q) {
        bool seen = false;
        for (int u = 0; u < len; ++u)
          if (d[u][0] == rel[q][0] && d[u][1] == rel[q][1] && d[u][2] == rel[q][2]) seen = true;
        if (seen) continue;
        if (len < kP2MaxOffsets)
          for (int c = 0; c < 3; ++c) d[len][c] = (signed char)rel[q][c];
        ++len;
      }
    });
    for (int u = 1; u < len && len <= kP2MaxOffsets; ++u)
      for (int v = u; v > 0; --v) {
        auto key = [&](int w) { return (d[w][2] * 8 + d[w][1]) * 8 + d[w][0]; };
        if (key(v - 1) <= key(v)) break;
        for (int c = 0; c < 3; ++c) {
          const signed char tmp = d[v][c];
          d[v][c] = d[v - 1][c];
          d[v - 1][c] = tmp;
        }
      }
    t.len[p] = len;
  }
  return t;
}
inline constexpr P2Offsets kP2Off = make_p2_offsets();
static_assert(kP2Off.len[0] == 65 && kP2Off.len[1] == 27 && kP2Off.len[2] == 19 &&
                  kP2Off.len[3] == 27 && kP2Off.len[4] == 27 && kP2Off.len[5] == 19 &&
                  kP2Off.len[6] == 27 && kP2Off.len[7] == 19,
              "P2 stencil sizes of the refined lattice");

// Weights per cell: [parity 8][boundary class 16][kP2MaxOffsets], zero where
// an offset is not reached; the class bits are those of point_class() on the
// fine lattice.
enum { kP2PerCell = kP2Parities * kNumClasses * kP2MaxOffsets };

// Unit-scale P2 weights of one cell with vertex coordinates X (level l: divide
// by 2^l, the micro-cells being the unit shapes scaled by 2^-l).
void p2_cell_weights(const double X[4][3], double* w /* [kP2PerCell] */);

// Work of one cell for the bulk kernel: k-march segments (j0 | k0 << 16, i0)
// of J rows x 124 points from plane k0.  Face points of the rows
// 1 <= j <= n - k - 1 (one boundary class per plane and face): face tiles
// (k0 | side << 16, jb) of kP2FaceK planes from k0 and the kP2FaceRows rows
// from jb, on face i = 0 (side 0) or i = n - j - k (side 1).  Face points on
// the edges j = 0 and (face i = 0) j = n - k, whose class varies along the
// edge: edge runs (side << 16 | s << 17 | edge << 19, k0) of the 64 points
// k = k0 + 2 lane + s of the edge j = 0 (edge 0) or j = n - k (edge 1).
struct P2Args {
  const void* x;
  void* y;
  const void* w;          // [nc][kP2PerCell] level-scaled weights
  const int2* tiles;      // k-march segments of one cell
  int64_t ntiles, nblk;   // tiles per cell, blocks per cell
  const int2* ftiles;     // face tiles of one cell
  int64_t nftiles;
  const int2* runs;       // edge runs of one cell
  int64_t nruns, nfblk;
  int64_t nc;
  int64_t stride, off_s0, off_s1;
  int n;                  // fine intervals per macro-edge, 2^(l+1)
  int kseg;               // planes per k-march segment (a multiple of 10)
};
enum { kP2TileI = 124, kP2FaceK = 8, kP2FaceRows = 128 };

void launch_p2(int dtype, int J, const P2Args& a, hipStream_t s);

// Conversion between the lattice layout and the paper's per-cell subgroup
// arrays (subgroup table, Section 4 AoS / SoA layouts).  Subgroup g (vertex,
// x, y, z, xy, xz, yz, xyz) at index (i, j, k) of its polytope of width w_g
// (2^l + 1, 2^l six times, 2^l - 1) is the fine point 2 (i, j, k) + shift_g.
struct P2PackArgs {
  const void* lattice;    // m vectors of the fine level, comp_stride apart
  void* arrays;           // [nc][m * N_tet(2^(l+1) + 1)]
  const int4* rows;       // (g, k, j, element offset of subgroup g for m = 1)
  int64_t nrows, nc;
  int64_t stride, off_s0, off_s1;
  int64_t comp_stride, cell_elems;
  int n;                  // fine intervals per macro-edge
  int m, soa, unpack;
};
void launch_p2_pack(int dtype, const P2PackArgs& a, hipStream_t s);

}  // namespace ht
