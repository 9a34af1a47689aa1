// Index functions of the refined macro-cell (host and device).
//
// Micro-vertices of a macro-cell refined to level l (n = 2^l) are the points
// (i, j, k) of the tetrahedral index polytope I_tet(n+1) = {i + j + k <= n}
// (Section 3.2, micro-vertex subgroup of width 2^l + 1).  Its cardinality is
// N_tet(w) = w(w+1)(w+2)/6 and the paper's linearisation
//   t_w(i,j,k) = N_tet(w) - N_tet(w-k) + N_tri(w-k) - N_tri(w-k-j) + i
// makes i the contiguous index (Section 4, eq. for t_w).
//
// Closure layout used for every per-cell array of this library.  The closure
// of a cell is split in three blocks so that all four macro-faces of the cell
// are stored contiguously (the ghost exchange between cells then reads and
// writes whole runs instead of one element per i-line):
//   M  : points with 1 <= i and i + j + k <= n - 1, at t_{n-1}(i-1, j, k)
//        (the i-lines without their first and last point);
//   S0 : points with i == 0, at t2_{n+1}(j, k)           (face i = 0);
//   S1 : points with i == n - j - k, j + k <= n - 1, at t2_n(j, k)
//        (slanted face, without the points already in S0).
// t2_w(j, k) = N_tri(w) - N_tri(w-k) + j is the restriction of t_w to the
// plane i = 0 (Section 3: the 2-D case is the restriction to a plane).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define HT_HD __host__ __device__ __forceinline__
#else
#define HT_HD inline
#endif

namespace ht {

HT_HD int64_t n_tet(int64_t w) { return w <= 0 ? 0 : w * (w + 1) * (w + 2) / 6; }
HT_HD int64_t n_tri(int64_t w) { return w <= 0 ? 0 : w * (w + 1) / 2; }

// Paper's linearisation of I_tet(w).
HT_HD int64_t t_w(int64_t w, int64_t i, int64_t j, int64_t k) {
  return n_tet(w) - n_tet(w - k) + n_tri(w - k) - n_tri(w - k - j) + i;
}
// 2-D version on I_tri(w): rows k, contiguous j.
HT_HD int64_t t2_w(int64_t w, int64_t j, int64_t k) {
  return n_tri(w) - n_tri(w - k) + j;
}

// Sizes and offsets of the closure blocks of one cell at n = 2^level.
struct CellLayout {
  int32_t n;         // intervals per macro-edge
  int64_t m_size;    // N_tet(n-1)
  int64_t s0_size;   // N_tri(n+1)
  int64_t s1_size;   // N_tri(n)
  int64_t off_s0;    // start of S0 inside a cell block
  int64_t off_s1;    // start of S1
  int64_t stride;    // elements per cell block (multiple of 64)
};

HT_HD int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

inline CellLayout make_layout(int level) {
  CellLayout L;
  L.n = 1 << level;
  L.m_size = n_tet(L.n - 1);
  L.s0_size = n_tri(L.n + 1);
  L.s1_size = n_tri(L.n);
  L.off_s0 = round_up(L.m_size, 16);
  L.off_s1 = L.off_s0 + round_up(L.s0_size, 16);
  L.stride = round_up(L.off_s1 + L.s1_size, 64);
  return L;
}

// Offset of closure point (i, j, k), i + j + k <= n, inside its cell block.
HT_HD int64_t slot_in_cell(const CellLayout& L, int i, int j, int k) {
  const int n = L.n;
  if (i == 0) return L.off_s0 + t2_w(n + 1, j, k);
  if (i + j + k == n) return L.off_s1 + t2_w(n, j, k);
  return t_w(n - 1, i - 1, j, k);
}

// Boundary class of a closure point: bit 0 -> i == 0, bit 1 -> j == 0,
// bit 2 -> k == 0, bit 3 -> i + j + k == n.  Bit b set means the point lies
// on the cell face opposite local vertex face_vertex[b].
HT_HD int point_class(int n, int i, int j, int k) {
  return (i == 0) | ((j == 0) << 1) | ((k == 0) << 2) | ((i + j + k == n) << 3);
}
// Local vertex whose barycentric weight vanishes on the face of class bit b.
HT_HD int face_vertex(int b) { return b == 3 ? 0 : b + 1; }

// The 15 stencil offsets: centre, then the seven edge directions of the
// refined cell and their negatives, interleaved (+d, -d).
//   x = (1,0,0), y = (0,1,0), z = (0,0,1), xy = (-1,1,0), xz = (-1,0,1),
//   yz = (0,-1,1), xyz = (1,-1,1)
// xyz is the inner diagonal v02 -> v13 chosen by the child order of eq. (bey).
HT_HD void stencil_offset(int d, int& di, int& dj, int& dk) {
  const signed char tab[15][3] = {
      {0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
      {0, 0, 1},  {0, 0, -1},  {-1, 1, 0},  {1, -1, 0}, {-1, 0, 1},
      {1, 0, -1}, {0, -1, 1},  {0, 1, -1},  {1, -1, 1}, {-1, 1, -1}};
  di = tab[d][0]; dj = tab[d][1]; dk = tab[d][2];
}
enum { kNumOffsets = 15, kNumClasses = 16 };

// Micro-cell shapes of a regularly refined cell.  Recursive application of
// eq. (bey) produces, on every level, translated copies of six shapes; below,
// each is given by the index offsets of its four vertices (in the vertex order
// of the eq. (bey) children) from its base point b.  Valid bases are
// b >= 0 with |b| <= n-1 (first), n-3 (second) and n-2 (the other four),
// i.e. polytope widths 2^l, 2^l-2 and 2^l-1 of the paper's cell subgroups.
constexpr int kShapeOffsets[6][4][3] = {
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}},
    {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, 0, 1}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}},
    {{0, 1, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}},
};

}  // namespace ht
