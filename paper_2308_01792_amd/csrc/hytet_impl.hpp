// Internal data structures of the hytet library (host side + device mirrors).
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <thread>
#include <memory>
#include <string>
#include <vector>

#include "hytet.h"
#include "index.hpp"

namespace ht {

// Run f(begin, end) over [0, n) on up to 16 host threads (static chunks).
inline void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f,
                         int64_t min_chunk = 1024) {
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 2 * min_chunk || nt == 1) { f(0, n); return; }
  nt = (int)std::min<int64_t>(nt, n / min_chunk);
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back(f, a, b);
  }
  for (auto& x : th) x.join();
}

// ------------------------------------------------------------ errors ----
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
#define HT_CHECK_HIP(expr)                                                  \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      throw ::ht::Error{HT_ERR_HIP, std::string(#expr) + ": " +             \
                                        hipGetErrorString(e_)};             \
  } while (0)

// ------------------------------------------------- macro primitives ----
// Incidence of a shared primitive (face, edge or vertex) on a macro-cell.
// lv[m] is the local index (0..3) in the cell of the primitive's m-th vertex,
// the primitive's vertices being sorted by ascending global id.
struct Incidence {
  int32_t cell;
  int8_t lv[3];
  int8_t cls;  // boundary class of the primitive's interior points in the cell
};

struct Prim {
  int dim;                    // 2 face, 1 edge, 0 vertex
  std::array<int64_t, 3> gv;  // ascending global vertex ids (dim + 1 used)
  bool boundary = false;      // lies on the domain boundary (Dirichlet)
  std::vector<Incidence> inc; // sorted by cell id; inc[0].cell owns it
  double diag_unit = 0.0;     // full stencil centre at unit scale
  double mass_unit = 0.0;     // full lumped mass at unit scale
};

// Per (cell, class) record; class 0 is the cell interior.
enum : uint8_t { kClsOwner = 1, kClsDirichlet = 2, kClsValid = 4 };
struct ClassInfo {
  double inv_diag_unit;  // 1 / full diagonal at unit scale (0 if Dirichlet)
  double mass_unit;      // full lumped mass at unit scale
  int32_t prim;          // shared primitive id, -1 for the cell interior
  uint8_t flags;
  uint8_t pad[3];
};

struct Cell {
  std::array<int64_t, 4> gv;        // global vertex ids in local order
  std::array<int32_t, 16> cls_prim; // primitive of every class (-1: interior)
  double stencil_unit[16][15];      // class partial stencils, unit scale
  double mass_unit[16];             // partial lumped masses, unit scale
  double shape_k[6][6];             // element-matrix couplings of the six
                                    // micro-cell shapes (vertex pairs 01 02
                                    // 03 12 13 23), unit scale
  double volume;
};

// Per level, per dtype workspace for the solvers.
struct LevelWork {
  void* u = nullptr;    // correction / iterate on coarse levels
  void* b = nullptr;    // right-hand side on coarse levels
  void* t = nullptr;    // Jacobi ping-pong and residual
  void* d = nullptr;    // Chebyshev direction (allocated when used)
};

// Exact coarse-level solver: A_II^-1 as dense blocks, one per independent
// problem of the mesh (a plain mesh is one problem, one block).
struct CoarseSolver {
  int level = -1;
  int64_t ndof = 0;
  std::vector<int64_t> owner_slot;     // slot of the owning copy per DoF
  std::vector<int64_t> copy_ptr;       // CSR over all copies of each DoF
  std::vector<int64_t> copy_slot;
  std::vector<int64_t> blk_dof;        // DoF range of block b: [blk_dof[b], blk_dof[b+1])
  std::vector<int64_t> blk_inv;        // start of block b's inverse in inv
  std::vector<int32_t> row_blk;        // block of every DoF
  std::vector<double> inv;             // dense inverse blocks, row-major
  double* d_inv = nullptr;
  int64_t* d_owner = nullptr;
  int64_t* d_copy_ptr = nullptr;
  int64_t* d_copy_slot = nullptr;
  int64_t* d_blk_dof = nullptr;
  int64_t* d_blk_inv = nullptr;
  int32_t* d_row_blk = nullptr;
  double* d_rhs = nullptr;             // gathered right-hand side
};

// A contiguous run of independent problems of a mesh: its cells [c0, c1)
// and its faces, edges and vertices (indices within each kind).
struct Range {
  int64_t c0, c1, f0, f1, e0, e1, v0, v1;
  bool empty() const { return c1 <= c0; }
};

struct DevPrim {
  int32_t inc_begin;
  int16_t inc_count;
  int8_t dim;
  uint8_t boundary;
  double inv_diag_unit;
};
struct DevInc {
  int32_t cell;
  int8_t lv[3];
  int8_t cls;
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
};

struct Mesh {
  // ---- host description
  int64_t nv = 0, nc = 0;
  int min_level = 0, max_level = 0;
  std::vector<double> xyz;                // [nv][3]
  std::vector<Cell> cells;
  std::vector<Prim> prims;                // faces, then edges, then vertices
  int64_t n_faces = 0, n_edges = 0, n_verts = 0;
  std::vector<ClassInfo> cls;             // [nc][16]
  // Independent problems (disjoint unions of meshes, see ht_batch): problem
  // p owns cells [pcell[p], pcell[p+1]) and likewise faces, edges, vertices.
  // act_cells[l]: cells of the problems present on level l, a prefix of the
  // cell list (problems are sorted by finest level, descending).
  int nprob = 1;
  std::vector<int64_t> pcell, pface, pedge, pvert;
  std::vector<int64_t> act_cells;         // per level

  // ---- device mirrors (created on first device call)
  bool uploaded = false;
  int device = -1;
  ClassInfo* d_cls = nullptr;
  DevPrim* d_prim = nullptr;
  DevInc* d_inc = nullptr;
  double* d_cell_xyz = nullptr;           // [nc][4][3] sorted by global id
  int8_t* d_cell_order = nullptr;         // [nc][4] local index in id order
  std::vector<double*> d_w64;             // per level [nc][16][15]
  std::vector<float*> d_w32;
  std::vector<double*> d_kc64;            // per level [nc][36] div(k grad)
  std::vector<float*> d_kc32;             // couplings / (4 n), on first use
  std::vector<double*> d_p2w64;           // per P2 level [nc][kP2PerCell]
  std::vector<float*> d_p2w32;            // level-scaled P2 stencils, on first use
  std::vector<double> p2_unit;            // [nc][kP2PerCell] unit scale (host)
  double* d_partials = nullptr;           // norm partial sums
  int64_t partials_cap = 0;
  double* d_scalar = nullptr;             // reduced scalars
  double* h_scalar = nullptr;             // pinned host copy
  hipStream_t capture_stream = nullptr;

  std::vector<LevelWork> work64, work32;  // per level
  std::map<int, CoarseSolver> coarse;     // per coarse level
  std::map<std::string, GraphEntry> graphs;

  // ---- profiling
  bool profiling = false;
  struct ProfEvent { std::string name; hipEvent_t a, b; };
  std::vector<ProfEvent> prof;

  ~Mesh();
};

// ------------------------------------------------------- host setup ----
void build_mesh(Mesh& m, const double* xyz, int64_t nv, const int64_t* cells,
                int64_t nc, int min_level, int max_level);
void slot_key(const Mesh& m, int level, int64_t slot, int64_t key[8],
              uint8_t* flags);
void slot_coords(const Mesh& m, int level, int64_t slot, double out[3]);
void build_coarse_solver(Mesh& m, int level, CoarseSolver& cs);
void set_problems(Mesh& m, const std::vector<int64_t>& cell_begin,
                  const std::vector<int>& finest_level);
Range problem_range(const Mesh& m, int p0, int p1);
inline Range full_range(const Mesh& m) { return problem_range(m, 0, m.nprob); }
void level_scaled_stencils(const Mesh& m, int level, std::vector<double>& w);

// ------------------------------------------------------ device side ----
void ensure_uploaded(Mesh& m);
int64_t level_slots(const Mesh& m, int level);

}  // namespace ht
