// Kernel argument blocks and launchers shared by kernels.hip and abi.cpp.
#pragma once
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include "hytet_impl.hpp"

namespace ht {

// OP_RESID32: FP64 residual delivered in FP32 (iterative refinement): the
// cell kernel writes finished points straight to y32 and FP64 partial rows
// of surface points to y; the exchange completes those in FP64 and writes
// y32.
// OP_CHEB: one step of the Chebyshev iteration on D^-1 A:
// d <- c1 d + c2 D^-1 (b - A x) (in place), y = x + d.
// OP_RESID32X: OP_RESID32 plus the first zero-guess Jacobi sweep
// omega D^-1 r of the next FP32 correction (efirst), so that iterative
// refinement needs no separate pass for that sweep.
// OP_JACOBIADD: the last Jacobi sweep of an FP32 correction e, whose result
// is not stored but added to the FP64 iterate (u += e_new at every slot), so
// that iterative refinement needs no separate update pass (band kernel,
// FP32 only).
enum { OP_APPLY = 0, OP_RESID = 1, OP_JACOBI = 2, OP_SYNC = 3, OP_FILL = 4,
       OP_RESTRICT = 5, OP_RESID32 = 6, OP_CHEB = 7, OP_RESID32X = 8,
       OP_JACOBIADD = 9 };
enum { EOP_ZERO_GUESS = 0, EOP_MASS = 1, EOP_ZERO_INTERIOR = 2, EOP_DOT = 3,
       EOP_FLAGS = 4, EOP_COORDS = 5, EOP_PROBE = 6 };
enum { FOP_COPY = 0, FOP_ADD = 1, FOP_ZERO = 2 };
enum { kMaxInc = 128 };  // incident cells per shared primitive (checked)
// Waves per stencil-kernel workgroup, stacked in j on one cell: a group
// covers kCellWaves x J rows and loads 2 halo rows for all of them.
#ifndef HT_CELL_WAVES
#define HT_CELL_WAVES 4
#endif
enum { kCellWaves = HT_CELL_WAVES };
// The "sweep" operations stream b besides x (residual, Jacobi, FP32
// residual, Chebyshev step); their tile shape is chosen separately from the
// apply's.
constexpr bool op_is_sweep(int op) {
  return op == OP_RESID || op == OP_JACOBI || op == OP_RESID32 || op == OP_CHEB ||
         op == OP_RESID32X || op == OP_JACOBIADD;
}

struct CellArgs {
  const void* x;        // operand (u for residual / Jacobi)
  void* y;              // output
  void* y32;            // FP32 residual (OP_RESID32, OP_RESID32X)
  void* efirst;         // OP_RESID32X: omega D^-1 r in FP32
  void* d;              // Chebyshev direction (OP_CHEB), updated in place
  double c1, c2;        // Chebyshev step coefficients
  const void* b;        // right-hand side (residual / Jacobi)
  const void* w;        // level-scaled class stencils [nc][16][15]
  const ClassInfo* cls; // [nc][16]
  double* partials;     // per-block norm partials (residual)
  const int2* tiles;    // (i0, j0) of the non-empty tiles of one cell
  int64_t ntiles, nblocks;
  int64_t stride, off_s0, off_s1;
  int n;
  // wave arrangement of a workgroup: 0 = stacked in j (rows j0 .. j0 +
  // kCellWaves J - 1), 1 = side by side in i (62 kCellWaves points of J rows)
  int waves_in_i;
  int kseg;             // planes per march segment of a tile (tiles carry k0)
  double omega, nscale; // nscale = 2^l (inverse diagonal scale)
  // restriction output (coarse level layout)
  int64_t stride_out, off_s0_out, off_s1_out;
};

struct ExchArgs {
  void* y;
  void* y32;            // FP32 residual (OP_RESID32, OP_RESID32X)
  void* efirst;         // OP_RESID32X: omega D^-1 r in FP32
  double* uadd;         // OP_JACOBIADD: FP64 iterate that receives the sweep
  void* d;              // Chebyshev direction (OP_CHEB)
  double c1, c2;
  const void* u;
  const void* b;
  const DevPrim* prim;
  const DevInc* inc;
  double* partials;
  int64_t stride, off_s0, off_s1;
  int n;
  int64_t n_faces, n_edges;             // faces and edges of the range
  int64_t prim_f0, prim_e0, prim_v0;    // primitive index of the range's
                                        // first face, edge and vertex
  int64_t face_pts, face_end, edge_end, total;  // points: total = all shared
  // blocks of 256 threads: bpf per face (face interiors first, kExchFacePts
  // points per thread), bpe per edge, then the vertices; nblocks in all (one
  // norm partial per block)
  int64_t bpf, bpe, fblk, eblk, nverts, nblocks;
  double omega, nscale, fill;
};

struct XferArgs {
  const void* src;
  void* dst;
  const ClassInfo* cls;
  const int2* tiles;    // walk tiles (64 x 8) of the walked level
  int64_t ntiles, nblocks;
  int64_t ncells;
  int nf, nc_;          // fine and coarse n
  int64_t stride_f, off_s0_f, off_s1_f;
  int64_t stride_c, off_s0_c, off_s1_c;
};

// Planes per walk tile of the transfer and elementwise kernels (even, so that
// the prolongation's plane pairs start on an even plane).
enum { kWalkSeg = 16 };
// Face points per thread of the exchange.
enum { kExchFacePts = 4 };

struct ElemArgs {
  void* out;
  const void* in0;
  const void* in1;
  const ClassInfo* cls;
  const int2* tiles;    // walk tiles (64 x 8)
  int64_t ntiles, nblocks;
  double* partials;
  const double* cell_xyz;
  const int8_t* cell_order;
  int64_t ncells;
  int n;
  int64_t stride, off_s0, off_s1;
  double alpha, nscale;
};

struct FlatArgs {
  void* out;
  const void* in;
  int64_t count;
};

struct CoarseArgs {
  const void* b;
  void* u;
  const double* inv;
  const int64_t* owner;
  const int64_t* copy_ptr;
  const int64_t* copy_slot;
  const int64_t* blk_dof;  // DoF range of each diagonal block
  const int64_t* blk_inv;  // offset of each block's inverse in inv
  const int32_t* row_blk;  // block of each DoF
  double* rhs;
  int64_t ndof;
};

// Per-segment sums of norm partials: out[s] = sum of p[lo[s] .. hi[s]).
struct SegArgs {
  const double* p;
  const int64_t* lo;
  const int64_t* hi;
  double* out;
  int nseg;
};

void launch_cell(int dtype, int op, int J, const CellArgs& a, hipStream_t s);
void launch_exchange(int dtype, int op, const ExchArgs& a, hipStream_t s);
void launch_prolong(int dtype, const XferArgs& a, hipStream_t s);
void launch_elem(int dtype, int eop, const ElemArgs& a, hipStream_t s);
void launch_flat(int dto, int dti, int fop, const FlatArgs& a, hipStream_t s);
void launch_sum_partials(const double* p, int64_t count, double* out, bool sq,
                         hipStream_t s);
void launch_coarse(int dtype, const CoarseArgs& a, hipStream_t s);
void launch_seg_sum(const SegArgs& a, hipStream_t s);
void launch_lane_selftest(int* out, hipStream_t s);

}  // namespace ht
