// Variable-coefficient operator div(k grad) (element-wise P1 form): kernel
// arguments and launcher shared by vcoef.hip and abi.cpp.
#pragma once
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include "hytet_impl.hpp"

namespace ht {

struct VCellArgs {
  const void* x;        // operand
  const void* kappa;    // coefficient values at the points (consistent copies)
  void* y;              // output: full rows inside, partial rows on the surface
  const void* kc;       // [nc][36] level-scaled couplings (6 shapes x 6 edges)
  void* w;              // stored rows [nc][15][stride] (assemble / stored apply)
  const int2* tiles;    // (i0, j0 | k0 << 16) march segments of one cell
  int64_t ntiles, nblocks;
  int64_t stride, off_s0, off_s1;
  int n;
  int kseg;             // planes per march segment (a multiple of 4)
};

// Couplings per cell: shape t, edge p (vertex pairs 01 02 03 12 13 23).
enum { kVcoefShapes = 6, kVcoefPerCell = 36 };

// VC_APPLY: y = A_k x matrix-free; VC_ASSEMBLE: write the 15 row entries of
// A_k per point into w (x unused); VC_STORED: y = A x with the rows in w.
enum { VC_APPLY = 0, VC_ASSEMBLE = 1, VC_STORED = 2 };

void launch_vcell(int dtype, int mode, int J, const VCellArgs& a, hipStream_t s);

}  // namespace ht
