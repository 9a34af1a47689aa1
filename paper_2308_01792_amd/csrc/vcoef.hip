// Element-wise P1 operator with a space-dependent coefficient: y = A_k x,
// A_k the stiffness matrix of div(k grad) (Section 5.2.1, the operator
// catalogue's div(k grad) form).  The coefficient k is a P1 field given by
// its values at the points; its linear interpolant times the constant P1
// gradients is integrated exactly, so micro-cell T of shape t contributes
// kbar_T K_t, kbar_T the mean of k at T's four vertices and K_t the element
// matrix of shape t (one of six per macro-cell).
//
// The kernel marches like the constant-coefficient stencil kernel: one wave
// holds a (64-lane x J-row) tile, planes k-1, k, k+1 of x and of k in
// registers, i +- 1 neighbours from DPP.  Per point it forms the 14
// differences x(neighbour) - x(point) and sums the contributions of its 24
// micro-cells, grouped by the faces of the cell each one would cross; on the
// cell's surface the groups that leave the closure are dropped, which gives
// the cell's partial row for the ghost exchange.
//
// The same march also serves the stored-stencil comparison (the paper's
// grid-aware precomputation, Section 5.2.1): VC_ASSEMBLE writes each point's
// 15 row entries (partial on the surface) in the iteration order, and
// VC_STORED applies them, loading 15 weights per point instead of k.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "vcoef.hpp"

namespace ht {
namespace {

// The 24 micro-cells around a point, from the six shapes' vertex offsets:
// for shape t and role q of the point, the stencil-offset indices (index.hpp
// order) of the other three vertices, the couplings 6 t + edge of the point
// with them, and the class bits of the faces through the point that the
// micro-cell crosses (bit 0: i = 0, 1: j = 0, 2: k = 0, 3: i + j + k = n).
struct VTet {
  signed char d[3], p[3], mask;
};
constexpr VTet kVTets[24] = {
    {{1, 3, 5}, {0, 1, 2}, 8},      {{2, 7, 9}, {0, 3, 4}, 1},
    {{4, 8, 11}, {1, 3, 5}, 2},     {{6, 10, 12}, {2, 4, 5}, 4},
    {{11, 9, 5}, {6, 7, 8}, 11},    {{12, 7, 3}, {6, 9, 10}, 13},
    {{10, 8, 1}, {7, 9, 11}, 14},   {{6, 4, 2}, {8, 10, 11}, 7},
    {{7, 9, 5}, {12, 13, 14}, 9},   {{8, 11, 13}, {12, 15, 16}, 10},
    {{10, 12, 1}, {13, 15, 17}, 12}, {{6, 14, 2}, {14, 16, 17}, 5},
    {{7, 3, 5}, {18, 19, 20}, 9},   {{8, 1, 13}, {18, 21, 22}, 10},
    {{4, 2, 11}, {19, 21, 23}, 3},  {{6, 14, 12}, {20, 22, 23}, 5},
    {{11, 13, 5}, {24, 25, 26}, 10}, {{12, 1, 3}, {24, 27, 28}, 12},
    {{14, 2, 7}, {25, 27, 29}, 5},  {{6, 4, 8}, {26, 28, 29}, 6},
    {{1, 13, 5}, {30, 31, 32}, 10}, {{2, 11, 9}, {30, 33, 34}, 3},
    {{14, 12, 7}, {31, 33, 35}, 5}, {{6, 10, 8}, {32, 34, 35}, 6},
};

// The 15 stencil-offset values of row rr for this lane from the planes
// k-1, k, k+1 (rows j0-1 .. j0+J in slots 0 .. J+1), index.hpp order.
template <typename T, int J>
__device__ __forceinline__ void gather15(T (&v)[15], const T (&pm)[J + 2],
                                         const T (&pc)[J + 2],
                                         const T (&pp)[J + 2], int rr) {
  v[0] = pc[rr + 1];
  v[1] = lane_next(v[0]);
  v[2] = lane_prev(v[0]);
  v[3] = pc[rr + 2];
  v[4] = pc[rr];
  v[5] = pp[rr + 1];
  v[6] = pm[rr + 1];
  v[7] = lane_prev(pc[rr + 2]);
  v[8] = lane_next(pc[rr]);
  v[9] = lane_prev(pp[rr + 1]);
  v[10] = lane_next(pm[rr + 1]);
  v[11] = pp[rr];
  v[12] = pm[rr + 2];
  v[13] = lane_next(pp[rr]);
  v[14] = lane_prev(pm[rr + 2]);
}

}  // namespace

template <typename T, int MODE, int J>
__global__ __launch_bounds__(64 * kCellWaves) __attribute__((amdgpu_waves_per_eu(2))) void k_vcell(VCellArgs a) {
  constexpr bool LOAD_X = MODE != VC_ASSEMBLE;
  constexpr bool LOAD_K = MODE != VC_STORED;
  __shared__ T ctab[kVcoefPerCell];
  // block -> (cell, tile group) in the stencil kernel's XCD-aware order
  const int64_t nb = a.nblocks;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t wb = (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
  if (wb >= nb) return;
  const int64_t cell = wb / a.ntiles;
  const int2 tile = a.tiles[wb % a.ntiles];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // tile (i0, j0 | k0 << 16): the march covers planes k0 .. k0 + kseg - 1
  const int i0 = tile.x, j0 = (tile.y & 0xffff) + wave * J, k0 = tile.y >> 16;
  const int n = a.n;
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t rk = make_rsrc((const T*)a.kappa + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  // stored rows: 15 blocks of the cell's closure, entry d of slot s at
  // d * stride + s
  const __amdgpu_buffer_rsrc_t rw =
      make_rsrc((T*)a.w + cell * 15 * a.stride, 15 * bytes);
  const unsigned wstep = (unsigned)(a.stride * (int64_t)sizeof(T));
  if (LOAD_K) {
    if (threadIdx.x < kVcoefPerCell)
      ctab[threadIdx.x] = ((const T*)a.kc)[cell * kVcoefPerCell + threadIdx.x];
    __syncthreads();
  }

  const int i = i0 - 1 + lane;
  const bool is0 = (i == 0);
  const unsigned out_mask = (lane >= 1 && lane <= 62) ? 0u : HT_OOB;
  // Scalar cursor over the planes (closure layout of index.hpp): element
  // bases of plane ck in the main block (minus one), in S0 and in S1.
  const int wm = n - 1;
  // (started at plane k0 - 1 from the closed forms of the plane sizes; for
  // k0 = 0 the plane -1 yields no offset and its advance lands on plane 0)
  int ck = k0 - 1;
  int cmb = -1 + tet32(wm) - tet32(wm - ck),
      csa = (int)a.off_s0 + tri32(n + 1) - tri32(n + 1 - ck),
      csb = (int)a.off_s1 + tri32(n) - tri32(n - ck);
  // Byte offsets of this lane's point in rows j0-1 .. j0+J of plane ck
  // (HT_OOB outside the closure), then move the cursor to the next plane.
  auto plane_offsets = [&](unsigned (&o)[J + 2]) {
    const int kk = ck, wk = wm - kk;
    const int jf = j0 - 1, js = jf > 0 ? jf : 0;
    int mb = cmb + js * wk - js * (js - 1) / 2;
    int sa = csa + js, sb = csb + js;
#pragma unroll
    for (int r = 0; r < J + 2; ++r) {
      const int j = jf + r;
      const int e = n - j - kk;
      const bool row_ok = j >= 0 && e >= 0 && kk >= 0;
      int el = (i == e) ? sb : mb + i;
      el = is0 ? sa : el;
      o[r] = (row_ok && (unsigned)i <= (unsigned)e) ? (unsigned)el * (unsigned)sizeof(T)
                                                    : HT_OOB;
      const bool inc = j >= 0;
      mb += inc ? wk - j : 0;
      sa += inc ? 1 : 0;
      sb += inc ? 1 : 0;
    }
    cmb += wk > 0 ? wk * (wk + 1) / 2 : 0;
    csa += n + 1 - ck;
    csb += n - ck;
    ++ck;
  };

  // Plane k from x planes (pm, pc, pp) and coefficient planes (qm, qc, qp)
  // while the loads of plane k+2 go into (pn, qn); VC_STORED holds the rows
  // of plane k in wc and loads those of plane k+1 (offsets op) into wp.
  auto step = [&](int k, T (&pm)[J + 2], T (&pc)[J + 2], T (&pp)[J + 2],
                  T (&pn)[J + 2], T (&qm)[J + 2], T (&qc)[J + 2],
                  T (&qp)[J + 2], T (&qn)[J + 2], unsigned (&oc)[J + 2],
                  unsigned (&op)[J + 2], unsigned (&on)[J + 2],
                  T (&wc)[J][15], T (&wp)[J][15]) {
    plane_offsets(on);
#pragma unroll
    for (int r = 0; r < J + 2; ++r) {
      if (LOAD_X) bload(pn[r], rx, on[r]);
      if (LOAD_K) bload(qn[r], rk, on[r]);
    }
    if (MODE == VC_STORED) {
#pragma unroll
      for (int r = 0; r < J; ++r)
#pragma unroll
        for (int d = 0; d < 15; ++d) bload(wp[r][d], rw, op[r + 1] + (unsigned)d * wstep);
    }
#pragma unroll
    for (int rr = 0; rr < J; ++rr) {
      const int j = j0 + rr;
      const int e = n - j - k;
      if (e < i0) continue;
      const unsigned so = oc[rr + 1] | out_mask;
      if (MODE == VC_STORED) {
        T u[15];
        gather15<T, J>(u, pm, pc, pp, rr);
        T acc = wc[rr][0] * u[0];
#pragma unroll
        for (int d = 1; d < 15; ++d) acc = fma(wc[rr][d], u[d], acc);
        bstore(acc, ry, so);
        continue;
      }
      T q[15];
      gather15<T, J>(q, qm, qc, qp, rr);
      // drop the micro-cells that leave the closure through a face the
      // point lies on
      const int cls = (int)is0 | ((j == 0) << 1) | ((k == 0) << 2) | ((i == e) << 3);
      if (MODE == VC_ASSEMBLE) {
        // row entries: sum over the kept micro-cells of kbar K[q][r] at the
        // offset of vertex r, minus their sum at the centre
        T wd[15];
#pragma unroll
        for (int d = 0; d < 15; ++d) wd[d] = (T)0;
#pragma unroll
        for (int t = 0; t < 24; ++t) {
          const VTet& v = kVTets[t];
          const T ks = (q[0] + q[v.d[0]]) + (q[v.d[1]] + q[v.d[2]]);
          const T f = (cls & v.mask) ? (T)0 : ks;
#pragma unroll
          for (int r = 0; r < 3; ++r) wd[v.d[r]] = fma(f, ctab[v.p[r]], wd[v.d[r]]);
        }
        T centre = (T)0;
#pragma unroll
        for (int d = 1; d < 15; ++d) centre -= wd[d];
        wd[0] = centre;
#pragma unroll
        for (int d = 0; d < 15; ++d)
          bstore(wd[d], rw, so < HT_OOB ? so + (unsigned)d * wstep : HT_OOB);
        continue;
      }
      T u[15];
      gather15<T, J>(u, pm, pc, pp, rr);
      T du[15];
#pragma unroll
      for (int d = 1; d < 15; ++d) du[d] = u[d] - u[0];
      T g[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) g[m] = (T)0;
#pragma unroll
      for (int t = 0; t < 24; ++t) {
        const VTet& v = kVTets[t];
        T rho = ctab[v.p[0]] * du[v.d[0]];
        rho = fma(ctab[v.p[1]], du[v.d[1]], rho);
        rho = fma(ctab[v.p[2]], du[v.d[2]], rho);
        const T ks = (q[0] + q[v.d[0]]) + (q[v.d[1]] + q[v.d[2]]);
        g[v.mask] = fma(ks, rho, g[v.mask]);
      }
      T acc = (T)0;
#pragma unroll
      for (int m = 1; m < 15; ++m) acc += (cls & m) ? (T)0 : g[m];
      bstore(acc, ry, so);
    }
  };

  T PA[J + 2], PB[J + 2], PC[J + 2], PD[J + 2];
  T QA[J + 2], QB[J + 2], QC[J + 2], QD[J + 2];
  unsigned OA[J + 2], OB[J + 2], OC[J + 2], OD[J + 2];
  T WA[J][15], WB[J][15];
  // planes k0 - 1 (all offsets out of range below the cell), k0, k0 + 1
  plane_offsets(OA);
#pragma unroll
  for (int r = 0; r < J + 2; ++r) {
    PA[r] = (T)0;
    QA[r] = (T)0;
    if (LOAD_X) bload(PA[r], rx, OA[r]);
    if (LOAD_K) bload(QA[r], rk, OA[r]);
  }
  plane_offsets(OB);
  plane_offsets(OC);
#pragma unroll
  for (int r = 0; r < J + 2; ++r) {
    if (LOAD_X) {
      bload(PB[r], rx, OB[r]);
      bload(PC[r], rx, OC[r]);
    }
    if (LOAD_K) {
      bload(QB[r], rk, OB[r]);
      bload(QC[r], rk, OC[r]);
    }
  }
  if (MODE == VC_STORED) {
#pragma unroll
    for (int r = 0; r < J; ++r)
#pragma unroll
      for (int d = 0; d < 15; ++d) bload(WA[r][d], rw, OB[r + 1] + (unsigned)d * wstep);
  }
  const int kcol = n - i0 - j0;
  const int kmax = kcol < k0 + a.kseg - 1 ? kcol : k0 + a.kseg - 1;
  for (int k = k0; k <= kmax; k += 4) {
    step(k, PA, PB, PC, PD, QA, QB, QC, QD, OB, OC, OD, WA, WB);
    if (k + 1 > kmax) break;
    step(k + 1, PB, PC, PD, PA, QB, QC, QD, QA, OC, OD, OA, WB, WA);
    if (k + 2 > kmax) break;
    step(k + 2, PC, PD, PA, PB, QC, QD, QA, QB, OD, OA, OB, WA, WB);
    if (k + 3 > kmax) break;
    step(k + 3, PD, PA, PB, PC, QD, QA, QB, QC, OA, OB, OC, WB, WA);
  }
}

template <typename T, int MODE>
static void launch_vcell_t(int J, const VCellArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(((a.nblocks + 7) / 8) * 8)), block(64 * kCellWaves);
  switch (J) {
    case 2: hipLaunchKernelGGL((k_vcell<T, MODE, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_vcell<T, MODE, 4>), grid, block, 0, s, a); break;
    default: throw Error{HT_ERR_ARG, "variable-coefficient tile rows must be 2 or 4"};
  }
}

template <typename T>
static void launch_vcell_mode(int mode, int J, const VCellArgs& a, hipStream_t s) {
  switch (mode) {
    case VC_APPLY: launch_vcell_t<T, VC_APPLY>(J, a, s); break;
    case VC_ASSEMBLE: launch_vcell_t<T, VC_ASSEMBLE>(J, a, s); break;
    case VC_STORED: launch_vcell_t<T, VC_STORED>(J, a, s); break;
    default: throw Error{HT_ERR_ARG, "unknown variable-coefficient kernel mode"};
  }
}

void launch_vcell(int dtype, int mode, int J, const VCellArgs& a, hipStream_t s) {
  if (a.nblocks <= 0) return;
  if ((mode == VC_APPLY || mode == VC_ASSEMBLE) && (!a.kappa || !a.kc))
    throw Error{HT_ERR_ARG, "div(k grad) kernel needs k and the couplings"};
  if ((mode == VC_ASSEMBLE || mode == VC_STORED) && !a.w)
    throw Error{HT_ERR_ARG, "stored-stencil kernel needs the row array"};
  if (dtype == HT_F64) launch_vcell_mode<double>(mode, J, a, s);
  else launch_vcell_mode<float>(mode, J, a, s);
}

}  // namespace ht
