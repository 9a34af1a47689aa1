// Band stencil kernel: arguments, work items and the LDS image geometry it
// shares with the host.
//
// A work item is a band of R consecutive rows j0 .. j0 + R - 1 of one
// macro-cell, taken through the planes k0 .. k1 - 1 (Section 4: i is the
// contiguous index, rows are indexed by (j, k)).  The workgroup stages the
// planes of the band in LDS as "images": image row r holds the closure row
// j = j0 - 1 + r of plane q (r = 0 and r = R + 1 are halo rows) as its
// L_r = n - j - q + 1 points plus one zero column on each side.  Image rows
// are packed back to back, so row r starts at
//   D(r) = r (L0 + 2) - r (r - 1) / 2,   L0 = n - (j0 - 1) - q + 1,
// and a plane image holds D(min(R + 2, L0 + 1)) values.
#pragma once
#include <stdint.h>

#include <vector>

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include "index.hpp"

namespace ht {

// LDS image capacity (values per plane slot) and ring depth.
// A workgroup is kBandComputeWaves compute waves and as many load waves;
// each load lane keeps kBandDepth planes in flight.
#ifndef HT_BAND_WAVES
#define HT_BAND_WAVES 4
#endif
// kBandPad values follow the ring: lanes that output nothing may read up to
// 198 positions past a slot (at 256 intervals, the largest level whose bands
// fit; 2048-value slots), and their values are never used.
enum { kBandComputeWaves = HT_BAND_WAVES, kBandLoadLanes = 64 * HT_BAND_WAVES,
       kBandThreads = 128 * HT_BAND_WAVES, kBandSlots = 4, kBandDepth = 4,
       kBandRowsMax = 32, kBandPad = 256 };
// Values per slot (a multiple of kBandLoadLanes): four FP64 slots are 64 KB
// and leave room for two workgroups per CU.  FP32 uses the same count: its
// load lanes then hold two 16-byte vectors per plane, which keeps the
// kernel within the registers of three workgroups per CU (a larger FP32 slot
// needs a third vector per lane and measured slower at two workgroups).
#ifndef HT_BAND_CAP64
#define HT_BAND_CAP64 2048
#endif
#ifndef HT_BAND_CAP32
#define HT_BAND_CAP32 2048
#endif
template <typename T> struct BandCap;
template <> struct BandCap<double> { static constexpr int value = HT_BAND_CAP64; };
template <> struct BandCap<float> { static constexpr int value = HT_BAND_CAP32; };
inline int band_cap(int dtype_is_f64) { return dtype_is_f64 ? HT_BAND_CAP64 : HT_BAND_CAP32; }

// Planes per work item (the march length of one workgroup), and the fewest
// rows per band for which a level uses the band kernel.
#ifndef HT_BAND_PLANES
#define HT_BAND_PLANES 32
#endif
enum { kBandPlanes = HT_BAND_PLANES, kBandMinRows = 4, kBandMaxLevel = 10 };

// Start of image row r for a plane whose row 0 has L0 points.
inline constexpr int band_row_start(int r, int L0) {
  return r * (L0 + 2) - ((r * (r - 1)) >> 1);
}
// Values in the image of plane q for the band (j0, R) at n intervals.
inline int band_image_size(int n, int j0, int R, int q) {
  const int L0 = n - j0 - q + 2;
  if (L0 < 0) return 0;
  const int rows = R + 2 < L0 + 1 ? R + 2 : L0 + 1;
  return band_row_start(rows, L0);
}

// Work items of one cell at n intervals: (j0 | R << 16, k0 | k1 << 16).
// Returns false when no band fits the capacity (the level is then left to
// the tile kernel).
inline bool make_band_items(int n, int cap, int min_rows, std::vector<int2>& items) {
  items.clear();
  for (int k0 = 0; k0 <= n; k0 += kBandPlanes) {
    const int k1 = k0 + kBandPlanes < n + 1 ? k0 + kBandPlanes : n + 1;
    for (int j0 = 0; j0 <= n - k0;) {
      int R = kBandRowsMax;
      // the first plane of the item's march (k0 - 1) has the largest image
      while (R > 1 && band_image_size(n, j0, R, k0 - 1) > cap) --R;
      if (band_image_size(n, j0, R, k0 - 1) > cap || R < min_rows) return false;
      if (R > n - k0 - j0 + 1) R = n - k0 - j0 + 1;
      int2 it;
      it.x = j0 | (R << 16);
      it.y = k0 | (k1 << 16);
      items.push_back(it);
      j0 += R;
    }
  }
  return true;
}

// Geometry of plane q of the band (j0 = jm + 1, R rows, march ending at
// k1), shared by the kernel and the host tables.  The main points of image
// row r start at run position Mr(r) = r (L0 - 2) - r (r - 1) / 2 + 2
// relative to element mq of the cell block (image position U of row r holds
// element mq + U - 4 r); rows rlo .. rm - 1 have main points, which form
// the run [F0, F1).  fa is F0 rounded down so that element mq + fa starts a
// 16-byte vector of V values.
struct BandPlane {
  int L0, rows, F0, F1, fa, mq, s0b, s1b;
  bool valid, zero;  // plane inside the cell and the march; plane outside the cell
};
HT_HD BandPlane band_plane(int n, int off_s0, int off_s1, int jm, int R, int k1, int q,
                           int V) {
  BandPlane P;
  P.L0 = n - jm - q + 1;
  P.valid = q >= 0 && q <= n && q <= k1 && P.L0 >= 0;
  P.zero = (q < 0 || q > n) && q <= k1;
  P.rows = P.valid ? (R + 2 < P.L0 + 1 ? R + 2 : P.L0 + 1) : 0;
  const int rlo = jm < 0 ? 1 : 0;
  const int rm = P.rows < P.L0 - 2 ? P.rows : P.L0 - 2;
  const int L0 = P.L0;
  auto Mr = [L0](int r) { return r * (L0 - 2) - ((r * (r - 1)) >> 1) + 2; };
  P.F0 = Mr(rlo);
  P.F1 = rm > rlo ? Mr(rm) : P.F0;
  // 32-bit tetrahedral and triangular numbers (n <= 2^10 wherever bands fit)
  auto tet = [](int w) { return w <= 0 ? 0 : w * (w + 1) * (w + 2) / 6; };
  auto tri = [](int w) { return w <= 0 ? 0 : (w * (w + 1)) >> 1; };
  P.mq = P.valid ? tet(n - 1) - tet(n - 1 - q) - 2 + jm * (n - 1 - q) - ((jm * (jm - 1)) >> 1)
                 : 0;
  P.fa = P.F0 - ((P.mq + P.F0) & (V - 1));
  P.s0b = off_s0 + tri(n + 1) - tri(n + 1 - q) + jm;
  P.s1b = off_s1 + tri(n) - tri(n - q) + jm;
  return P;
}

// Main-run vectors per load lane and plane (V values each), and the bytes of
// row data per load lane and plane (NM V, rounded up to 8 or 16).
inline constexpr int band_nm(int cap, int V) {
  return (cap - 4 + V - 1 + kBandLoadLanes * V - 1) / (kBandLoadLanes * V);
}
inline constexpr int band_tb(int nv) { return nv <= 8 ? 8 : 16; }
// Planes per item in the row table: the march's planes k0 - 1 .. k0 + kBandPlanes.
enum { kBandTabPlanes = kBandPlanes + 2 };

// Row table.  Every cell of a level has the same closure layout, so the
// image row of each main-run element of each plane of each work item is a
// property of the level alone.  Byte m V + t of load lane l's TB-byte entry
// in block 1 + item kBandTabPlanes + (q - k0 + 1) is 4 r for the run element
// fa + V (l + kBandLoadLanes m) + t of plane q (r its image row, so that the
// element goes to image position f + 4 r), or 0xff where that element is
// outside [F0, F1).  Block 0 is all 0xff (planes past the march).
inline void make_band_rowtab(int level, int cap, int esize, const std::vector<int2>& items,
                             std::vector<uint8_t>& tab) {
  const CellLayout L = make_layout(level);
  const int n = L.n, V = 16 / esize, NM = band_nm(cap, V), TB = band_tb(NM * V);
  const size_t blk = (size_t)kBandLoadLanes * TB;
  tab.assign((1 + items.size() * (size_t)kBandTabPlanes) * blk, 0xff);
  for (size_t it = 0; it < items.size(); ++it) {
    const int j0 = items[it].x & 0xffff, R = items[it].x >> 16, k1 = items[it].y >> 16;
    const int k0 = items[it].y & 0xffff, jm = j0 - 1;
    for (int qr = 0; qr < kBandTabPlanes; ++qr) {
      const BandPlane P = band_plane(n, (int)L.off_s0, (int)L.off_s1, jm, R, k1, k0 - 1 + qr, V);
      if (!P.valid || P.F1 <= P.F0) continue;
      uint8_t* t = &tab[(1 + it * (size_t)kBandTabPlanes + qr) * blk];
      const int rlo = jm < 0 ? 1 : 0;
      int f = P.F0;
      for (int r = rlo; f < P.F1; ++r)
        for (int c = 2; c <= P.L0 - r - 1; ++c, ++f) {  // main points of row r
          const int i = f - P.fa, v = i / V;
          t[(size_t)(v % kBandLoadLanes) * TB + (v / kBandLoadLanes) * V + i % V] =
              (uint8_t)(4 * r);
        }
    }
  }
}

struct ClassInfo;

struct BandArgs {
  const void* x;     // operand (the iterate u of the sweeps)
  void* y;           // output (partial rows at surface points)
  const void* w;     // level-scaled class stencils [nc][16][15]
  const int2* items; // work items of one cell
  const uint8_t* rtab;  // row table of the level (make_band_rowtab)
  // Jacobi sweep and residual (OP_JACOBI, OP_RESID): right-hand side, the
  // cells' class data (inverse diagonal), one norm partial per compute wave
  // (|r|^2 of the points the wave finishes), omega and the level scale
  const void* b;
  const ClassInfo* cls;
  double* partials;
  double omega, nscale;
  // FP64 residual with FP32 outputs (OP_RESID32, OP_RESID32X): r in FP32 at
  // the finished points (y then holds the partial rows of the others), and
  // for OP_RESID32X the next correction's first Jacobi sweep omega D^-1 r
  float* y32;
  float* efirst;
  // the last sweep of an FP32 correction (OP_JACOBIADD): u += e_new in FP64
  // at the finished points (y holds the partial rows of the others)
  double* uadd;
  int64_t nitems, nblocks;
  int64_t stride, off_s0, off_s1;
  int n;
};

void launch_band(int dtype, int op, const BandArgs& a, hipStream_t s);

}  // namespace ht
