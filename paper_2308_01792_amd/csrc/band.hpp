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

namespace ht {

// LDS image capacity (values per plane slot) and ring depth.
// A workgroup is kBandComputeWaves compute waves and as many load waves;
// each load lane keeps kBandDepth planes in flight.
#ifndef HT_BAND_WAVES
#define HT_BAND_WAVES 4
#endif
enum { kBandComputeWaves = HT_BAND_WAVES, kBandLoadLanes = 64 * HT_BAND_WAVES,
       kBandThreads = 128 * HT_BAND_WAVES, kBandSlots = 4, kBandDepth = 4,
       kBandRowsMax = 32 };
// Values per slot (a multiple of kBandLoadLanes): four FP64 slots are 64 KB
// and leave room for two workgroups per CU.
#ifndef HT_BAND_CAP64
#define HT_BAND_CAP64 2048
#endif
#ifndef HT_BAND_CAP32
#define HT_BAND_CAP32 3072
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

struct BandArgs {
  const void* x;     // operand
  void* y;           // output (partial rows at surface points)
  const void* w;     // level-scaled class stencils [nc][16][15]
  const int2* items; // work items of one cell
  int64_t nitems, nblocks;
  int64_t stride, off_s0, off_s1;
  int n;
};

void launch_band(int dtype, int op, const BandArgs& a, hipStream_t s);

}  // namespace ht
