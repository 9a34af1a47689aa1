// Device helpers shared by the kernel sources: 32-bit closure index
// arithmetic, DPP lane shifts, wave reductions and raw buffer access.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ht {

// 32-bit index arithmetic for device code.  A cell block holds fewer than
// 2^31 elements up to level 10 (w (w+1) (w+2) <= 1025 * 1026 * 1027 <
// 2^31), so the tetrahedral and triangular numbers of index.hpp are formed
// without 64-bit multiplies and divisions.
__device__ __forceinline__ int tet32(int w) { return w <= 0 ? 0 : w * (w + 1) * (w + 2) / 6; }
__device__ __forceinline__ int tri32(int w) { return w <= 0 ? 0 : w * (w + 1) / 2; }
__device__ __forceinline__ int tw32(int w, int i, int j, int k) {
  return tet32(w) - tet32(w - k) + tri32(w - k) - tri32(w - k - j) + i;
}
__device__ __forceinline__ int t2w32(int w, int j, int k) {
  return tri32(w) - tri32(w - k) + j;
}

// ------------------------------------------------------- lane exchange --
// DPP wave shifts (GFX9 family): wave_shr:1 gives lane L the value of lane
// L-1, wave_shl:1 the value of lane L+1.  With bound_ctrl set, lanes shifted
// in from outside the wave read 0 and no "old" value has to be materialised.
__device__ __forceinline__ int dpp_prev(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_next(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(dpp_prev(__float_as_int(v)));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(dpp_next(__float_as_int(v)));
}
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_prev((int)(b & 0xffffffffll));
  const int hi = dpp_prev((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_next((int)(b & 0xffffffffll));
  const int hi = dpp_next((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ----------------------------------------------------- closure helpers --
struct Lay {
  int n;
  int64_t stride, off_s0, off_s1;
};
__device__ __forceinline__ Lay lay_of(const CellLayout& L) {
  return Lay{L.n, L.stride, L.off_s0, L.off_s1};
}
// Row bases of the three closure blocks for row (j, k).
struct RowBase {
  int e;           // last i of the row (n - j - k)
  int32_t s0, s1;  // offsets of (0, j, k) in S0 and (e, j, k) in S1
  int32_t m;       // offset of (1, j, k) in M
};
__device__ __forceinline__ RowBase row_base(const Lay& L, int j, int k) {
  RowBase r;
  const int n = L.n;
  r.e = n - j - k;
  r.s0 = (int32_t)(L.off_s0 + t2w32(n + 1, j, k));
  r.s1 = (int32_t)(L.off_s1 + t2w32(n, j, k));
  r.m = (int32_t)tw32(n - 1, 0, j, k);
  return r;
}
// The same bases from per-plane parts: row (j, k) starts at
// m = pm - tri32(n - 1 - k - j) in M and at ps0 + j, ps1 + j in S0 and S1,
// so a wave walking the rows of a plane forms the plane part once.  Rows
// outside the plane (j < 0 or j + k > n) get offsets that are never used.
struct PlaneBase {
  int k;
  int32_t pm, ps0, ps1;
};
__device__ __forceinline__ PlaneBase plane_base(const Lay& L, int k) {
  const int n = L.n, w = n - 1;
  PlaneBase p;
  p.k = k;
  p.pm = tet32(w) - tet32(w - k) + tri32(w - k);
  p.ps0 = (int32_t)L.off_s0 + tri32(n + 1) - tri32(n + 1 - k);
  p.ps1 = (int32_t)L.off_s1 + tri32(n) - tri32(n - k);
  return p;
}
__device__ __forceinline__ RowBase row_base(const Lay& L, const PlaneBase& p, int j) {
  RowBase r;
  r.e = L.n - j - p.k;
  r.s0 = p.ps0 + j;
  r.s1 = p.ps1 + j;
  r.m = p.pm - tri32(L.n - 1 - p.k - j);
  return r;
}
__device__ __forceinline__ int32_t row_slot(const RowBase& r, int i) {
  return i == 0 ? r.s0 : (i == r.e ? r.s1 : r.m + i - 1);
}
__device__ __forceinline__ int64_t slot_of(const Lay& L, int i, int j, int k) {
  const int n = L.n;
  if (i == 0) return L.off_s0 + t2w32(n + 1, j, k);
  if (i + j + k == n) return L.off_s1 + t2w32(n, j, k);
  return tw32(n - 1, i - 1, j, k);
}

template <typename T>
__device__ __forceinline__ T ldv(const T* p) { return *p; }

// ------------------------------------------------------- buffer access --
// Buffer loads/stores with a per-cell range: an offset at or beyond the range
// reads 0 and drops the store, which replaces per-lane branches.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
#define HT_OOB 0x80000000u
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p,
                                                           int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bload(double& v, __amdgpu_buffer_rsrc_t r,
                                      unsigned off) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bload(float& v, __amdgpu_buffer_rsrc_t r,
                                      unsigned off) {
  v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r,
                                       unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
// Two consecutive values in one store (16 B in FP64, 8 B in FP32); the
// offset must be a multiple of the pair's size.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bstore2(double a, double b, __amdgpu_buffer_rsrc_t r,
                                        unsigned off) {
  const u32x2 lo = __builtin_bit_cast(u32x2, a), hi = __builtin_bit_cast(u32x2, b);
  const u32x4 v = {lo.x, lo.y, hi.x, hi.y};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
}
__device__ __forceinline__ void bstore2(float a, float b, __amdgpu_buffer_rsrc_t r,
                                        unsigned off) {
  const u32x2 v = {__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r,
                                       unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

}  // namespace ht
