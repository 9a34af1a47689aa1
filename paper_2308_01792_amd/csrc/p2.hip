// P2 operator y = A x (Section 5.1 composition of vertex and edge DoFs,
// Section 5.2 stencil application) on the closure layout of the next level.
//
// Bulk kernel: one wave per tile of J rows x 124 points of one plane k; lane
// L holds the points i0 + 2L and i0 + 2L + 1 of every row, so the two point
// parities of a row sit in two register components and every stencil entry
// is a fixed (component, lane shift) pair.  For each of the five planes
// k - 2 .. k + 2 the wave loads the J + 4 rows it needs once; each stencil
// entry is then one FMA with a wave-uniform weight (scalar memory), summed
// per lane shift (-1, 0, +1) and shifted once at the end (DPP).  The bulk
// kernel writes the points strictly inside their row (1 <= i <= e - 1, the
// M block); their boundary class depends only on j == 0 and k == 0, which
// are uniform over a row.
//
// Face kernel: the points of the faces i = 0 and i = n - j - k, one thread
// each, with the weights of their own boundary class and a gather over the
// stencil of their parity.
//
// Points on the cell surface get the cell's partial row; the ghost exchange
// completes them and zeroes Dirichlet rows.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "device.hpp"
#include "hytet_impl.hpp"
#include "p2.hpp"

namespace ht {
namespace {

__constant__ P2Offsets kP2OffDev = make_p2_offsets();

template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// XCD-aware block order (block b runs on XCD b % 8): each XCD gets a
// contiguous run of work so that neighbouring tiles share an L2.
__device__ __forceinline__ int64_t xcd_block(int64_t nb) {
  const int64_t chunk = (nb + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
}

template <typename T, int J, int JB, int KB>
__device__ __forceinline__ void p2_bulk_tile(const P2Args& a, int64_t cell,
                                             int k, int j0, int i0) {
  const int lane = threadIdx.x & 63;
  const int n = a.n;
  const Lay L{n, a.stride, a.off_s0, a.off_s1};
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  // the weights are read-only for the whole kernel: reading them through the
  // constant address space lets every wave-uniform weight come from scalar
  // loads instead of vector memory instructions
  typedef const __attribute__((address_space(4))) T* wptr;
  const wptr wc = (wptr)((const T*)a.w + cell * (int64_t)kP2PerCell);
  T acc[J][2][3];
#pragma unroll
  for (int r = 0; r < J; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < 3; ++s) acc[r][c][s] = 0;

  static_for<5>([&](auto DK) {
    constexpr int dk = decltype(DK)::value - 2;
    const int kk = k + dk;
    if (kk < 0 || kk > n) return;
    T xr[J + 4][2];
#pragma unroll
    for (int rr = 0; rr < J + 4; ++rr) {
      const int jj = j0 - 2 + rr;
      const bool rv = jj >= 0 && jj + kk <= n;
      const RowBase rb = row_base(L, rv ? jj : 0, kk);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int ii = i0 + 2 * lane + c;
        const bool ok = rv && ii >= 0 && ii <= rb.e;
        bload(xr[rr][c], rx, ok ? (unsigned)row_slot(rb, ii) * (unsigned)sizeof(T) : HT_OOB);
      }
    }
    static_for<J>([&](auto R) {
      constexpr int r = decltype(R)::value;
      constexpr int jb = JB ^ (r & 1);
      const int cls = ((j0 + r == 0) << 1) | ((k == 0) << 2);
      static_for<2>([&](auto C) {
        constexpr int c = decltype(C)::value;
        constexpr int P = c | (jb << 1) | (KB << 2);
        const wptr wp = wc + (P * kNumClasses + cls) * kP2MaxOffsets;
        static_for<kP2Off.len[P]>([&](auto TT) {
          constexpr int t = decltype(TT)::value;
          if constexpr (kP2Off.d[P][t][2] == dk) {
            constexpr int di = kP2Off.d[P][t][0], dj = kP2Off.d[P][t][1];
            constexpr int s = c + di;            // source at i0 + 2 (L + sig) + comp
            constexpr int comp = s & 1;
            constexpr int sig = (s - comp) / 2;
            acc[r][c][sig + 1] += wp[t] * xr[r + dj + 2][comp];
          }
        });
      });
    });
  });

#pragma unroll
  for (int r = 0; r < J; ++r) {
    const int j = j0 + r;
    const int e = n - j - k;
    const RowBase rb = row_base(L, e >= 0 ? j : 0, k);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T v = acc[r][c][1] + lane_next(acc[r][c][2]) + lane_prev(acc[r][c][0]);
      const int i = i0 + 2 * lane + c;
      const bool st = lane >= 1 && lane <= 62 && i >= 1 && i <= e - 1;
      bstore(v, ry, st ? (unsigned)(rb.m + i - 1) * (unsigned)sizeof(T) : HT_OOB);
    }
  }
}

template <typename T, int J>
__global__ __launch_bounds__(256) void k_p2_bulk(P2Args a) {
  const int64_t wb = xcd_block(a.nc * a.nblk);
  if (wb >= a.nc * a.nblk) return;
  const int64_t cell = wb / a.nblk;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tix = (wb % a.nblk) * 4 + wave;
  if (tix >= a.ntiles) return;
  const int2 tl = a.tiles[tix];
  const int k = tl.x & 0xffff, j0 = tl.x >> 16, i0 = tl.y;
  switch (((j0 & 1) << 1) | (k & 1)) {
    case 0: p2_bulk_tile<T, J, 0, 0>(a, cell, k, j0, i0); break;
    case 1: p2_bulk_tile<T, J, 0, 1>(a, cell, k, j0, i0); break;
    case 2: p2_bulk_tile<T, J, 1, 0>(a, cell, k, j0, i0); break;
    default: p2_bulk_tile<T, J, 1, 1>(a, cell, k, j0, i0); break;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_p2_face(P2Args a) {
  const int64_t wb = xcd_block(a.nc * a.nfblk);
  if (wb >= a.nc * a.nfblk) return;
  const int64_t cell = wb / a.nfblk;
  const int64_t rix = (wb % a.nfblk) * 4 + (threadIdx.x >> 6);
  if (rix >= a.nruns) return;
  const int2 run = a.runs[rix];
  const int n = a.n, k = run.x, j = run.y + (int)(threadIdx.x & 63);
  if (j + k > n) return;
  const Lay L{n, a.stride, a.off_s0, a.off_s1};
  const T* x = (const T*)a.x + cell * a.stride;
  T* y = (T*)a.y + cell * a.stride;
  const T* wc = (const T*)a.w + cell * (int64_t)kP2PerCell;
  for (int side = 0; side < 2; ++side) {
    const int i = side == 0 ? 0 : n - j - k;
    if (side == 1 && i == 0) break;  // a one-point row lies in face i = 0
    const int P = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
    const T* wp = wc + (P * kNumClasses + point_class(n, i, j, k)) * kP2MaxOffsets;
    T acc = 0;
    const int len = kP2OffDev.len[P];
    for (int t = 0; t < len; ++t) {
      const T wt = wp[t];
      if (wt == T(0)) continue;
      const int ii = i + kP2OffDev.d[P][t][0], jj = j + kP2OffDev.d[P][t][1],
                kk = k + kP2OffDev.d[P][t][2];
      if (ii < 0 || jj < 0 || kk < 0 || ii + jj + kk > n) continue;
      acc += wt * x[slot_of(L, ii, jj, kk)];
    }
    y[slot_of(L, i, j, k)] = acc;
  }
}

template <typename T>
void launch_p2_t(int J, const P2Args& a, hipStream_t s) {
  const dim3 block(256);
  const int64_t nb = a.nc * a.nblk, nf = a.nc * a.nfblk;
  if (nb > 0) {
    const dim3 grid((unsigned)(((nb + 7) / 8) * 8));
    switch (J) {
      case 2: hipLaunchKernelGGL((k_p2_bulk<T, 2>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_p2_bulk<T, 4>), grid, block, 0, s, a); break;
      default: throw Error{HT_ERR_ARG, "P2 tile rows must be 2 or 4"};
    }
  }
  if (nf > 0) {
    const dim3 grid((unsigned)(((nf + 7) / 8) * 8));
    hipLaunchKernelGGL((k_p2_face<T>), grid, block, 0, s, a);
  }
}

}  // namespace

void launch_p2(int dtype, int J, const P2Args& a, hipStream_t s) {
  if (!a.x || !a.y || !a.w) throw Error{HT_ERR_ARG, "P2 kernel needs x, y and the weights"};
  if (dtype == HT_F64) launch_p2_t<double>(J, a, s);
  else launch_p2_t<float>(J, a, s);
}

}  // namespace ht
