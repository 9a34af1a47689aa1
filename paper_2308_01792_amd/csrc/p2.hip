// P2 operator y = A x (Section 5.1 composition of vertex and edge DoFs,
// Section 5.2 stencil application) on the closure layout of the next level.
//
// Bulk kernel (k_p2_march): a tile is J rows x 124 points of a plane k;
// lane L holds the points i0 + 2L and i0 + 2L + 1 of every row, so the two
// point parities of a row sit in two register components and every stencil
// entry is a fixed (component, lane shift) pair.  Each stencil entry is one
// FMA with a wave-uniform weight (scalar memory), summed per lane shift
// (-1, 0, +1) and shifted once at the end (DPP).  A wave marches its tile
// column through a segment of planes with the planes k - 2 .. k + 2 in a
// register ring, loading each plane once.  It writes the points strictly
// inside their row (1 <= i <= e - 1, the M block), whose boundary class
// depends only on j == 0 and k == 0, uniform over a row.
//
// Face kernel: the points of the faces i = 0 and i = n - j - k, one lane
// each, waves of one node parity, with the weights of their own boundary
// class and a gather over the unrolled stencil of their parity.
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

// ------------------------------------------------------------ k-march --
// One wave per tile column (j0, i0) and plane segment keeps the planes
// k - 2 .. k + 2 of its J + 4 rows in a register ring, so every plane is
// loaded once per column.  The march is unrolled by ten so that ring slots
// and the parity of k are compile-time.
template <typename T, int J>
__device__ __forceinline__ void p2_load_plane(T (&xp)[J + 4][2],
                                              __amdgpu_buffer_rsrc_t rx,
                                              const Lay& L, int kk, int j0,
                                              int i0, int lane) {
  const int n = L.n;
  const bool pv = kk >= 0 && kk <= n;
  const PlaneBase pb = plane_base(L, kk);
  // M offsets of consecutive rows: tri32(a - 1) = tri32(a) - max(a, 0)
  int a = n - 1 - kk - (j0 - 2);
  int ta = tri32(a);
#pragma unroll
  for (int rr = 0; rr < J + 4; ++rr) {
    const int jj = j0 - 2 + rr;
    const bool rv = pv && jj >= 0 && jj + kk <= n;
    RowBase rb;
    rb.e = n - jj - kk;
    rb.s0 = pb.ps0 + jj;
    rb.s1 = pb.ps1 + jj;
    rb.m = pb.pm - ta;
    ta -= a > 0 ? a : 0;
    --a;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int ii = i0 + 2 * lane + c;
      const bool ok = rv && ii >= 0 && ii <= rb.e;
      bload(xp[rr][c], rx, ok ? (unsigned)row_slot(rb, ii) * (unsigned)sizeof(T) : HT_OOB);
    }
  }
}

template <typename T, int J, int JB>
__device__ __forceinline__ void p2_march_column(const P2Args& a, int64_t cell,
                                                int j0, int i0, int k0) {
  const int lane = threadIdx.x & 63;
  const int n = a.n;
  const Lay L{n, a.stride, a.off_s0, a.off_s1};
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  typedef const __attribute__((address_space(4))) T* wptr;
  const wptr wc = (wptr)((const T*)a.w + cell * (int64_t)kP2PerCell);
  // last plane with a stored point: row j0 needs 1 <= i <= e - 1 for some
  // i >= i0 + 2
  // The column is marched from k0 (a multiple of 10, so that plane p sits in
  // ring slot p mod 5 and the parity of k is that of the phase) for at most
  // a.kseg planes.
  const int kcol = n - j0 - (i0 + 3 > 2 ? i0 + 3 : 2);
  const int kmax = kcol < k0 + a.kseg - 1 ? kcol : k0 + a.kseg - 1;
  T ring[5][J + 4][2];
  p2_load_plane<T, J>(ring[3], rx, L, k0 - 2, j0, i0, lane);
  p2_load_plane<T, J>(ring[4], rx, L, k0 - 1, j0, i0, lane);
  p2_load_plane<T, J>(ring[0], rx, L, k0, j0, i0, lane);
  p2_load_plane<T, J>(ring[1], rx, L, k0 + 1, j0, i0, lane);
  for (int kb = k0; kb <= kmax; kb += 10) {
    bool done = false;
    static_for<10>([&](auto PH) {
      constexpr int ph = decltype(PH)::value;
      constexpr int KB = ph & 1;  // kb is even
      const int k = kb + ph;
      if (done || k > kmax) { done = true; return; }
      p2_load_plane<T, J>(ring[(ph + 2) % 5], rx, L, k + 2, j0, i0, lane);
      T acc[J][2][3];
#pragma unroll
      for (int r = 0; r < J; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[r][c][q] = 0;
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
            constexpr int di = kP2Off.d[P][t][0], dj = kP2Off.d[P][t][1],
                          dk = kP2Off.d[P][t][2];
            constexpr int slot = (ph + dk + 10) % 5;
            constexpr int sh = c + di;
            constexpr int comp = sh & 1;
            constexpr int sig = (sh - comp) / 2;
            acc[r][c][sig + 1] += wp[t] * ring[slot][r + dj + 2][comp];
          });
        });
      });
      const PlaneBase pk = plane_base(L, k);
#pragma unroll
      for (int r = 0; r < J; ++r) {
        const int j = j0 + r;
        const int e = n - j - k;
        const RowBase rb = row_base(L, pk, j);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const T v = acc[r][c][1] + lane_next(acc[r][c][2]) + lane_prev(acc[r][c][0]);
          const int i = i0 + 2 * lane + c;
          const bool st = lane >= 1 && lane <= 62 && i >= 1 && i <= e - 1;
          bstore(v, ry, st ? (unsigned)(rb.m + i - 1) * (unsigned)sizeof(T) : HT_OOB);
        }
      }
    });
    if (done) break;
  }
}

template <typename T, int J>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_p2_march(P2Args a) {
  const int64_t wb = xcd_block(a.nc * a.nblk);
  if (wb >= a.nc * a.nblk) return;
  const int64_t cell = wb / a.nblk;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tix = (wb % a.nblk) * 4 + wave;
  if (tix >= a.ntiles) return;
  const int2 tl = a.tiles[tix];
  const int j0 = tl.x & 0xffff, k0 = tl.x >> 16;
  if (j0 & 1) p2_march_column<T, J, 1>(a, cell, j0, tl.y, k0);
  else p2_march_column<T, J, 0>(a, cell, j0, tl.y, k0);
}

// Edge points of one face of one cell for one parity class: SIDE 0 is the
// face i = 0 (S0), SIDE 1 the face i = n - j - k (S1, points with i >= 1);
// each lane has its own boundary class.  The stencil is unrolled at compile
// time; entries that always have zero weight on that face (di < 0 on i = 0,
// di + dj + dk > 0 on the slanted face) are dropped, so every remaining
// neighbour lies inside the closure whenever its row exists.
template <typename T, int P, int SIDE>
__device__ __forceinline__ void p2_edge_points(const P2Args& a, int64_t cell,
                                               int k, int j, bool valid) {
  const int n = a.n;
  const int i = SIDE == 0 ? 0 : n - j - k;
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const int cls = point_class(n, i, j, k);
  const T* wp = (const T*)a.w + cell * (int64_t)kP2PerCell +
                (P * kNumClasses + cls) * kP2MaxOffsets;
  T acc = 0;
  static_for<kP2Off.len[P]>([&](auto TT) {
    constexpr int t = decltype(TT)::value;
    constexpr int di = kP2Off.d[P][t][0], dj = kP2Off.d[P][t][1], dk = kP2Off.d[P][t][2];
    if constexpr ((SIDE == 0 && di >= 0) || (SIDE == 1 && di + dj + dk <= 0)) {
      const int ii = i + di, jj = j + dj, kk = k + dk;
      const bool ok = valid && jj >= 0 && kk >= 0 && ii >= 0 && ii + jj + kk <= n;
      // closure offset: face i = 0, slanted face, or M block (index.hpp);
      // all candidates computed, then selected (no branch per lane)
      int32_t off;
      if constexpr (SIDE == 0 && di == 0) {
        off = (int32_t)a.off_s0 + t2w32(n + 1, jj, kk);
      } else if constexpr (SIDE == 1 && di + dj + dk == 0) {
        // on the slanted face too; a one-point row (i = 0) lies in S0
        const int32_t s0 = (int32_t)a.off_s0 + t2w32(n + 1, jj, kk);
        const int32_t s1 = (int32_t)a.off_s1 + t2w32(n, jj, kk);
        off = ii == 0 ? s0 : s1;
      } else {
        const int w = n - 1 - kk;
        const int32_t m = tet32(n - 1) - tet32(w) + tri32(w) - tri32(w - jj) + ii - 1;
        const int32_t s1 = (int32_t)a.off_s1 + t2w32(n, jj, kk);
        const int32_t s0 = (int32_t)a.off_s0 + t2w32(n + 1, jj, kk);
        off = ii == 0 ? s0 : (ii + jj + kk == n ? s1 : m);
      }
      T xv;
      bload(xv, rx, ok ? (unsigned)off * (unsigned)sizeof(T) : HT_OOB);
      acc += wp[t] * xv;
    }
  });
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  const int el = SIDE == 0 ? (int)a.off_s0 + t2w32(n + 1, j, k) : (int)a.off_s1 + t2w32(n, j, k);
  bstore(acc, ry, valid ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB);
}

template <typename T, int SIDE>
__device__ __forceinline__ void p2_edge_run(const P2Args& a, int64_t cell, int k,
                                            int j, bool valid, int P) {
  switch (P) {
    case 0: p2_edge_points<T, 0, SIDE>(a, cell, k, j, valid); break;
    case 1: p2_edge_points<T, 1, SIDE>(a, cell, k, j, valid); break;
    case 2: p2_edge_points<T, 2, SIDE>(a, cell, k, j, valid); break;
    case 3: p2_edge_points<T, 3, SIDE>(a, cell, k, j, valid); break;
    case 4: p2_edge_points<T, 4, SIDE>(a, cell, k, j, valid); break;
    case 5: p2_edge_points<T, 5, SIDE>(a, cell, k, j, valid); break;
    case 6: p2_edge_points<T, 6, SIDE>(a, cell, k, j, valid); break;
    default: p2_edge_points<T, 7, SIDE>(a, cell, k, j, valid); break;
  }
}

// One wave per edge run (make_p2_edge_runs), with a uniform node parity: the
// points k = k0 + 2 lane + s of the edge j = 0 or, on face i = 0, of the
// edge j = n - k (k < n).
template <typename T>
__global__ __launch_bounds__(256) void k_p2_edge(P2Args a) {
  const int64_t wb = xcd_block(a.nc * a.nfblk);
  if (wb >= a.nc * a.nfblk) return;
  const int64_t cell = wb / a.nfblk;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t rix = (wb % a.nfblk) * 4 + wave;
  if (rix >= a.nruns) return;
  const int2 run = a.runs[rix];
  const int n = a.n, lane = (int)(threadIdx.x & 63);
  const int side = (run.x >> 16) & 1, s = (run.x >> 17) & 1;
  const int edge = (run.x >> 19) & 1;
  const int k = run.y + 2 * lane + s;
  const int j = edge ? n - k : 0;
  const bool valid = side == 0 ? (edge ? k < n : k <= n) : k <= n - 1;
  // node parity (n is even): i = 0 on side 0, i = n - j - k on side 1
  const int sj = j & 1, sk = k & 1;
  if (side == 0) p2_edge_run<T, 0>(a, cell, k, j, valid, (sj << 1) | (sk << 2));
  else p2_edge_run<T, 1>(a, cell, k, j, valid, ((sj + sk) & 1) | (sj << 1) | (sk << 2));
}

// ------------------------------------------------------- face tiles --
// The face points of the rows 1 <= j <= n - k - 1 of kP2FaceK planes, for
// kP2FaceRows rows from jb.  The stencil of a point on face i = 0 reaches the
// first three points of the rows j - 2 .. j + 2 of the planes k - 2 .. k + 2
// (di = 0, 1, 2), and that of a point on the slanted face the last three
// (distance t = -(di + dj + dk) = 0, 1, 2 from the face).  Those three
// values of every row are staged once in LDS, the first from S0 or S1
// (contiguous over j) and the other two from the head or tail of the row's M
// run (two neighbouring lanes per row, one cache line), and every point then
// reads its stencil from LDS.  Rows are split by the parity of j so that the
// lanes of a wave (every other row) read consecutive LDS words.
enum { kFaceStage = kP2FaceRows + 4, kFaceHalf = kFaceStage / 2,
       kFacePlanes = kP2FaceK + 4 };

template <typename T>
struct FaceImage {
  T v[kFacePlanes][3][2][kFaceHalf];  // [plane k0 - 2 + p][t][j parity][row / 2]
};

// Offset of point (i, j, k) with 0 <= i <= e = n - j - k.
__device__ __forceinline__ int32_t face_slot(const Lay& L, int i, int j, int k) {
  const int n = L.n, e = n - j - k;
  const int32_t s0 = (int32_t)L.off_s0 + t2w32(n + 1, j, k);
  const int32_t s1 = (int32_t)L.off_s1 + t2w32(n, j, k);
  const int32_t m = tw32(n - 1, i - 1, j, k);
  return i == 0 ? s0 : (i == e ? s1 : m);
}

template <typename T, int P, int SIDE>
__device__ __forceinline__ void p2_face_tile_points(const P2Args& a, const FaceImage<T>& im,
                                                    int64_t cell, int q, int k, int jb,
                                                    int lane) {
  constexpr int S = (P >> 1) & 1;  // parity of j (jb is even)
  const int n = a.n;
  const int j = jb + S + 2 * lane;
  const bool valid = j >= 1 && j <= n - k - 1;
  const int cls = (SIDE == 0 ? 1 : 8) | ((k == 0) << 2);
  typedef const __attribute__((address_space(4))) T* wptr;
  const wptr wp = (wptr)((const T*)a.w + cell * (int64_t)kP2PerCell) +
                  (P * kNumClasses + cls) * kP2MaxOffsets;
  T acc = 0;
  static_for<kP2Off.len[P]>([&](auto TT) {
    constexpr int t = decltype(TT)::value;
    constexpr int di = kP2Off.d[P][t][0], dj = kP2Off.d[P][t][1], dk = kP2Off.d[P][t][2];
    static_assert(di >= -2 && di <= 2 && dj >= -2 && dj <= 2 && dk >= -2 && dk <= 2 &&
                      di + dj + dk >= -2 && di + dj + dk <= 2,
                  "P2 stencil reaches two points in every direction");
    if constexpr ((SIDE == 0 && di >= 0) || (SIDE == 1 && di + dj + dk <= 0)) {
      constexpr int tt = SIDE == 0 ? di : -(di + dj + dk);
      // staged row j + dj is row index j - jb + 2 + dj = S + 2 + dj + 2 lane
      constexpr int r = S + 2 + dj;
      acc += wp[t] * im.v[q + 2 + dk][tt][r & 1][(r >> 1) + lane];
    }
  });
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  const int el = SIDE == 0 ? (int)a.off_s0 + t2w32(n + 1, j, k) : (int)a.off_s1 + t2w32(n, j, k);
  bstore(acc, ry, valid ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB);
}

template <typename T, int SIDE>
__device__ __forceinline__ void p2_face_tile_task(const P2Args& a, const FaceImage<T>& im,
                                                  int64_t cell, int q, int k, int jb,
                                                  int lane, int P) {
  switch (P) {
    case 0: p2_face_tile_points<T, 0, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 1: p2_face_tile_points<T, 1, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 2: p2_face_tile_points<T, 2, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 3: p2_face_tile_points<T, 3, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 4: p2_face_tile_points<T, 4, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 5: p2_face_tile_points<T, 5, SIDE>(a, im, cell, q, k, jb, lane); break;
    case 6: p2_face_tile_points<T, 6, SIDE>(a, im, cell, q, k, jb, lane); break;
    default: p2_face_tile_points<T, 7, SIDE>(a, im, cell, q, k, jb, lane); break;
  }
}

// One workgroup per face tile (make_p2_face_tiles).
template <typename T>
__global__ __launch_bounds__(256) void k_p2_face(P2Args a) {
  __shared__ FaceImage<T> im;
  const int64_t wb = xcd_block(a.nc * a.nftiles);
  if (wb >= a.nc * a.nftiles) return;
  const int64_t cell = wb / a.nftiles;
  const int2 tl = a.ftiles[wb % a.nftiles];
  const int k0 = tl.x & 0xffff, side = (tl.x >> 16) & 1, jb = tl.y;
  const int n = a.n;
  const Lay L{n, a.stride, a.off_s0, a.off_s1};
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  // t = 0: the face point of every staged row (S0 on face i = 0; S1 on the
  // slanted face, S0 for a one-point row)
  for (int e = threadIdx.x; e < kFacePlanes * kFaceStage; e += 256) {
    const int p = e / kFaceStage, r = e - p * kFaceStage;
    const int kk = k0 - 2 + p, jj = jb - 2 + r, ee = n - jj - kk;
    const bool ok = kk >= 0 && jj >= 0 && ee >= 0;
    const int i = side == 0 ? 0 : ee;
    T v;
    bload(v, rx, ok ? (unsigned)face_slot(L, i, jj, kk) * (unsigned)sizeof(T) : HT_OOB);
    im.v[p][0][r & 1][r >> 1] = v;
  }
  // t = 1, 2: two neighbouring lanes per row
  for (int e = threadIdx.x; e < 2 * kFacePlanes * kFaceStage; e += 256) {
    const int pr = e >> 1, t = 1 + (e & 1);
    const int p = pr / kFaceStage, r = pr - p * kFaceStage;
    const int kk = k0 - 2 + p, jj = jb - 2 + r, ee = n - jj - kk;
    const bool ok = kk >= 0 && jj >= 0 && t <= ee;
    const int i = side == 0 ? t : ee - t;
    T v;
    bload(v, rx, ok ? (unsigned)face_slot(L, i, jj, kk) * (unsigned)sizeof(T) : HT_OOB);
    im.v[p][t][r & 1][r >> 1] = v;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  for (int task = wave; task < 2 * kP2FaceK; task += 4) {
    const int q = task >> 1, sj = task & 1, k = k0 + q;
    if (k > n - 2) break;  // no rows 1 <= j <= n - k - 1 from here on
    const int sk = k & 1;
    if (side == 0) p2_face_tile_task<T, 0>(a, im, cell, q, k, jb, lane, (sj << 1) | (sk << 2));
    else p2_face_tile_task<T, 1>(a, im, cell, q, k, jb, lane,
                                 ((sj + sk) & 1) | (sj << 1) | (sk << 2));
  }
}

template <typename T>
void launch_p2_t(int J, const P2Args& a, hipStream_t s) {
  const dim3 block(256);
  const int64_t nb = a.nc * a.nblk, nf = a.nc * a.nfblk;
  if (nb > 0) {
    const dim3 grid((unsigned)(((nb + 7) / 8) * 8));
    // rows per march column: 2 in FP64 (register ring of 127 VGPRs), 4 in FP32
    constexpr int JT = sizeof(T) == 8 ? 2 : 4;
    if (J != JT) throw Error{HT_ERR_ARG, "P2 tile rows must be 2 in FP64 and 4 in FP32"};
    hipLaunchKernelGGL((k_p2_march<T, JT>), grid, block, 0, s, a);
  }
  if (nf > 0) {
    const dim3 grid((unsigned)(((nf + 7) / 8) * 8));
    hipLaunchKernelGGL((k_p2_edge<T>), grid, block, 0, s, a);
  }
  const int64_t nt = a.nc * a.nftiles;
  if (nt > 0) {
    const dim3 grid((unsigned)(((nt + 7) / 8) * 8));
    hipLaunchKernelGGL((k_p2_face<T>), grid, block, 0, s, a);
  }
}

// One wave per subgroup row (g, k, j) of one cell; lanes walk i.
template <typename T>
__global__ __launch_bounds__(256) void k_p2_pack(P2PackArgs a) {
  const int64_t nblk = (a.nrows + 3) / 4;
  const int64_t b = blockIdx.x;
  if (b >= a.nc * nblk) return;
  const int64_t cell = b / nblk;
  const int64_t r = (b % nblk) * 4 + (threadIdx.x >> 6);
  if (r >= a.nrows) return;
  const int4 row = a.rows[r];
  const int g = row.x, k = row.y, j = row.z;
  const int nco = a.n / 2;
  const int w = g == 0 ? nco + 1 : (g == 7 ? nco - 1 : nco);
  const int sx = (g == 1 || g == 4 || g == 5 || g == 7);
  const int sy = (g == 2 || g == 4 || g == 6 || g == 7);
  const int sz = (g == 3 || g == 5 || g == 6 || g == 7);
  const int64_t N = tet32(w);
  const Lay L{a.n, a.stride, a.off_s0, a.off_s1};
  const int64_t base = cell * a.cell_elems + (int64_t)a.m * row.w;
  T* lat = (T*)a.lattice;
  T* arr = (T*)a.arrays;
  for (int i = threadIdx.x & 63; i < w - k - j; i += 64) {
    const int64_t slot = cell * a.stride + slot_of(L, 2 * i + sx, 2 * j + sy, 2 * k + sz);
    const int64_t t = tw32(w, i, j, k);
    for (int d = 0; d < a.m; ++d) {
      const int64_t e = base + (a.soa ? d * N + t : (int64_t)a.m * t + d);
      const int64_t q = d * a.comp_stride + slot;
      if (a.unpack) lat[q] = arr[e];
      else arr[e] = lat[q];
    }
  }
}

}  // namespace

void launch_p2_pack(int dtype, const P2PackArgs& a, hipStream_t s) {
  const int64_t nb = a.nc * ((a.nrows + 3) / 4);
  if (nb <= 0) return;
  if (dtype == HT_F64) hipLaunchKernelGGL((k_p2_pack<double>), dim3((unsigned)nb), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_p2_pack<float>), dim3((unsigned)nb), dim3(256), 0, s, a);
}

void launch_p2(int dtype, int J, const P2Args& a, hipStream_t s) {
  if (!a.x || !a.y || !a.w) throw Error{HT_ERR_ARG, "P2 kernel needs x, y and the weights"};
  if (dtype == HT_F64) launch_p2_t<double>(J, a, s);
  else launch_p2_t<float>(J, a, s);
}

}  // namespace ht
