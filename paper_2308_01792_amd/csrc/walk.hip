// Transfer and elementwise kernels over the closure points of each cell:
// prolongation, the zero-guess Jacobi sweep, dots, masses, flags,
// coordinates.  A wave walks one (cell, walk tile) plane by plane.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"

namespace ht {

// --------------------------------------------------------- tile walker --
// The transfer and elementwise kernels visit the closure points of one
// (cell, walk tile) per wave: lanes are 64 consecutive i = i0 + lane, rows
// j0 .. j0 + kWalkRows - 1, planes k0 .. k0 + kWalkSeg - 1 (up to
// n - i0 - j0; a column of tiles is cut into segments so that no wave walks
// far longer than the others).  A workgroup holds kWalkWaves waves on
// consecutive walk tiles, so that enough waves are resident per CU for these
// streaming kernels.
enum { kWalkRows = 8, kWalkWaves = 4 };

// (block, wave) -> (cell, tile).  Consecutive blocks go to different XCDs;
// each XCD gets one contiguous run of tiles, as in the stencil kernel.
__device__ __forceinline__ bool walk_block(int64_t nblocks, int64_t ntiles,
                                           const int2* tiles, int wave,
                                           int64_t& cell, int& i0, int& j0, int& k0,
                                           int64_t& w) {
  const int64_t groups = (nblocks + kWalkWaves - 1) / kWalkWaves;
  const int64_t chunk = (groups + 7) / 8;
  w = ((int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8) * kWalkWaves + wave;
  if (w >= nblocks) return false;
  cell = w / ntiles;
  const int2 t = tiles[w % ntiles];
  i0 = t.x;
  j0 = t.y & 0xffff;
  k0 = t.y >> 16;
  return true;
}

// Prolongation u_f += P e_c, fine walk: a fine point with even index copies
// the coarse value at half its index; otherwise it is the midpoint of the
// coarse micro-edge along the one direction d with the same parity, and
// takes the mean of the coarse values at (f - d)/2 and (f + d)/2 (for even
// points both parents coincide and the mean is exact).  Coarse Dirichlet
// values count as zero.
//
// The parity of (i, j, k) fixes d.  A walk tile starts at i0 = 64 m and
// j0 = 8 m', so a lane's i parity is its own, a row's j parity is fixed by
// its place in the tile, and the planes are walked in pairs (even k, odd k):
// every parent row is then one of five coarse rows j0/2 .. j0/2 + 4 of the
// coarse planes k/2 and k/2 + 1, whose bases are formed once per pair.
struct CRow {
  int mb, sa, sb, e;
};
__device__ __forceinline__ CRow crow(const Lay& L, int j, int k) {
  const int n = L.n;
  CRow r;
  r.e = n - j - k;
  r.mb = (int)tw32(n - 1, 0, j, k) - 1;
  r.sa = (int)L.off_s0 + (int)t2w32(n + 1, j, k);
  r.sb = (int)L.off_s1 + (int)t2w32(n, j, k);
  return r;
}
// direction with parity p = (i & 1) | (j & 1) << 1 | (k & 1) << 2 among
// x, y, xy, z, xz, yz, xyz (zero for p = 0)
constexpr int kParDi[8] = {0, 1, 0, -1, 0, -1, 0, 1};
constexpr int kParDj[8] = {0, 0, 1, 1, 0, 0, -1, -1};

template <typename T>
__global__ __launch_bounds__(64 * kWalkWaves) void k_prolong(XferArgs a) {
  int64_t cell, w;
  int i0, j0, k0;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (!walk_block(a.nblocks, a.ntiles, a.tiles, wave, cell, i0, j0, k0, w)) return;
  const int lane = threadIdx.x & 63;
  const uint8_t fl = lane < 16 ? a.cls[cell * 16 + lane].flags : 0;
  const unsigned dmask = (unsigned)__ballot((fl & kClsDirichlet) != 0) & 0xffffu;
  const Lay Lf{a.nf, a.stride_f, a.off_s0_f, a.off_s1_f};
  const Lay Lc{a.nc_, a.stride_c, a.off_s0_c, a.off_s1_c};
  const __amdgpu_buffer_rsrc_t rc =
      make_rsrc((const T*)a.src + cell * Lc.stride, Lc.stride * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ru =
      make_rsrc((T*)a.dst + cell * Lf.stride, Lf.stride * (int64_t)sizeof(T));
  const int n = Lf.n, w1 = n - 1, i = i0 + lane;
  const bool odd = (lane & 1) != 0;
  const int jc0 = j0 >> 1;
  const int kmax = min(n - i0 - j0, k0 + kWalkSeg - 1);  // k0 is even

  // Fine plane k (parity PK); R[p][s] is coarse row jc0 + s of plane
  // k / 2 + p.  All loads of the plane's rows first, then the updates.
  auto plane = [&](auto pk_tag, int k, const CRow (&R)[2][5]) {
    constexpr int PK = decltype(pk_tag)::value;
    const int kc = k >> 1;
    unsigned ou[kWalkRows], oa[kWalkRows], ob[kWalkRows];
    bool za[kWalkRows], zb[kWalkRows];
    int mb = (int)(tet32(w1) - tet32(w1 - k)) - 1 + j0 * (w1 - k) - j0 * (j0 - 1) / 2;
    int sa = (int)Lf.off_s0 + (int)(tri32(n + 1) - tri32(n + 1 - k)) + j0;
    int sb = (int)Lf.off_s1 + (int)(tri32(n) - tri32(n - k)) + j0;
#pragma unroll
    for (int r = 0; r < kWalkRows; ++r) {
      const int j = j0 + r;
      const int e = n - j - k;
      const bool valid = e >= i0 && i <= e;
      const int el = i == 0 ? sa : (i == e ? sb : mb + i);
      ou[r] = valid ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB;
      mb += w1 - k - j;
      ++sa;
      ++sb;
      // parities of the even and odd lanes of this row
      const int q0 = ((r & 1) << 1) | (PK << 2), q1 = q0 | 1;
      const int di = odd ? kParDi[q1] : kParDi[q0];
      // parent -d: coarse row (r - dj) / 2 of plane k / 2 (either parity
      // of k); parent +d: row (r + dj) / 2 of plane (k + PK) / 2
      auto parent = [&](int sgn, int pp, int s0, int s1, unsigned& off,
                        bool& zero) {
        const CRow& C = odd ? R[pp][s1] : R[pp][s0];
        const int jr = jc0 + (odd ? s1 : s0), kr = kc + pp;
        const int ic = (i + sgn * di) >> 1;
        int e2 = (ic == C.e) ? C.sb : C.mb + ic;
        e2 = (ic == 0) ? C.sa : e2;
        const int cls = (ic == 0) | ((jr == 0) << 1) | ((kr == 0) << 2) | ((ic == C.e) << 3);
        off = valid ? (unsigned)e2 * (unsigned)sizeof(T) : HT_OOB;
        zero = ((dmask >> cls) & 1u) != 0;
      };
      parent(-1, 0, (r - kParDj[q0]) >> 1, (r - kParDj[q1]) >> 1, oa[r], za[r]);
      parent(+1, PK, (r + kParDj[q0]) >> 1, (r + kParDj[q1]) >> 1, ob[r], zb[r]);
    }
    T u[kWalkRows], va[kWalkRows], vb[kWalkRows];
#pragma unroll
    for (int r = 0; r < kWalkRows; ++r) {
      bload(u[r], ru, ou[r]);
      bload(va[r], rc, oa[r]);
      bload(vb[r], rc, ob[r]);
    }
#pragma unroll
    for (int r = 0; r < kWalkRows; ++r) {
      const T x = za[r] ? (T)0 : va[r];
      const T y = zb[r] ? (T)0 : vb[r];
      bstore(u[r] + (T)0.5 * (x + y), ru, ou[r]);
    }
  };

  for (int k = k0; k <= kmax; k += 2) {
    CRow R[2][5];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int s = 0; s < 5; ++s) R[p][s] = crow(Lc, jc0 + s, (k >> 1) + p);
    plane(std::integral_constant<int, 0>{}, k, R);
    if (k + 1 <= kmax) plane(std::integral_constant<int, 1>{}, k + 1, R);
  }
}

// Elementwise kernels over the closure points.  Per plane, the offsets of
// all rows of the tile are formed first and every load is issued before any
// result is used.
template <typename T, int EOP>
__global__ __launch_bounds__(64 * kWalkWaves) void k_elem(ElemArgs a) {
  int64_t cell, w;
  int i0, j0, k0;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const bool live = walk_block(a.nblocks, a.ntiles, a.tiles, wave, cell, i0, j0, k0, w);
  // class table of the wave's cell; every wave reaches the barrier
  __shared__ ClassInfo cis[kWalkWaves][16];
  // zero-guess factor per class: omega / diagonal, 0 at Dirichlet points
  __shared__ T gz[kWalkWaves][16];
  if (live && lane < 16) {
    const ClassInfo c = a.cls[cell * 16 + lane];
    cis[wave][lane] = c;
    gz[wave][lane] = (c.flags & kClsDirichlet) ? (T)0 : (T)(a.alpha * a.nscale * c.inv_diag_unit);
  }
  __syncthreads();
  if (!live) return;
  const ClassInfo* ci = cis[wave];
  const Lay L{a.n, a.stride, a.off_s0, a.off_s1};
  const int64_t cb = cell * L.stride;
  const int64_t bytes = L.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t r0 =
      make_rsrc(a.in0 ? (const T*)a.in0 + cb : (const T*)a.out + cb, bytes);
  const __amdgpu_buffer_rsrc_t r1 =
      make_rsrc(a.in1 ? (const T*)a.in1 + cb : (const T*)a.out + cb, bytes);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc((T*)a.out + cb, bytes);
  const int n = L.n, w1 = n - 1, i = i0 + lane;
  const int kmax = min(n - i0 - j0, k0 + kWalkSeg - 1);
  double acc = 0.0;
  for (int k = k0; k <= kmax; ++k) {
    unsigned off[kWalkRows];
    int cl[kWalkRows], elr[kWalkRows];
    int mb = (int)(tet32(w1) - tet32(w1 - k)) - 1 + j0 * (w1 - k) - j0 * (j0 - 1) / 2;
    int sa = (int)L.off_s0 + (int)(tri32(n + 1) - tri32(n + 1 - k)) + j0;
    int sb = (int)L.off_s1 + (int)(tri32(n) - tri32(n - k)) + j0;
#pragma unroll
    for (int r = 0; r < kWalkRows; ++r) {
      const int j = j0 + r;
      const int e = n - j - k;
      const bool valid = e >= i0 && i <= e;
      elr[r] = i == 0 ? sa : (i == e ? sb : mb + i);
      off[r] = valid ? (unsigned)elr[r] * (unsigned)sizeof(T) : HT_OOB;
      cl[r] = valid ? ((i == 0) | ((j == 0) << 1) | ((k == 0) << 2) | ((i == e) << 3)) : -1;
      mb += w1 - k - j;
      ++sa;
      ++sb;
    }
    if (EOP == EOP_ZERO_GUESS) {
      // first Jacobi sweep from u = 0: u = omega D^-1 b
      T bv[kWalkRows];
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) bload(bv[r], r0, off[r]);
      // rows off the faces j = 0 and k = 0 hold classes 0, 1 (i = 0),
      // 8 (i = e) and 9 (i = 0 = e) only: select among four factors
      // instead of a lookup
      const T g0 = gz[wave][0], g1 = gz[wave][1], g8 = gz[wave][8], g9 = gz[wave][9];
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) {
        T f;
        if (j0 + r > 0 && k > 0)
          f = (cl[r] & 1) ? ((cl[r] & 8) ? g9 : g1) : ((cl[r] & 8) ? g8 : g0);
        else f = gz[wave][cl[r] < 0 ? 0 : cl[r]];
        bstore(f * bv[r], ro, off[r]);
      }
    } else if (EOP == EOP_DOT) {
      T xv[kWalkRows], yv[kWalkRows];
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) {
        bload(xv[r], r0, off[r]);
        bload(yv[r], r1, off[r]);
      }
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) {
        const uint8_t f = cl[r] < 0 ? 0 : ci[cl[r]].flags;
        const bool use = (f & kClsOwner) && !(f & kClsDirichlet);
        acc += use ? (double)xv[r] * (double)yv[r] : 0.0;
      }
    } else if (EOP == EOP_MASS) {
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r)
        bstore((T)(ci[cl[r] < 0 ? 0 : cl[r]].mass_unit * a.nscale), ro, off[r]);
    } else if (EOP == EOP_ZERO_INTERIOR) {
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) {
        const bool dir = cl[r] >= 0 && (ci[cl[r]].flags & kClsDirichlet);
        bstore((T)0, ro, dir ? HT_OOB : off[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kWalkRows; ++r) {
        if (cl[r] < 0) continue;
        const ClassInfo& c = ci[cl[r]];
        const int64_t s = cb + elr[r];
        if (EOP == EOP_FLAGS) {
          uint8_t f = (c.flags & kClsOwner) ? HT_SLOT_OWNER : HT_SLOT_GHOST;
          if (c.flags & kClsDirichlet) f |= HT_SLOT_DIRICHLET;
          ((uint8_t*)a.out)[s] = f;
        } else if (EOP == EOP_COORDS || EOP == EOP_PROBE) {
          const double* X = a.cell_xyz + cell * 12;     // sorted by global id
          const int8_t* ord = a.cell_order + cell * 4;  // local index per sorted
          const int j = j0 + r;
          const int wl[4] = {n - i - j - k, i, j, k};
          T* o = (T*)a.out;
          double xyz[3];
          for (int a3 = 0; a3 < 3; ++a3) {
            double sum = 0.0;
            for (int q = 0; q < 4; ++q) {
              const int wq = wl[ord[q]];
              if (wq > 0) sum += (double)wq * X[3 * q + a3];
            }
            xyz[a3] = sum * a.alpha;
            if (EOP == EOP_COORDS) o[3 * s + a3] = (T)xyz[a3];
          }
          if (EOP == EOP_PROBE) {
            // start vector of the power iteration: a field that oscillates
            // on the scale of the finest micro-cells, zero on the boundary
            const double ph = 1000.0 * xyz[0] + 1700.0 * xyz[1] + 2300.0 * xyz[2];
            o[s] = (c.flags & kClsDirichlet) ? (T)0 : (T)sin(ph);
          }
        }
      }
    }
  }
  if (EOP == EOP_DOT) {
    acc = wave_sum(acc);
    if (lane == 0) a.partials[w] = acc;
  }
}

// --------------------------------------------------------- launchers ----
static dim3 walk_grid(int64_t nblocks) {
  const int64_t groups = (nblocks + kWalkWaves - 1) / kWalkWaves;
  return dim3((unsigned)(((groups + 7) / 8) * 8));
}

void launch_prolong(int dtype, const XferArgs& a, hipStream_t s) {
  const dim3 grid = walk_grid(a.nblocks), block(64 * kWalkWaves);
  if (dtype == HT_F64) hipLaunchKernelGGL(k_prolong<double>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_prolong<float>, grid, block, 0, s, a);
}

template <typename T>
static void launch_elem_t(int eop, const ElemArgs& a, hipStream_t s) {
  const dim3 grid = walk_grid(a.nblocks), block(64 * kWalkWaves);
  switch (eop) {
    case EOP_ZERO_GUESS: hipLaunchKernelGGL((k_elem<T, EOP_ZERO_GUESS>), grid, block, 0, s, a); break;
    case EOP_MASS: hipLaunchKernelGGL((k_elem<T, EOP_MASS>), grid, block, 0, s, a); break;
    case EOP_ZERO_INTERIOR: hipLaunchKernelGGL((k_elem<T, EOP_ZERO_INTERIOR>), grid, block, 0, s, a); break;
    case EOP_DOT: hipLaunchKernelGGL((k_elem<T, EOP_DOT>), grid, block, 0, s, a); break;
    case EOP_FLAGS: hipLaunchKernelGGL((k_elem<T, EOP_FLAGS>), grid, block, 0, s, a); break;
    case EOP_COORDS: hipLaunchKernelGGL((k_elem<T, EOP_COORDS>), grid, block, 0, s, a); break;
    case EOP_PROBE: hipLaunchKernelGGL((k_elem<T, EOP_PROBE>), grid, block, 0, s, a); break;
  }
}
void launch_elem(int dtype, int eop, const ElemArgs& a, hipStream_t s) {
  if (dtype == HT_F64) launch_elem_t<double>(eop, a, s);
  else launch_elem_t<float>(eop, a, s);
}

}  // namespace ht
