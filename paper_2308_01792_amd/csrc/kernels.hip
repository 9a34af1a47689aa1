// Device kernels of the hytet library (gfx950, wave64).
//
// Vectors are per-cell closure blocks (index.hpp).  One operator application
// is two launches:
//   1. the cell kernel streams every macro-cell's closure once, marching in k
//      with the planes k-1, k, k+1 of a (64-lane x J-row) tile in registers,
//      and writes the full 15-point row at cell-interior points and the
//      cell's partial row at points on its faces, edges and vertices;
//   2. the ghost-exchange kernel visits every micro-vertex shared by several
//      cells once, sums the partial rows of all incident cells, applies the
//      operation's epilogue and writes the result into every copy.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ht {

// ------------------------------------------------------- lane exchange --
// DPP wave shifts (GFX9 family): wave_shr:1 gives lane L the value of lane
// L-1, wave_shl:1 the value of lane L+1.  Lanes shifted in from outside the
// wave read 0.
__device__ __forceinline__ int dpp_prev(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_next(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
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

// Self-test of the lane exchange: out[l] = prev(l), out[64 + l] = next(l).
__global__ void k_lane_selftest(int* out) {
  const int l = threadIdx.x;
  out[l] = (int)lane_prev((double)(l + 1));
  out[64 + l] = (int)lane_next((float)(l + 1));
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
  r.s0 = (int32_t)(L.off_s0 + t2_w(n + 1, j, k));
  r.s1 = (int32_t)(L.off_s1 + t2_w(n, j, k));
  r.m = (int32_t)t_w(n - 1, 0, j, k);
  return r;
}
__device__ __forceinline__ int32_t row_slot(const RowBase& r, int i) {
  return i == 0 ? r.s0 : (i == r.e ? r.s1 : r.m + i - 1);
}
__device__ __forceinline__ int64_t slot_of(const Lay& L, int i, int j, int k) {
  const int n = L.n;
  if (i == 0) return L.off_s0 + t2_w(n + 1, j, k);
  if (i + j + k == n) return L.off_s1 + t2_w(n, j, k);
  return t_w(n - 1, i - 1, j, k);
}

template <typename T>
__device__ __forceinline__ T ldv(const T* p) { return *p; }

// ----------------------------------------------------------- cell kernel --
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
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r,
                                       unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// One wave = one tile of 64 consecutive i (62 outputs, one halo lane on each
// side) and J rows j0..j0+J-1, marching k upwards with the planes k-1, k,
// k+1 of rows j0-1..j0+J in registers; i +- 1 neighbours come from DPP.
//
// Points on the cell's faces get the cell's partial row.  On rows with
// j >= 1, k >= 1 and line end e >= 2 only two lanes can be surface points:
// i = 0 (face i = 0) and i = e (slanted face).  Their partial row equals the
// interior row (values outside the closure load as 0) plus a 7-term
// correction over the in-face offsets with uniform weights.  Rows with
// j == 0, k == 0 or e <= 1 take per-lane class weights from LDS.
template <typename T, int OP, int J>
__global__ __launch_bounds__(64) void k_cell(CellArgs a) {
  __shared__ T wtab[16 * 15];
  __shared__ T wdel[14];  // in-face corrections: face i = 0, slanted face
  const int lane = threadIdx.x;
  // XCD-aware block order: block b runs on XCD b % 8; give each XCD a
  // contiguous run of (cell, tile) work so tiles sharing halo rows share L2.
  const int64_t nb = a.nblocks;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t w = (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
  if (w >= nb) return;
  const int64_t cell = w / a.ntiles;
  const int2 tile = a.tiles[w % a.ntiles];
  const int i0 = tile.x, j0 = tile.y;
  const int n = a.n;
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t rb =
      make_rsrc(a.b ? (const T*)a.b + cell * a.stride : (const T*)a.y, bytes);
  const T* wc = (const T*)a.w + cell * 240;
  for (int t = lane; t < 240; t += 64) wtab[t] = wc[t];
  if (lane < 14) {
    const int d0[7] = {0, 3, 4, 5, 6, 11, 12}, d8[7] = {0, 7, 8, 9, 10, 11, 12};
    const int d = lane < 7 ? d0[lane] : d8[lane - 7];
    const int cls = lane < 7 ? 1 : 8;
    wdel[lane] = wc[cls * 15 + d] - wc[d];
  }
  __syncthreads();
  const T w0 = wc[0], w1 = wc[1], w2 = wc[2], w3 = wc[3], w4 = wc[4],
          w5 = wc[5], w6 = wc[6], w7 = wc[7], w8 = wc[8], w9 = wc[9],
          w10 = wc[10], w11 = wc[11], w12 = wc[12], w13 = wc[13], w14 = wc[14];
  const T omega_invd = (T)(a.omega * a.nscale * a.cls[cell * 16].inv_diag_unit);
  const int off_s0 = (int)a.off_s0, off_s1 = (int)a.off_s1;

  const int i = i0 - 1 + lane;
  const bool is0 = (i == 0);
  const unsigned out_mask = (lane >= 1 && lane <= 62) ? 0u : HT_OOB;
  // Offsets of the rows j0-1 .. j0+J of plane kk.  Row j of a plane: main
  // block base mb(j) (element of i = 0 if it were stored there), S0 and S1
  // entries sa(j), sb(j); consecutive rows differ by the main-block row
  // length (n-1-kk-j) and by 1 in S0/S1.
  auto plane_offsets = [&](int kk, unsigned (&o)[J + 2]) {
    const int w1 = n - 1;
    int mb = (int)(n_tet(w1) - n_tet(w1 - kk)) - 1;
    int sa = off_s0 + (int)(n_tri(n + 1) - n_tri(n + 1 - kk));
    int sb = off_s1 + (int)(n_tri(n) - n_tri(n - kk));
    const int jf = j0 - 1;
    if (jf > 0) {
      mb += jf * (w1 - kk) - jf * (jf - 1) / 2;
      sa += jf;
      sb += jf;
    }
#pragma unroll
    for (int r = 0; r < J + 2; ++r) {
      const int j = jf + r;
      const int e = n - j - kk;
      unsigned off = HT_OOB;
      if (j >= 0 && e >= 0 && kk <= n) {
        int el = (i == e) ? sb : mb + i;
        el = is0 ? sa : el;
        off = ((unsigned)i <= (unsigned)e) ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB;
      }
      o[r] = off;
      if (j >= 0) {
        mb += w1 - kk - j;
        ++sa;
        ++sb;
      }
    }
  };

  T xm[J + 2], xc[J + 2], xp[J + 2];
  unsigned oc[J + 2];
  plane_offsets(0, oc);
#pragma unroll
  for (int r = 0; r < J + 2; ++r) {
    xm[r] = (T)0;
    bload(xc[r], rx, oc[r]);
  }
  double nsq = 0.0;
  const int kmax = n - i0 - j0;
  for (int k = 0; k <= kmax; ++k) {
    unsigned op[J + 2];
    plane_offsets(k + 1, op);
#pragma unroll
    for (int r = 0; r < J + 2; ++r) bload(xp[r], rx, op[r]);
#pragma unroll
    for (int rr = 0; rr < J; ++rr) {
      const int j = j0 + rr;
      const int e = n - j - k;
      if (e >= i0) {
        const T c = xc[rr + 1];
        const T v1 = lane_next(c), v2 = lane_prev(c);
        const T v3 = xc[rr + 2], v4 = xc[rr];
        const T v5 = xp[rr + 1], v6 = xm[rr + 1];
        const T v7 = lane_prev(xc[rr + 2]), v8 = lane_next(xc[rr]);
        const T v9 = lane_prev(xp[rr + 1]), v10 = lane_next(xm[rr + 1]);
        const T v11 = xp[rr], v12 = xm[rr + 2];
        const T v13 = lane_next(xp[rr]), v14 = lane_prev(xm[rr + 2]);
        T acc = w0 * c;
        acc = fma(w1, v1, acc); acc = fma(w2, v2, acc); acc = fma(w3, v3, acc);
        acc = fma(w4, v4, acc); acc = fma(w5, v5, acc); acc = fma(w6, v6, acc);
        acc = fma(w7, v7, acc); acc = fma(w8, v8, acc); acc = fma(w9, v9, acc);
        acc = fma(w10, v10, acc); acc = fma(w11, v11, acc);
        acc = fma(w12, v12, acc); acc = fma(w13, v13, acc);
        acc = fma(w14, v14, acc);
        bool surf;
        if (j == 0 || k == 0 || e <= 1) {
          const int cls = (int)is0 | ((j == 0) << 1) | ((k == 0) << 2) | ((i == e) << 3);
          const T* wt = wtab + cls * 15;
          T sacc = wt[0] * c;
          sacc = fma(wt[1], v1, sacc); sacc = fma(wt[2], v2, sacc);
          sacc = fma(wt[3], v3, sacc); sacc = fma(wt[4], v4, sacc);
          sacc = fma(wt[5], v5, sacc); sacc = fma(wt[6], v6, sacc);
          sacc = fma(wt[7], v7, sacc); sacc = fma(wt[8], v8, sacc);
          sacc = fma(wt[9], v9, sacc); sacc = fma(wt[10], v10, sacc);
          sacc = fma(wt[11], v11, sacc); sacc = fma(wt[12], v12, sacc);
          sacc = fma(wt[13], v13, sacc); sacc = fma(wt[14], v14, sacc);
          acc = sacc;
          surf = cls != 0;
        } else {
          const bool ise = (i == e);
          if (i0 == 0) {  // face i = 0: class-1 minus interior weights
            T cc = wdel[0] * c;
            cc = fma(wdel[1], v3, cc); cc = fma(wdel[2], v4, cc);
            cc = fma(wdel[3], v5, cc); cc = fma(wdel[4], v6, cc);
            cc = fma(wdel[5], v11, cc); cc = fma(wdel[6], v12, cc);
            acc = is0 ? acc + cc : acc;
          }
          if (e <= i0 + 61) {  // slanted face: class-8 minus interior weights
            T cc = wdel[7] * c;
            cc = fma(wdel[8], v7, cc); cc = fma(wdel[9], v8, cc);
            cc = fma(wdel[10], v9, cc); cc = fma(wdel[11], v10, cc);
            cc = fma(wdel[12], v11, cc); cc = fma(wdel[13], v12, cc);
            acc = ise ? acc + cc : acc;
          }
          surf = is0 || ise;
        }
        const unsigned so = oc[rr + 1] | out_mask;
        T out = acc;
        if (OP == OP_RESID || OP == OP_JACOBI) {
          T bval;
          bload(bval, rb, oc[rr + 1]);
          if (OP == OP_RESID) {
            const T r = bval - acc;
            out = surf ? acc : r;
            const bool counted = !surf && so < HT_OOB;
            nsq += counted ? (double)r * (double)r : 0.0;
          } else {
            out = surf ? acc : fma(omega_invd, bval - acc, c);
          }
        }
        bstore(out, ry, so);
      }
    }
#pragma unroll
    for (int r = 0; r < J + 2; ++r) {
      xm[r] = xc[r];
      xc[r] = xp[r];
      oc[r] = op[r];
    }
  }
  if (OP == OP_RESID) {
    nsq = wave_sum(nsq);
    if (lane == 0) a.partials[w] = nsq;
  }
}

// ------------------------------------------------ ghost-exchange kernel --
// Decode p in [0, N_tri(m)) into (a, b) with rows b of length m - b.
__device__ __forceinline__ void tri_decode(int64_t p, int m, int& a, int& b) {
  const double q = 2.0 * m + 1.0;
  int bb = (int)floor((q - sqrt(q * q - 8.0 * (double)p)) * 0.5);
  auto start = [&](int r) -> int64_t { return (int64_t)r * m - (int64_t)r * (r - 1) / 2; };
  if (bb < 0) bb = 0;
  while (bb > 0 && start(bb) > p) --bb;
  while (bb + 1 < m && start(bb + 1) <= p) ++bb;
  b = bb;
  a = (int)(p - start(bb));
}

template <typename T, int OP>
__global__ __launch_bounds__(256) void k_exchange(ExchArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Lay L{a.n, a.stride, a.off_s0, a.off_s1};
  const int n = L.n;
  double nsq = 0.0;
  if (t < a.total) {
    int64_t prim;
    int gw[3] = {0, 0, 0};
    if (t < a.face_end) {
      const int64_t fp = a.face_pts;
      prim = t / fp;
      int aa, bb;
      tri_decode(t - prim * fp, n - 2, aa, bb);
      gw[1] = aa + 1;
      gw[2] = bb + 1;
      gw[0] = n - gw[1] - gw[2];
    } else if (t < a.edge_end) {
      const int64_t s = t - a.face_end;
      const int64_t ep = n - 1;
      prim = a.n_faces + s / ep;
      gw[1] = (int)(s % ep) + 1;
      gw[0] = n - gw[1];
    } else {
      prim = a.n_faces + a.n_edges + (t - a.edge_end);
      gw[0] = n;
    }
    const DevPrim P = a.prim[prim];
    const int cnt = P.inc_count;
    // slot of this point in the closure of the q-th incident cell
    auto slot_q = [&](int q) -> int64_t {
      const DevInc I = a.inc[P.inc_begin + q];
      int w[4] = {0, 0, 0, 0};
      w[I.lv[0]] = gw[0];
      if (I.lv[1] >= 0) w[I.lv[1]] = gw[1];
      if (I.lv[2] >= 0) w[I.lv[2]] = gw[2];
      return (int64_t)I.cell * L.stride + slot_of(L, w[1], w[2], w[3]);
    };
    T* y = (T*)a.y;
    const int64_t s0 = slot_q(0);
    if (OP == OP_SYNC) {
      const T v = y[s0];
      for (int q = 1; q < cnt; ++q) y[slot_q(q)] = v;
    } else if (OP == OP_FILL) {
      if (P.boundary)
        for (int q = 0; q < cnt; ++q) y[slot_q(q)] = (T)a.fill;
    } else {
      // partial rows of the incident cells, summed in cell order
      T sum = y[s0];
      for (int q = 1; q < cnt; ++q) sum += y[slot_q(q)];
      T val;
      if (P.boundary) {
        val = (OP == OP_JACOBI) ? ((const T*)a.u)[s0] : (T)0;
      } else if (OP == OP_RESID) {
        val = ((const T*)a.b)[s0] - sum;
        nsq = (double)val * (double)val;
      } else if (OP == OP_JACOBI) {
        const T invd = (T)(a.nscale * P.inv_diag_unit);
        val = ((const T*)a.u)[s0] + (T)a.omega * invd * (((const T*)a.b)[s0] - sum);
      } else {
        val = sum;
      }
      y[s0] = val;
      for (int q = 1; q < cnt; ++q) y[slot_q(q)] = val;
    }
  }
  if (OP == OP_RESID) {
    __shared__ double red[4];
    nsq = wave_sum(nsq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nsq;
    __syncthreads();
    if (threadIdx.x == 0)
      a.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ----------------------------------------------------- per-row kernels --
// Grid: x = closure row (k outer, j inner) of a cell, y = cell.  Threads run
// along i.  Used by transfers and elementwise kernels.
__device__ __forceinline__ bool decode_row(int n, int r, int& j, int& k) {
  int base = 0;
  for (k = 0; k <= n; ++k) {
    const int rows = n + 1 - k;
    if (r < base + rows) { j = r - base; return true; }
    base += rows;
  }
  return false;
}

template <typename T>
__global__ __launch_bounds__(64) void k_restrict(XferArgs a) {
  const Lay Lf{a.nf, a.stride_f, a.off_s0_f, a.off_s1_f};
  const Lay Lc{a.nc_, a.stride_c, a.off_s0_c, a.off_s1_c};
  int j, k;
  if (!decode_row(Lc.n, blockIdx.x, j, k)) return;
  const int64_t cell = blockIdx.y;
  const T* rf = (const T*)a.src + cell * Lf.stride;
  T* rc = (T*)a.dst + cell * Lc.stride;
  const ClassInfo* ci = a.cls + cell * 16;
  const int e = Lc.n - j - k;
  for (int i = threadIdx.x; i <= e; i += 64) {
    const int F0 = 2 * i, F1 = 2 * j, F2 = 2 * k;
    T s = (T)0;
#pragma unroll
    for (int d = 0; d < 15; ++d) {
      int di, dj, dk;
      stencil_offset(d, di, dj, dk);
      const int fi = F0 + di, fj = F1 + dj, fk = F2 + dk;
      if (fi < 0 || fj < 0 || fk < 0 || fi + fj + fk > Lf.n) continue;
      const int cls = point_class(Lf.n, fi, fj, fk);
      const uint8_t fl = ci[cls].flags;
      if (!(fl & kClsOwner) || (fl & kClsDirichlet)) continue;
      const T v = rf[slot_of(Lf, fi, fj, fk)];
      s += d == 0 ? v : (T)0.5 * v;
    }
    rc[slot_of(Lc, i, j, k)] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_prolong(XferArgs a) {
  const Lay Lf{a.nf, a.stride_f, a.off_s0_f, a.off_s1_f};
  const Lay Lc{a.nc_, a.stride_c, a.off_s0_c, a.off_s1_c};
  int j, k;
  if (!decode_row(Lf.n, blockIdx.x, j, k)) return;
  const int64_t cell = blockIdx.y;
  const T* ec = (const T*)a.src + cell * Lc.stride;
  T* uf = (T*)a.dst + cell * Lf.stride;
  const ClassInfo* ci = a.cls + cell * 16;
  // direction with parity p (bits i, j, k) among the seven edge directions
  const signed char dir[8][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0}, {-1, 1, 0},
                                 {0, 0, 1},  {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};
  const int e = Lf.n - j - k;
  auto coarse = [&](int ci_, int cj, int ck) -> T {
    const int cls = point_class(Lc.n, ci_, cj, ck);
    if (ci[cls].flags & kClsDirichlet) return (T)0;
    return ec[slot_of(Lc, ci_, cj, ck)];
  };
  for (int i = threadIdx.x; i <= e; i += 64) {
    const int cls = point_class(Lf.n, i, j, k);
    if (ci[cls].flags & kClsDirichlet) continue;
    const int p = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
    T v;
    if (p == 0) {
      v = coarse(i >> 1, j >> 1, k >> 1);
    } else {
      const int di = dir[p][0], dj = dir[p][1], dk = dir[p][2];
      v = (T)0.5 * (coarse((i - di) >> 1, (j - dj) >> 1, (k - dk) >> 1) +
                    coarse((i + di) >> 1, (j + dj) >> 1, (k + dk) >> 1));
    }
    uf[slot_of(Lf, i, j, k)] += v;
  }
}

// Elementwise kernels over closure rows.
template <typename T, int EOP>
__global__ __launch_bounds__(64) void k_elem(ElemArgs a) {
  const Lay L{a.n, a.stride, a.off_s0, a.off_s1};
  int j, k;
  if (!decode_row(L.n, blockIdx.x, j, k)) return;
  const int64_t cell = blockIdx.y;
  const ClassInfo* ci = a.cls + cell * 16;
  const int e = L.n - j - k;
  double acc = 0.0;
  for (int i = threadIdx.x; i <= e; i += 64) {
    const int cls = point_class(L.n, i, j, k);
    const ClassInfo c = ci[cls];
    const int64_t s = cell * L.stride + slot_of(L, i, j, k);
    if (EOP == EOP_ZERO_GUESS) {
      // first Jacobi sweep from u = 0: u = omega D^-1 b
      T* u = (T*)a.out;
      const T* b = (const T*)a.in0;
      u[s] = (c.flags & kClsDirichlet)
                 ? (T)0
                 : (T)(a.alpha * a.nscale * c.inv_diag_unit) * b[s];
    } else if (EOP == EOP_MASS) {
      ((T*)a.out)[s] = (T)(c.mass_unit * a.nscale);
    } else if (EOP == EOP_ZERO_INTERIOR) {
      if (!(c.flags & kClsDirichlet)) ((T*)a.out)[s] = (T)0;
    } else if (EOP == EOP_DOT) {
      if ((c.flags & kClsOwner) && !(c.flags & kClsDirichlet))
        acc += (double)((const T*)a.in0)[s] * (double)((const T*)a.in1)[s];
    } else if (EOP == EOP_FLAGS) {
      uint8_t f = (c.flags & kClsOwner) ? HT_SLOT_OWNER : HT_SLOT_GHOST;
      if (c.flags & kClsDirichlet) f |= HT_SLOT_DIRICHLET;
      ((uint8_t*)a.out)[s] = f;
    } else if (EOP == EOP_COORDS) {
      const double* X = a.cell_xyz + cell * 12;     // sorted by global id
      const int8_t* ord = a.cell_order + cell * 4;  // local index per sorted
      const int wl[4] = {L.n - i - j - k, i, j, k};
      double p[3] = {0.0, 0.0, 0.0};
      for (int a3 = 0; a3 < 3; ++a3) {
        double sum = 0.0;
        for (int q = 0; q < 4; ++q) {
          const int wq = wl[ord[q]];
          if (wq > 0) sum += (double)wq * X[3 * q + a3];
        }
        p[a3] = sum * a.alpha;
      }
      T* o = (T*)a.out;
      o[3 * s] = (T)p[0];
      o[3 * s + 1] = (T)p[1];
      o[3 * s + 2] = (T)p[2];
    }
  }
  if (EOP == EOP_DOT) {
    acc = wave_sum(acc);
    if (threadIdx.x == 0) a.partials[cell * gridDim.x + blockIdx.x] = acc;
  }
}

// Flat elementwise kernels over all slots (padding included).
template <typename TO, typename TI, int FOP>
__global__ __launch_bounds__(256) void k_flat(FlatArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.count) return;
  TO* o = (TO*)a.out;
  const TI* in = (const TI*)a.in;
  if (FOP == FOP_COPY) o[s] = (TO)in[s];
  else if (FOP == FOP_ADD) o[s] += (TO)in[s];
  else if (FOP == FOP_ZERO) o[s] = (TO)0;
}

// Deterministic final reduction of per-block partial sums.
__global__ __launch_bounds__(256) void k_sum_partials(const double* p,
                                                      int64_t count,
                                                      double* out, int sqrt_) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < count; t += 256) s += p[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    *out = sqrt_ ? sqrt(tot) : tot;
  }
}

// --------------------------------------------------------- coarse solve --
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gather(CoarseArgs a) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d < a.ndof) a.rhs[d] = (double)((const T*)a.b)[a.owner[d]];
}
// One wave per row of the dense inverse; the result goes to every copy.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gemv(CoarseArgs a) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= a.ndof) return;
  const double* r = a.inv + row * a.ndof;
  double s = 0.0;
  for (int64_t c = lane; c < a.ndof; c += 64) s += r[c] * a.rhs[c];
  s = wave_sum(s);
  T* u = (T*)a.u;
  for (int64_t q = a.copy_ptr[row] + lane; q < a.copy_ptr[row + 1]; q += 64)
    u[a.copy_slot[q]] = (T)s;
}

// --------------------------------------------------------- host launchers
#define HT_INST_CELL(T, OP, J) template __global__ void k_cell<T, OP, J>(CellArgs);
template <typename T, int OP>
static void launch_cell_t(const CellArgs& a, int J, hipStream_t s) {
  const dim3 grid((unsigned)(((a.nblocks + 7) / 8) * 8));
  switch (J) {
    case 4: hipLaunchKernelGGL((k_cell<T, OP, 4>), grid, dim3(64), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_cell<T, OP, 8>), grid, dim3(64), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_cell<T, OP, 16>), grid, dim3(64), 0, s, a); break;
    default: hipLaunchKernelGGL((k_cell<T, OP, 8>), grid, dim3(64), 0, s, a); break;
  }
}

void launch_cell(int dtype, int op, int J, const CellArgs& a, hipStream_t s) {
  if (dtype == HT_F64) {
    if (op == OP_APPLY) launch_cell_t<double, OP_APPLY>(a, J, s);
    else if (op == OP_RESID) launch_cell_t<double, OP_RESID>(a, J, s);
    else launch_cell_t<double, OP_JACOBI>(a, J, s);
  } else {
    if (op == OP_APPLY) launch_cell_t<float, OP_APPLY>(a, J, s);
    else if (op == OP_RESID) launch_cell_t<float, OP_RESID>(a, J, s);
    else launch_cell_t<float, OP_JACOBI>(a, J, s);
  }
}

template <typename T>
static void launch_exchange_t(int op, const ExchArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.total + 255) / 256));
  switch (op) {
    case OP_APPLY: hipLaunchKernelGGL((k_exchange<T, OP_APPLY>), grid, dim3(256), 0, s, a); break;
    case OP_RESID: hipLaunchKernelGGL((k_exchange<T, OP_RESID>), grid, dim3(256), 0, s, a); break;
    case OP_JACOBI: hipLaunchKernelGGL((k_exchange<T, OP_JACOBI>), grid, dim3(256), 0, s, a); break;
    case OP_SYNC: hipLaunchKernelGGL((k_exchange<T, OP_SYNC>), grid, dim3(256), 0, s, a); break;
    case OP_FILL: hipLaunchKernelGGL((k_exchange<T, OP_FILL>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_exchange<T, OP_APPLY>), grid, dim3(256), 0, s, a); break;
  }
}
void launch_exchange(int dtype, int op, const ExchArgs& a, hipStream_t s) {
  if (a.total <= 0) return;
  if (dtype == HT_F64) launch_exchange_t<double>(op, a, s);
  else launch_exchange_t<float>(op, a, s);
}

void launch_restrict(int dtype, const XferArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)n_tri(a.nc_ + 1), (unsigned)a.ncells);
  if (dtype == HT_F64) hipLaunchKernelGGL(k_restrict<double>, grid, dim3(64), 0, s, a);
  else hipLaunchKernelGGL(k_restrict<float>, grid, dim3(64), 0, s, a);
}
void launch_prolong(int dtype, const XferArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)n_tri(a.nf + 1), (unsigned)a.ncells);
  if (dtype == HT_F64) hipLaunchKernelGGL(k_prolong<double>, grid, dim3(64), 0, s, a);
  else hipLaunchKernelGGL(k_prolong<float>, grid, dim3(64), 0, s, a);
}

template <typename T>
static void launch_elem_t(int eop, const ElemArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)n_tri(a.n + 1), (unsigned)a.ncells);
  switch (eop) {
    case EOP_ZERO_GUESS: hipLaunchKernelGGL((k_elem<T, EOP_ZERO_GUESS>), grid, dim3(64), 0, s, a); break;
    case EOP_MASS: hipLaunchKernelGGL((k_elem<T, EOP_MASS>), grid, dim3(64), 0, s, a); break;
    case EOP_ZERO_INTERIOR: hipLaunchKernelGGL((k_elem<T, EOP_ZERO_INTERIOR>), grid, dim3(64), 0, s, a); break;
    case EOP_DOT: hipLaunchKernelGGL((k_elem<T, EOP_DOT>), grid, dim3(64), 0, s, a); break;
    case EOP_FLAGS: hipLaunchKernelGGL((k_elem<T, EOP_FLAGS>), grid, dim3(64), 0, s, a); break;
    case EOP_COORDS: hipLaunchKernelGGL((k_elem<T, EOP_COORDS>), grid, dim3(64), 0, s, a); break;
  }
}
void launch_elem(int dtype, int eop, const ElemArgs& a, hipStream_t s) {
  if (dtype == HT_F64) launch_elem_t<double>(eop, a, s);
  else launch_elem_t<float>(eop, a, s);
}

void launch_flat(int dto, int dti, int fop, const FlatArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.count + 255) / 256));
  if (a.count <= 0) return;
#define HT_FLAT(TO, TI)                                                        \
  switch (fop) {                                                               \
    case FOP_COPY: hipLaunchKernelGGL((k_flat<TO, TI, FOP_COPY>), grid, dim3(256), 0, s, a); break; \
    case FOP_ADD: hipLaunchKernelGGL((k_flat<TO, TI, FOP_ADD>), grid, dim3(256), 0, s, a); break;   \
    case FOP_ZERO: hipLaunchKernelGGL((k_flat<TO, TI, FOP_ZERO>), grid, dim3(256), 0, s, a); break; \
  }
  if (dto == HT_F64 && dti == HT_F64) { HT_FLAT(double, double) }
  else if (dto == HT_F64 && dti == HT_F32) { HT_FLAT(double, float) }
  else if (dto == HT_F32 && dti == HT_F64) { HT_FLAT(float, double) }
  else { HT_FLAT(float, float) }
#undef HT_FLAT
}

void launch_sum_partials(const double* p, int64_t count, double* out, bool sq,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, p, count, out,
                     sq ? 1 : 0);
}

void launch_coarse(int dtype, const CoarseArgs& a, hipStream_t s) {
  const dim3 g1((unsigned)((a.ndof + 255) / 256)), g2((unsigned)((a.ndof + 3) / 4));
  if (a.ndof <= 0) return;
  if (dtype == HT_F64) {
    hipLaunchKernelGGL(k_coarse_gather<double>, g1, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_coarse_gemv<double>, g2, dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_coarse_gather<float>, g1, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_coarse_gemv<float>, g2, dim3(256), 0, s, a);
  }
}

void launch_lane_selftest(int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lane_selftest, dim3(1), dim3(64), 0, s, out);
}

}  // namespace ht
