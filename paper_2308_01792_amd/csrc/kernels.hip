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

#include "device.hpp"

namespace ht {

// Self-test of the lane exchange: out[l] = prev(l), out[64 + l] = next(l).
__global__ void k_lane_selftest(int* out) {
  const int l = threadIdx.x;
  out[l] = (int)lane_prev((double)(l + 1));
  out[64 + l] = (int)lane_next((float)(l + 1));
}

// In-face offsets of the face i = 0 (class 1) and of the slanted face
// i + j + k = n (class 8), as indices into the 15-offset list.
__constant__ int kInFace1[7] = {0, 3, 4, 5, 6, 11, 12};
__constant__ int kInFace8[7] = {0, 7, 8, 9, 10, 11, 12};

// One wave = one tile of 64 consecutive i (62 outputs, one halo lane on each
// side) and J rows j0..j0+J-1, marching k upwards with the planes k-1, k,
// k+1 of rows j0-1..j0+J in registers; i +- 1 neighbours come from DPP.  The
// loads of plane k+2 are issued before plane k is computed, so memory
// latency overlaps one plane of arithmetic.
//
// Points on the cell's faces get the cell's partial row.  On rows with
// j >= 1, k >= 1 and line end e >= 2 ("generic" rows) only two lanes are
// surface points: i = 0 (face i = 0) and i = e (slanted face).  The interior
// formula evaluated with zero outside the closure differs from their exact
// partial row by a 7-term sum over the in-face offsets only, which the one
// tile holding the lane adds.  Rows with j == 0, k == 0 or e <= 1 take
// exact per-lane class weights from LDS.
//
// OP_RESTRICT runs the same march over a fine residual with the fixed
// stencil of P^T (1 at the centre, 1/2 on the 14 edge neighbours) and
// evaluates it at even (i, j, k) only, writing the coarse point (i,j,k)/2.
// Fine points this cell does not own (or Dirichlet points) read as zero, so
// every fine micro-vertex is restricted by exactly one cell and shared coarse
// points receive partial sums for the ghost exchange.
template <typename T, int OP, int J>
__global__ __launch_bounds__(64 * kCellWaves) void k_cell(CellArgs a) {
  constexpr bool RESTR = (OP == OP_RESTRICT);
  __shared__ T wtab[16 * 15];
  // in-face parts of (class weights - interior weights) on the faces i = 0
  // (class 1, offsets 0 3 4 5 6 11 12) and i + j + k = n (class 8, offsets
  // 0 7 8 9 10 11 12), in that order
  __shared__ T dwtab[14];
  // A workgroup is kCellWaves waves on adjacent tiles of one cell, marching
  // in near lockstep on one CU: stacked in j (rows j0 .. j0 + kCellWaves J
  // - 1), each wave's halo rows are its neighbours' rows, fetched once; side
  // by side in i (a.waves_in_i), each row is one contiguous run.
  // XCD-aware block order: block b runs on XCD b % 8; give each XCD a
  // contiguous run of (cell, tile group) work so neighbouring groups share
  // an L2.
  const int64_t nb = a.nblocks;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t wb = (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
  if (wb >= nb) return;
  const int64_t cell = wb / a.ntiles;
  // tile (i0, j0 | k0 << 16): the march covers planes k0 .. k0 + segment - 1
  const int2 tile_raw = a.tiles[wb % a.ntiles];
  const int k0 = tile_raw.y >> 16;
  const int2 tile = make_int2(tile_raw.x, tile_raw.y & 0xffff);
  const int lane = threadIdx.x & 63;
  // wave index, uniform over the wave: say so, so that the row bookkeeping
  // derived from it lives in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t w = wb * kCellWaves + wave;  // partial-sum slot of this wave
  const bool in_i = a.waves_in_i != 0;
  const int i0 = tile.x + (in_i ? 62 * wave : 0), j0 = tile.y + (in_i ? 0 : wave * J);
  const int n = a.n;
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const int64_t ostride = RESTR ? a.stride_out : a.stride;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
  const __amdgpu_buffer_rsrc_t ry =
      make_rsrc((T*)a.y + cell * ostride, ostride * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rb =
      make_rsrc(a.b ? (const T*)a.b + cell * a.stride : (const T*)a.y, bytes);
  constexpr bool CHEB = (OP == OP_CHEB);
  const __amdgpu_buffer_rsrc_t rd =
      make_rsrc(CHEB ? (T*)a.d + cell * a.stride : (T*)a.y, bytes);
  T w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0, w6 = 0, w7 = 0, w8 = 0,
    w9 = 0, w10 = 0, w11 = 0, w12 = 0, w13 = 0, w14 = 0;
  unsigned own16 = 0;
  if (!RESTR) {
    const T* wc = (const T*)a.w + cell * 240;
    for (int t = threadIdx.x; t < 240; t += 64 * kCellWaves) wtab[t] = wc[t];
    __syncthreads();
    if (threadIdx.x < 14) {
      const int t = threadIdx.x;
      const int d = t < 7 ? kInFace1[t] : kInFace8[t - 7];
      dwtab[t] = wtab[(t < 7 ? 1 : 8) * 15 + d] - wtab[d];
    }
    __syncthreads();
    // interior weights from LDS: they stay in VGPRs and leave the scalar
    // registers to the row bookkeeping
    w0 = wtab[0]; w1 = wtab[1]; w2 = wtab[2]; w3 = wtab[3]; w4 = wtab[4];
    w5 = wtab[5]; w6 = wtab[6]; w7 = wtab[7]; w8 = wtab[8]; w9 = wtab[9];
    w10 = wtab[10]; w11 = wtab[11]; w12 = wtab[12]; w13 = wtab[13];
    w14 = wtab[14];
  } else {
    const uint8_t fl = lane < 16 ? a.cls[cell * 16 + lane].flags : 0;
    own16 = (unsigned)__ballot((fl & kClsOwner) && !(fl & kClsDirichlet)) & 0xffffu;
  }
  const T omega_invd =
      RESTR ? (T)0 : (T)(a.omega * a.nscale * a.cls[cell * 16].inv_diag_unit);
  const int off_s0 = (int)a.off_s0, off_s1 = (int)a.off_s1;

  const int i = i0 - 1 + lane;
  const bool is0 = (i == 0);
  const unsigned out_mask = (lane >= 1 && lane <= 62) ? 0u : HT_OOB;
  // Offsets of the rows j0-1 .. j0+J of plane kk.  Row j of a plane: main
  // block base mb(j) (element of i = 0 if it were stored there), S0 and S1
  // entries sa(j), sb(j); consecutive rows differ by the main-block row
  // length (n-1-kk-j) and by 1 in S0/S1.
  // Scalar cursor over the planes to load: element bases of plane ck in the
  // main block (minus one), in S0 and in S1 (closure layout of index.hpp).
  // Each plane advances them by its own size, so no plane recomputes the
  // tetrahedral numbers.
  const int wm = n - 1;  // width of the main block's polytope
  // (started at plane k0 - 1, or 0, from the closed forms of the plane sizes)
  int ck = k0 > 0 ? k0 - 1 : 0;
  int cmb = -1 + tet32(wm) - tet32(wm - ck), csa = off_s0 + tri32(n + 1) - tri32(n + 1 - ck),
      csb = off_s1 + tri32(n) - tri32(n - ck);
  auto advance = [&]() {
    const int wk = wm - ck;
    cmb += wk > 0 ? wk * (wk + 1) / 2 : 0;
    csa += n + 1 - ck;
    csb += n - ck;
    ++ck;
  };
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
      const bool row_ok = j >= 0 && e >= 0;
      int el = (i == e) ? sb : mb + i;
      el = is0 ? sa : el;
      o[r] = (row_ok && (unsigned)i <= (unsigned)e) ? (unsigned)el * (unsigned)sizeof(T)
                                                    : HT_OOB;
      const bool inc = j >= 0;
      mb += inc ? wk - j : 0;
      sa += inc ? 1 : 0;
      sb += inc ? 1 : 0;
    }
    advance();
  };
  // restriction: fine points not owned by this cell read as zero
  auto mask_plane = [&](int kk, T (&v)[J + 2]) {
    if (RESTR) {
#pragma unroll
      for (int r = 0; r < J + 2; ++r) {
        const int j = j0 - 1 + r;
        const int cls = (int)is0 | ((j == 0) << 1) | ((kk == 0) << 2) | ((i == n - j - kk) << 3);
        v[r] = ((own16 >> cls) & 1u) ? v[r] : (T)0;
      }
    }
  };

  constexpr bool FUSE = (OP == OP_RESID32X);
  constexpr bool R32 = (OP == OP_RESID32 || FUSE);
  constexpr bool NEED_B =
      (OP == OP_RESID || OP == OP_JACOBI || R32 || OP == OP_CHEB);
  const __amdgpu_buffer_rsrc_t ry32 = make_rsrc(
      R32 ? (float*)a.y32 + cell * a.stride : (float*)a.y,
      a.stride * (int64_t)sizeof(float));
  // OP_RESID32X: the first sweep of the next correction
  const __amdgpu_buffer_rsrc_t ref = make_rsrc(
      FUSE ? (float*)a.efirst + cell * a.stride : (float*)a.y,
      a.stride * (int64_t)sizeof(float));
  double nsq = 0.0;
  // One plane step: compute plane k from (pm, pc, pp) = planes k-1, k, k+1
  // while the loads of plane k+2 go into pn.  The k loop is unrolled by four
  // so the four plane buffers rotate by renaming, not by register moves.
  auto step = [&](int k, T (&pm)[J + 2], T (&pc)[J + 2], T (&pp)[J + 2],
                  T (&pn)[J + 2], unsigned (&oc)[J + 2], unsigned (&op)[J + 2],
                  unsigned (&on)[J + 2], T (&bc)[J], T (&bp)[J], T (&dc)[J],
                  T (&dp)[J]) {
    plane_offsets(on);
#pragma unroll
    for (int r = 0; r < J + 2; ++r) bload(pn[r], rx, on[r]);
    if (NEED_B) {
#pragma unroll
      for (int r = 0; r < J; ++r) bload(bp[r], rb, op[r + 1]);
    }
    if (CHEB) {
      // the first step of an application has c1 = 0: d is not read
#pragma unroll
      for (int r = 0; r < J; ++r) dp[r] = (T)0;
      if (a.c1 != 0.0) {
#pragma unroll
        for (int r = 0; r < J; ++r) bload(dp[r], rd, op[r + 1]);
      }
    }
    mask_plane(k + 1, pp);
    if (RESTR && (k & 1)) return;
#pragma unroll
    for (int rr = 0; rr < J; ++rr) {
      const int j = j0 + rr;
      const int e = n - j - k;
      if (RESTR && (rr & 1)) continue;
      if (e < i0) continue;
      const T c = pc[rr + 1];
      if (RESTR) {
        const T v1 = lane_next(c), v2 = lane_prev(c);
        const T v3 = pc[rr + 2], v4 = pc[rr];
        const T v5 = pp[rr + 1], v6 = pm[rr + 1];
        const T v7 = lane_prev(pc[rr + 2]), v8 = lane_next(pc[rr]);
        const T v9 = lane_prev(pp[rr + 1]), v10 = lane_next(pm[rr + 1]);
        const T v11 = pp[rr], v12 = pm[rr + 2];
        const T v13 = lane_next(pp[rr]), v14 = lane_prev(pm[rr + 2]);
        // P^T at the even fine point (i, j, k) -> coarse (i, j, k) / 2
        const T nb14 = ((v1 + v2) + (v3 + v4)) + ((v5 + v6) + (v7 + v8)) +
                       ((v9 + v10) + (v11 + v12)) + (v13 + v14);
        const T val = fma((T)0.5, nb14, c);
        const int nc = n >> 1, jc = j >> 1, kc = k >> 1, ec = nc - jc - kc;
        const int mbc = (int)tw32(nc - 1, 0, jc, kc) - 1;
        const int sac = (int)a.off_s0_out + (int)t2w32(nc + 1, jc, kc);
        const int sbc = (int)a.off_s1_out + (int)t2w32(nc, jc, kc);
        const int ic = i >> 1;
        int el = (ic == ec) ? sbc : mbc + ic;
        el = (ic == 0) ? sac : el;
        const bool ok = ((i & 1) == 0) && out_mask == 0u && i >= 0 && i <= e;
        bstore(val, ry, ok ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB);
        continue;
      }
      // Interior weights are the same on every lane, and a lane shift is
      // linear: the four terms taken at i + 1 (offsets 1, 8, 10, 13) are
      // summed first and shifted once, likewise the four at i - 1 (offsets
      // 2, 7, 9, 14): 2 shifts per row instead of 8.
      const T sn = fma(w13, pp[rr], fma(w10, pm[rr + 1], fma(w8, pc[rr], w1 * c)));
      const T sp = fma(w14, pm[rr + 2], fma(w9, pp[rr + 1], fma(w7, pc[rr + 2], w2 * c)));
      T acc = w0 * c;
      acc = fma(w3, pc[rr + 2], acc); acc = fma(w4, pc[rr], acc);
      acc = fma(w5, pp[rr + 1], acc); acc = fma(w6, pm[rr + 1], acc);
      acc = fma(w11, pp[rr], acc); acc = fma(w12, pm[rr + 2], acc);
      acc += lane_next(sn);
      acc += lane_prev(sp);
      bool surf;
      if (j == 0 || k == 0 || e <= 1) {
        // per-lane class weights: shift every neighbour individually
        const T v1 = lane_next(c), v2 = lane_prev(c);
        const T v3 = pc[rr + 2], v4 = pc[rr];
        const T v5 = pp[rr + 1], v6 = pm[rr + 1];
        const T v7 = lane_prev(pc[rr + 2]), v8 = lane_next(pc[rr]);
        const T v9 = lane_prev(pp[rr + 1]), v10 = lane_next(pm[rr + 1]);
        const T v11 = pp[rr], v12 = pm[rr + 2];
        const T v13 = lane_next(pp[rr]), v14 = lane_prev(pm[rr + 2]);
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
        // generic row: the interior formula with zero outside the closure is
        // the cell's partial row everywhere except at i = 0 and i = e, where
        // the in-face weights differ.  Only the tile holding that lane adds
        // the difference (a uniform branch).
        surf = is0 || (i == e);
        // Residual and Jacobi hold b as well: there the weights are read
        // where used, indexed by k >> 30 (always 0, k < 2^30) so that they
        // are not hoisted out of the plane loop into 28 registers held for
        // the whole march (which would cost a wave per SIMD).  The apply has
        // the registers to spare and keeps them hoisted.
        const T* dw = dwtab + (NEED_B ? (k >> 30) : 0);
        if (i0 == 0) {
          T c1 = dw[0] * c;
          c1 = fma(dw[1], pc[rr + 2], c1); c1 = fma(dw[2], pc[rr], c1);
          c1 = fma(dw[3], pp[rr + 1], c1); c1 = fma(dw[4], pm[rr + 1], c1);
          c1 = fma(dw[5], pp[rr], c1); c1 = fma(dw[6], pm[rr + 2], c1);
          acc += is0 ? c1 : (T)0;
        }
        if (e >= i0 && e <= i0 + 61) {
          T c8 = dw[7] * c;
          c8 = fma(dw[12], pp[rr], c8); c8 = fma(dw[13], pm[rr + 2], c8);
          c8 += lane_next(fma(dw[9], pc[rr], dw[11] * pm[rr + 1]));
          c8 += lane_prev(fma(dw[8], pc[rr + 2], dw[10] * pp[rr + 1]));
          acc += (i == e) ? c8 : (T)0;
        }
      }
      const unsigned so = oc[rr + 1] | out_mask;
      T out = acc;
      if (NEED_B) {
        const T bval = bc[rr];
        // both epilogues form r = b - A u and add |r|^2 of the points this
        // wave finishes to the norm partials (a Jacobi sweep thereby also
        // yields the residual norm of the iterate it starts from)
        const T r = bval - acc;
        const bool counted = !surf && so < HT_OOB;
        nsq += counted ? (double)r * (double)r : 0.0;
        if (OP == OP_RESID) {
          out = surf ? acc : r;
        } else if (OP == OP_JACOBI) {
          out = surf ? acc : fma(omega_invd, r, c);
        } else if (OP == OP_CHEB) {
          // omega = 1: omega_invd is the inverse diagonal
          const T dn = fma((T)a.c1, dc[rr], (T)a.c2 * (omega_invd * r));
          out = surf ? acc : c + dn;
          bstore(dn, rd, surf ? HT_OOB : so);
        }
        if (R32) {
          // finished points: FP32 residual (element offset = so / 2);
          // surface points: the FP64 partial row, completed by the exchange
          bstore((float)r, ry32, surf ? HT_OOB : so >> 1);
          bstore(acc, ry, surf ? so : HT_OOB);
          if (FUSE) {
            // the next correction's first sweep at the finished points, in
            // FP32 as the separate zero-guess sweep forms it (the factor
            // rounded to FP32 times the FP32 residual: bit for bit)
            bstore((float)omega_invd * (float)r, ref, surf ? HT_OOB : so >> 1);
          }
          continue;
        }
      }
      bstore(out, ry, so);
    }
  };

  T PA[J + 2], PB[J + 2], PC[J + 2], PD[J + 2];
  unsigned OA[J + 2], OB[J + 2], OC[J + 2], OD[J + 2];
  T BA[J], BB[J], DA[J], DB[J];
  if (k0 > 0) {
    plane_offsets(OA);
#pragma unroll
    for (int r = 0; r < J + 2; ++r) bload(PA[r], rx, OA[r]);
  } else {
#pragma unroll
    for (int r = 0; r < J + 2; ++r) {
      PA[r] = (T)0;
      OA[r] = HT_OOB;
    }
  }
  plane_offsets(OB);
  plane_offsets(OC);
#pragma unroll
  for (int r = 0; r < J + 2; ++r) {
    bload(PB[r], rx, OB[r]);
    bload(PC[r], rx, OC[r]);
  }
  if (NEED_B) {
#pragma unroll
    for (int r = 0; r < J; ++r) bload(BA[r], rb, OB[r + 1]);
  }
  if (CHEB) {
#pragma unroll
    for (int r = 0; r < J; ++r) DA[r] = (T)0;
    if (a.c1 != 0.0) {
#pragma unroll
      for (int r = 0; r < J; ++r) bload(DA[r], rd, OB[r + 1]);
    }
  }
  if (k0 > 0) mask_plane(k0 - 1, PA);
  mask_plane(k0, PB);
  const int kcol = n - i0 - j0;
  const int kmax = kcol < k0 + a.kseg - 1 ? kcol : k0 + a.kseg - 1;
  for (int k = k0; k <= kmax; k += 4) {
    step(k, PA, PB, PC, PD, OB, OC, OD, BA, BB, DA, DB);
    if (k + 1 > kmax) break;
    step(k + 1, PB, PC, PD, PA, OC, OD, OA, BB, BA, DB, DA);
    if (k + 2 > kmax) break;
    step(k + 2, PC, PD, PA, PB, OD, OA, OB, BA, BB, DA, DB);
    if (k + 3 > kmax) break;
    step(k + 3, PD, PA, PB, PC, OA, OB, OC, BB, BA, DB, DA);
  }
  if (NEED_B) {
    nsq = wave_sum(nsq);
    if (lane == 0) a.partials[w] = nsq;
  }
}

// ------------------------------------------------ ghost-exchange kernel --
// Decode p in [0, N_tri(m)) into (a, b) with rows b of length m - b, for
// m <= 2046: row b starts at b m - b (b - 1) / 2; the FP32 root of the
// quadratic is exact to one row (all operands are integers below 2^24), and
// one comparison each way corrects it.
__device__ __forceinline__ void tri_decode(int p, int m, int& a, int& b) {
  const float q = 2.0f * (float)m + 1.0f;
  int bb = (int)((q - __builtin_sqrtf(q * q - 8.0f * (float)p)) * 0.5f);
  bb = bb < 0 ? 0 : (bb > m - 1 ? m - 1 : bb);
  auto start = [&](int r) { return r * m - ((r * (r - 1)) >> 1); };
  if (start(bb) > p) --bb;
  else if (bb + 1 < m && start(bb + 1) <= p) ++bb;
  b = bb;
  a = p - start(bb);
}

// Interior points of one face (one or two copies), kExchFacePts per thread:
// the points chunk * 256 kExchFacePts + 256 u + thread.  All their loads are
// issued before any store, so that one thread has several independent loads
// in flight (the per-point chain of loads is what bounds the exchange).
// Same arithmetic as the generic path below; returns the thread's |r|^2.
template <typename T, int OP>
__device__ __forceinline__ double exch_face(const ExchArgs& a, const Lay& L, int64_t fl,
                                            int chunk, int tid) {
  constexpr int U = kExchFacePts;
  constexpr bool NEED_B = OP == OP_RESID || OP == OP_RESID32 || OP == OP_RESID32X ||
                          OP == OP_JACOBI || OP == OP_JACOBIADD || OP == OP_CHEB;
  constexpr bool NEED_U = OP == OP_JACOBI || OP == OP_JACOBIADD || OP == OP_CHEB;
  const int n = L.n;
  const DevPrim P = a.prim[a.prim_f0 + fl];
  const int cnt = P.inc_count;  // 2, or 1 on the domain boundary
  const DevInc I0 = a.inc[P.inc_begin];
  const DevInc I1 = a.inc[P.inc_begin + (cnt > 1 ? 1 : 0)];
  auto slot = [&](const DevInc& I, const int (&gw)[3]) -> int64_t {
    int w[4] = {0, 0, 0, 0};
    w[I.lv[0]] = gw[0];
    w[I.lv[1]] = gw[1];
    w[I.lv[2]] = gw[2];
    return (int64_t)I.cell * L.stride + slot_of(L, w[1], w[2], w[3]);
  };
  T* y = (T*)a.y;
  bool ok[U];
  int64_t s0[U], s1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = chunk * (256 * U) + 256 * u + tid;
    ok[u] = p < a.face_pts;
    int aa = 0, bb = 0;
    tri_decode(ok[u] ? p : 0, n - 2, aa, bb);
    const int gw[3] = {n - aa - bb - 2, aa + 1, bb + 1};
    s0[u] = slot(I0, gw);
    s1[u] = cnt > 1 ? slot(I1, gw) : s0[u];
  }
  // loads: the copies' values (partial rows, or the value to copy), b, u, d
  T y0[U], y1[U], bv[U], uv[U], dv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    y0[u] = y1[u] = bv[u] = uv[u] = dv[u] = (T)0;
    if (!ok[u]) continue;
    if (OP != OP_FILL) y0[u] = y[s0[u]];
    if (OP != OP_SYNC && OP != OP_FILL && cnt > 1) y1[u] = y[s1[u]];
    if (NEED_B) bv[u] = ((const T*)a.b)[s0[u]];
    if (NEED_U) uv[u] = ((const T*)a.u)[s0[u]];
    if (OP == OP_CHEB && a.c1 != 0.0) dv[u] = ((const T*)a.d)[s0[u]];
  }
  double nsq = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!ok[u]) continue;
    if (OP == OP_SYNC) {
      if (cnt > 1) y[s1[u]] = y0[u];
      continue;
    }
    if (OP == OP_FILL) {
      if (P.boundary) {
        y[s0[u]] = (T)a.fill;
        if (cnt > 1) y[s1[u]] = (T)a.fill;
      }
      continue;
    }
    // partial rows of the incident cells, summed in cell order
    T sum = (T)0;
    sum += y0[u];
    if (cnt > 1) sum += y1[u];
    T val;
    if (P.boundary) {
      val = NEED_U ? uv[u] : (T)0;
    } else if (OP == OP_RESID || OP == OP_RESID32 || OP == OP_RESID32X) {
      val = bv[u] - sum;
      nsq += (double)val * (double)val;
    } else if (OP == OP_JACOBI || OP == OP_JACOBIADD) {
      const T invd = (T)(a.nscale * P.inv_diag_unit);
      const T r = bv[u] - sum;
      nsq += (double)r * (double)r;
      val = uv[u] + (T)a.omega * invd * r;
    } else if (OP == OP_CHEB) {
      const T invd = (T)(a.nscale * P.inv_diag_unit);
      const T r = bv[u] - sum;
      nsq += (double)r * (double)r;
      T* d = (T*)a.d;
      const T dn = fma((T)a.c1, a.c1 != 0.0 ? dv[u] : (T)0, (T)a.c2 * (invd * r));
      val = uv[u] + dn;
      d[s0[u]] = dn;
      if (cnt > 1) d[s1[u]] = dn;
    } else {
      val = sum;
    }
    if (OP == OP_RESID32 || OP == OP_RESID32X) {
      float* y32 = (float*)a.y32;
      y32[s0[u]] = (float)val;
      if (cnt > 1) y32[s1[u]] = (float)val;
      if (OP == OP_RESID32X) {
        const float e = (float)(a.omega * a.nscale * P.inv_diag_unit) * (float)val;
        float* ef = (float*)a.efirst;
        ef[s0[u]] = e;
        if (cnt > 1) ef[s1[u]] = e;
      }
    } else if (OP == OP_JACOBIADD) {
      double* ua = a.uadd;
      ua[s0[u]] += (double)val;
      if (cnt > 1) ua[s1[u]] += (double)val;
    } else {
      y[s0[u]] = val;
      if (cnt > 1) y[s1[u]] = val;
    }
  }
  return nsq;
}

// One thread per micro-vertex shared by several cells: blocks of one face's
// interior points (kExchFacePts per thread), then of one edge's, then of the
// vertices.  Sums the partial rows of all incident cells in cell order,
// applies the epilogue of OP and writes every copy.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_exchange(ExchArgs a) {
  const Lay L{a.n, a.stride, a.off_s0, a.off_s1};
  const int n = L.n;
  const int tid = (int)threadIdx.x;
  // the block's primitive: uniform, so the divisions are scalar
  const int64_t blk = blockIdx.x;
  int64_t prim = 0;
  bool valid = false;
  int gw[3] = {0, 0, 0};
  double nsq = 0.0;
  if (blk < a.fblk) {
    const int64_t fl = blk / a.bpf;  // face within the range
    nsq = exch_face<T, OP>(a, L, fl, (int)(blk - fl * a.bpf), tid);
  } else if (blk < a.fblk + a.eblk) {
    const int64_t eb = blk - a.fblk;
    const int64_t el = eb / a.bpe;
    const int s = (int)(eb - el * a.bpe) * 256 + tid;
    prim = a.prim_e0 + el;
    valid = s < n - 1;
    gw[1] = s + 1;
    gw[0] = n - gw[1];
  } else {
    const int64_t v = (blk - a.fblk - a.eblk) * 256 + tid;
    prim = a.prim_v0 + v;
    valid = v < a.nverts;
    gw[0] = n;
  }
  if (valid) {
    const DevPrim P = a.prim[prim];
    const int cnt = P.inc_count;
    // local index of this point in the q-th incident cell
    auto local_q = [&](int q, int& i, int& j, int& k) {
      const DevInc I = a.inc[P.inc_begin + q];
      int w[4] = {0, 0, 0, 0};
      w[I.lv[0]] = gw[0];
      if (I.lv[1] >= 0) w[I.lv[1]] = gw[1];
      if (I.lv[2] >= 0) w[I.lv[2]] = gw[2];
      i = w[1]; j = w[2]; k = w[3];
      return I;
    };
    auto slot_q = [&](int q) -> int64_t {
      int i, j, k;
      const DevInc I = local_q(q, i, j, k);
      return (int64_t)I.cell * L.stride + slot_of(L, i, j, k);
    };
    T* y = (T*)a.y;
    // slots of the first two copies (all of a face's) formed once
    const int64_t s0 = slot_q(0);
    const int64_t s1 = cnt > 1 ? slot_q(1) : s0;
    auto slot_c = [&](int q) -> int64_t { return q == 0 ? s0 : (q == 1 ? s1 : slot_q(q)); };
    if (OP == OP_SYNC) {
      const T v = y[s0];
      for (int q = 1; q < cnt; ++q) y[slot_c(q)] = v;
    } else if (OP == OP_FILL) {
      if (P.boundary)
        for (int q = 0; q < cnt; ++q) y[slot_c(q)] = (T)a.fill;
    } else {
      // partial rows of the incident cells, summed in cell order
      T sum = (T)0;
      for (int q = 0; q < cnt; ++q) sum += y[slot_c(q)];
      T val;
      if (P.boundary) {
        val = (OP == OP_JACOBI || OP == OP_JACOBIADD || OP == OP_CHEB) ? ((const T*)a.u)[s0]
                                                                      : (T)0;
      } else if (OP == OP_RESID || OP == OP_RESID32 || OP == OP_RESID32X) {
        val = ((const T*)a.b)[s0] - sum;
        nsq = (double)val * (double)val;
      } else if (OP == OP_JACOBI || OP == OP_JACOBIADD) {
        const T invd = (T)(a.nscale * P.inv_diag_unit);
        const T r = ((const T*)a.b)[s0] - sum;
        nsq = (double)r * (double)r;
        val = ((const T*)a.u)[s0] + (T)a.omega * invd * r;
      } else if (OP == OP_CHEB) {
        const T invd = (T)(a.nscale * P.inv_diag_unit);
        const T r = ((const T*)a.b)[s0] - sum;
        nsq = (double)r * (double)r;
        T* d = (T*)a.d;
        const T dn = fma((T)a.c1, a.c1 != 0.0 ? d[s0] : (T)0, (T)a.c2 * (invd * r));
        val = ((const T*)a.u)[s0] + dn;
        d[s0] = dn;
        for (int q = 1; q < cnt; ++q) d[slot_c(q)] = dn;
      } else {
        val = sum;
      }
      if (OP == OP_RESID32 || OP == OP_RESID32X) {
        float* y32 = (float*)a.y32;
        y32[s0] = (float)val;
        for (int q = 1; q < cnt; ++q) y32[slot_c(q)] = (float)val;
        if (OP == OP_RESID32X) {
          // first zero-guess sweep of the next correction (0 on the
          // Dirichlet boundary, where val is 0)
          // (FP32 factor times FP32 residual, as the zero-guess sweep)
          const float e = (float)(a.omega * a.nscale * P.inv_diag_unit) * (float)val;
          float* ef = (float*)a.efirst;
          ef[s0] = e;
          for (int q = 1; q < cnt; ++q) ef[slot_c(q)] = e;
        }
      } else if (OP == OP_JACOBIADD) {
        double* ua = a.uadd;
        ua[s0] += (double)val;
        for (int q = 1; q < cnt; ++q) ua[slot_c(q)] += (double)val;
      } else {
        y[s0] = val;
        for (int q = 1; q < cnt; ++q) y[slot_c(q)] = val;
      }
    }
  }
  if (OP == OP_RESID || OP == OP_JACOBI || OP == OP_RESID32 || OP == OP_CHEB ||
      OP == OP_RESID32X || OP == OP_JACOBIADD) {
    __shared__ double red[4];
    nsq = wave_sum(nsq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nsq;
    __syncthreads();
    if (threadIdx.x == 0)
      a.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
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

// Deterministic two-level reduction of per-block partial sums: stage 1
// writes 256 strided sums to p + count, stage 2 adds them in order.
__global__ __launch_bounds__(256) void k_sum_stage1(const double* p,
                                                    int64_t count, double* q) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += 256 * 256)
    s += p[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) q[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(256) void k_sum_stage2(const double* q,
                                                    double* out, int sqrt_) {
  __shared__ double red[4];
  double s = wave_sum(q[threadIdx.x]);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    *out = sqrt_ ? sqrt(tot) : tot;
  }
}

// Segmented sums of norm partials, one wave per segment, fixed order.
__global__ __launch_bounds__(256) void k_seg_sum(SegArgs a) {
  const int seg = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (seg >= a.nseg) return;
  double s = 0.0;
  for (int64_t q = a.lo[seg] + lane; q < a.hi[seg]; q += 64) s += a.p[q];
  s = wave_sum(s);
  if (lane == 0) a.out[seg] = s;
}

// --------------------------------------------------------- coarse solve --
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gather(CoarseArgs a) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d < a.ndof) a.rhs[d] = (double)((const T*)a.b)[a.owner[d]];
}
// One wave per row of the block-diagonal inverse; the result goes to every
// copy.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gemv(CoarseArgs a) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= a.ndof) return;
  const int b = a.row_blk[row];
  const int64_t d0 = a.blk_dof[b], nb = a.blk_dof[b + 1] - d0;
  const double* r = a.inv + a.blk_inv[b] + (row - d0) * nb;
  const double* x = a.rhs + d0;
  double s = 0.0;
  for (int64_t c = lane; c < nb; c += 64) s += r[c] * x[c];
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
    case 4: hipLaunchKernelGGL((k_cell<T, OP, 4>), grid, dim3(64 * kCellWaves), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_cell<T, OP, 8>), grid, dim3(64 * kCellWaves), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_cell<T, OP, 16>), grid, dim3(64 * kCellWaves), 0, s, a); break;
    default: throw Error{HT_ERR_ARG, "tile rows must be 4, 8 or 16"};
  }
}

void launch_cell(int dtype, int op, int J, const CellArgs& a, hipStream_t s) {
  if (dtype == HT_F64) {
    if (op == OP_APPLY) launch_cell_t<double, OP_APPLY>(a, J, s);
    else if (op == OP_RESID) launch_cell_t<double, OP_RESID>(a, J, s);
    else if (op == OP_JACOBI) launch_cell_t<double, OP_JACOBI>(a, J, s);
    else if (op == OP_RESID32) launch_cell_t<double, OP_RESID32>(a, J, s);
    else if (op == OP_RESID32X) launch_cell_t<double, OP_RESID32X>(a, J, s);
    else if (op == OP_CHEB) launch_cell_t<double, OP_CHEB>(a, J, s);
    else launch_cell_t<double, OP_RESTRICT>(a, J, s);
  } else {
    if (op == OP_RESID32 || op == OP_RESID32X)
      throw Error{HT_ERR_ARG, "FP32 residual output needs FP64 input"};
    if (op == OP_CHEB) { launch_cell_t<float, OP_CHEB>(a, J, s); return; }
    if (op == OP_APPLY) launch_cell_t<float, OP_APPLY>(a, J, s);
    else if (op == OP_RESID) launch_cell_t<float, OP_RESID>(a, J, s);
    else if (op == OP_JACOBI) launch_cell_t<float, OP_JACOBI>(a, J, s);
    else launch_cell_t<float, OP_RESTRICT>(a, J, s);
  }
}

template <typename T>
static void launch_exchange_t(int op, const ExchArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)a.nblocks);
  switch (op) {
    case OP_APPLY: hipLaunchKernelGGL((k_exchange<T, OP_APPLY>), grid, dim3(256), 0, s, a); break;
    case OP_RESID: hipLaunchKernelGGL((k_exchange<T, OP_RESID>), grid, dim3(256), 0, s, a); break;
    case OP_JACOBI: hipLaunchKernelGGL((k_exchange<T, OP_JACOBI>), grid, dim3(256), 0, s, a); break;
    case OP_SYNC: hipLaunchKernelGGL((k_exchange<T, OP_SYNC>), grid, dim3(256), 0, s, a); break;
    case OP_FILL: hipLaunchKernelGGL((k_exchange<T, OP_FILL>), grid, dim3(256), 0, s, a); break;
    case OP_RESTRICT: hipLaunchKernelGGL((k_exchange<T, OP_RESTRICT>), grid, dim3(256), 0, s, a); break;
    case OP_RESID32: hipLaunchKernelGGL((k_exchange<T, OP_RESID32>), grid, dim3(256), 0, s, a); break;
    case OP_RESID32X: hipLaunchKernelGGL((k_exchange<T, OP_RESID32X>), grid, dim3(256), 0, s, a); break;
    case OP_CHEB: hipLaunchKernelGGL((k_exchange<T, OP_CHEB>), grid, dim3(256), 0, s, a); break;
    case OP_JACOBIADD:
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((k_exchange<T, OP_JACOBIADD>), grid, dim3(256), 0, s, a);
      break;
  }
}
void launch_exchange(int dtype, int op, const ExchArgs& a, hipStream_t s) {
  if (a.total <= 0) return;
  if (op != OP_APPLY && op != OP_RESID && op != OP_JACOBI && op != OP_SYNC &&
      op != OP_FILL && op != OP_RESTRICT && op != OP_RESID32 && op != OP_CHEB &&
      op != OP_RESID32X && op != OP_JACOBIADD)
    throw Error{HT_ERR_ARG, "unknown exchange operation"};
  // the residual and Jacobi epilogues read u and b at the owner copy
  if ((op == OP_RESID || op == OP_JACOBI || op == OP_RESID32 || op == OP_CHEB ||
       op == OP_RESID32X || op == OP_JACOBIADD) &&
      (!a.u || !a.b))
    throw Error{HT_ERR_ARG, "exchange for residual/Jacobi needs u and b"};
  if (op == OP_CHEB && !a.d) throw Error{HT_ERR_ARG, "Chebyshev step needs d"};
  if ((op == OP_RESID32 || op == OP_RESID32X) && (dtype != HT_F64 || !a.y32))
    throw Error{HT_ERR_ARG, "FP32 residual output needs FP64 input and y32"};
  if (op == OP_RESID32X && !a.efirst)
    throw Error{HT_ERR_ARG, "fused refinement pass needs the first-sweep output"};
  if (op == OP_JACOBIADD && (dtype != HT_F32 || !a.uadd))
    throw Error{HT_ERR_ARG, "the sweep added to the iterate is an FP32 sweep into FP64 u"};
  if (dtype == HT_F64) launch_exchange_t<double>(op, a, s);
  else launch_exchange_t<float>(op, a, s);
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
  // p must have room for 256 more doubles after count
  hipLaunchKernelGGL(k_sum_stage1, dim3(256), dim3(256), 0, s, p, count,
                     const_cast<double*>(p) + count);
  hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(256), 0, s, p + count, out,
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

void launch_seg_sum(const SegArgs& a, hipStream_t s) {
  if (a.nseg <= 0) return;
  hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)((a.nseg + 3) / 4)), dim3(256), 0, s, a);
}

void launch_lane_selftest(int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lane_selftest, dim3(1), dim3(64), 0, s, out);
}

}  // namespace ht
