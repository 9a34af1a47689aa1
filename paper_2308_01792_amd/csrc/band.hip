// Band stencil kernel (gfx950, wave64): the P1 operator y = A x over every
// macro-cell's closure with the planes staged in LDS.
//
// The tile kernel (kernels.hip) gives each wave a fixed (64 i x J rows)
// tile; rows of the index polytope have every length from 1 to n + 1
// (Section 3.2), so many of its lanes fall past the row ends and its loads
// and stores touch short, unaligned pieces of several rows.  Here a
// workgroup owns a band of whole rows of one cell, and
//   * loads each plane of the band once, as one contiguous run of the main
//     block in 16-byte vectors plus the band's face entries, into an LDS
//     image (band.hpp), each value's image row coming from a per-level
//     table shared by all cells;
//   * gives each lane a 2 x 2 block of outputs: two consecutive points of
//     two consecutive rows, which share four of their seven neighbour rows,
//     so ten paired LDS reads serve four points;
//   * keeps a four-plane ring in LDS (planes k - 1, k, k + 1 are read while
//     plane k + 2 is written) and four more planes in flight from HBM.
// The workgroup's waves are split by role: four load waves stream the band's
// planes into registers and from there into the ring, four compute waves
// read the ring and store the results.  Each wave's memory counter then
// covers only its own kind of access, so a load wave waits for its oldest
// plane alone, never for stores, and stores never wait for loads.
// The image carries a zero column at both ends of every row, so the i - 1
// and i + 1 terms taken from the neighbouring lanes (DPP) are those of the
// zero-extended row at every point, including the row ends.  Points inside
// a row (the main block) take the cell's interior stencil (or the uniform
// class stencil of the faces j = 0 and k = 0); the two end points of each
// row (faces i = 0 and i + j + k = n) are computed by one wave per plane
// with per-point class stencils, which gives the cell's exact partial row
// for the ghost exchange (Section 5.2, element-wise assembly restricted to
// the micro-cells of one macro-cell).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "band.hpp"
#include "device.hpp"

namespace ht {

// Start of image row r (band.hpp).  Row indices stay below 64 and L0 below
// 2^11, so the products fit the 24-bit multiplier (full rate, where a 32-bit
// multiply issues at quarter rate).
__device__ __forceinline__ int bstart(int r, int L0) {
  return __mul24(r, L0 + 2) - (__mul24(r, r - 1) >> 1);
}

// Pair index of position u in the concatenation of the first rows of the
// output row pairs: the largest p with E(p) = p b - p^2 <= u (b = L0 + 2),
// i.e. the floor of the smaller root (b - sqrt(b^2 - 4 u)) / 2.  The radicand
// is an integer below 2^24, exact in FP32, and the hardware square root is
// within 1 ulp; the root estimate biased down by 1e-3 is then floor(p) or
// floor(p) - 1 (checked exhaustively for every b up to 1100 with the square
// root off by one ulp either way), and one comparison settles which.
// Returns p and E(p).
__device__ __forceinline__ int bpair(int u, int b, int& Ep) {
  const float bf = (float)b;
  const float x = fmaxf(fmaf(-4.0f, (float)u, bf * bf), 0.0f);
  const int p = (int)fmaf(bf - __builtin_amdgcn_sqrtf(x), 0.5f, -1e-3f);
  const int e0 = __mul24(p, b - p);
  const int e1 = e0 + b - 2 * p - 1;  // E(p + 1)
  const bool up = e1 <= u;
  Ep = up ? e1 : e0;
  return up ? p + 1 : p;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every outstanding global load and store of the wave, which
// would drain the load waves' planes in flight at every step.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T, int OP>
__global__ __launch_bounds__(kBandThreads)
__attribute__((amdgpu_waves_per_eu(4))) void k_band(BandArgs a) {
  constexpr int CAP = BandCap<T>::value;
  constexpr int NL = CAP / kBandLoadLanes;  // image values per load lane
  constexpr int PD = kBandDepth;            // planes in flight per load lane
  // the ring plus a pad that the reads of unused lanes may reach
  __shared__ T ring[kBandSlots * CAP + kBandPad];
  __shared__ T wtab[16 * 15];
  // XCD-aware block order: block b runs on XCD b % 8, and each XCD gets a
  // contiguous run of the (cell, item) work, cell by cell, so the
  // neighbouring bands of one cell (whose halo rows and planes overlap) run
  // together on one XCD and share its L2.  (Grouping a few cells item by
  // item measured slower and read more from HBM.)
  const int64_t nb = a.nblocks;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t wb = (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
  if (wb >= nb) return;
  const int64_t cell = wb / a.nitems;
  const int64_t item = wb - cell * a.nitems;
  const int2 it = a.items[item];
  const int j0 = it.x & 0xffff, R = it.x >> 16, k0 = it.y & 0xffff, k1 = it.y >> 16;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int n = a.n;
  const int64_t bytes = a.stride * (int64_t)sizeof(T);
  const T* wc = (const T*)a.w + cell * 240;
  for (int t = threadIdx.x; t < 240; t += kBandThreads) wtab[t] = wc[t];
  const int off_s0 = (int)a.off_s0, off_s1 = (int)a.off_s1;
  const int jm = j0 - 1;  // row of image row 0
  auto slot = [](int q) { return ((q + kBandSlots) & (kBandSlots - 1)) * CAP; };

  if (wave >= kBandComputeWaves) {
    // ---------------------------------------------------- load waves --
    // Plane q of the band.  Row r of its image is closure row jm + r: the
    // row's first point (i = 0) is in S0, its last (i = e) in S1, the others
    // in the main block, where consecutive rows follow each other: the main
    // points of the image rows form one contiguous run of the cell block
    // (band_plane).  Load lanes read that run in 16-byte vectors (V values
    // each) and place every value at image position f + 4 r, the row r of
    // run element f coming from the level's row table (band.hpp), which is
    // read with the data; 64 lanes of two waves read the rows' two end
    // points.  The address unit handles a fixed number of lanes per cycle,
    // so few wide loads beat one load per image position.  Every plane
    // issues the same loads per lane (out-of-range ones return zero without
    // touching memory), so the wait for the oldest plane is a fixed count.
    constexpr int V = 16 / (int)sizeof(T);
    constexpr int NM = band_nm(CAP, V);
    constexpr int TB = band_tb(NM * V);
    typedef typename std::conditional<TB == 8, u32x2, u32x4>::type TabT;
    const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
    const int lw = wave - kBandComputeWaves;
    const int lpos = lw * 64 + lane;
    // each load lane's own discard position in the ring's pad (values there
    // are never used)
    const int discard = kBandSlots * CAP + (lpos & (kBandPad - 1));
    u32x4 buf[PD][NM];  // main-run vectors of the planes in flight
    T eb[PD];           // end point of each plane in flight
    TabT tr[PD];        // row-table entries of the planes in flight
    int fas[PD];        // run start fa of the planes in flight (uniform)
    auto issue = [&](int q, u32x4 (&b)[NM], T& e, TabT& t, int& fa) {
      const BandPlane P = band_plane(n, off_s0, off_s1, jm, R, k1, q, V);
      fa = P.fa;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int f = P.fa + V * (lpos + kBandLoadLanes * m);
        const bool ok = (f + V > P.F0) & (f < P.F1);
        b[m] = __builtin_amdgcn_raw_buffer_load_b128(
            rx, ok ? (unsigned)(P.mq + f) * (unsigned)sizeof(T) : HT_OOB, 0, 0);
      }
      const int qr = q - (k0 - 1);
      const int64_t blk = (P.valid && qr < kBandTabPlanes) ? 1 + item * kBandTabPlanes + qr : 0;
      const __amdgpu_buffer_rsrc_t rt =
          make_rsrc(a.rtab + blk * (kBandLoadLanes * TB), kBandLoadLanes * TB);
      if constexpr (TB == 8)
        t = __builtin_amdgcn_raw_buffer_load_b64(rt, (unsigned)(lpos * TB), 0, 0);
      else
        t = __builtin_amdgcn_raw_buffer_load_b128(rt, (unsigned)(lpos * TB), 0, 0);
      // lanes 0 .. 63: S0 point of row lpos; lanes 64 .. 127: S1 point of
      // row lpos - 64
      const int r = lpos & 63, Lr = P.L0 - r;
      const bool side = lpos >= 64;
      const bool eok = (lpos < 128) & (r < P.rows) & (jm + r >= 0) &
                       (side ? Lr >= 2 : Lr >= 1);
      const int el = (side ? P.s1b : P.s0b) + r;
      bload(e, rx, eok ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB);
    };
    auto commit = [&](int q, const u32x4 (&b)[NM], const T e, const TabT& t, const int fa) {
      // the plane's validity and rows (as band_plane has them)
      const int L0 = n - jm - q + 1;
      const bool valid = q >= 0 && q <= n && q <= k1 && L0 >= 0;
      const int rows = valid ? (R + 2 < L0 + 1 ? R + 2 : L0 + 1) : 0;
      T* s = ring + slot(q);
      if ((q < 0 || q > n) && q <= k1) {  // outside the cell: zeros
        for (int u = lpos; u < CAP; u += kBandLoadLanes) s[u] = (T)0;
        return;
      }
      if (!valid) return;  // past the march: no later step reads it
      const int base = slot(q);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int f = fa + V * (lpos + kBandLoadLanes * m);
        const T* v = reinterpret_cast<const T*>(&b[m]);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const int w = m * V + i;  // byte w of the lane's table entry
          const unsigned r4 = (t[w >> 2] >> (8 * (w & 3))) & 0xffu;
          ring[r4 != 0xffu ? base + f + i + (int)r4 : discard] = v[i];
        }
      }
      // pads and end points of the rows
      const int r = lpos & 63;
      if ((lpos < 128) & (r < rows)) {
        const int D = bstart(r, L0), Lr = L0 - r;
        if (lpos < 64) {
          s[D] = (T)0;
          s[D + 1] = e;
        } else {
          if (Lr >= 2) s[D + Lr] = e;
          s[D + Lr + 1] = (T)0;
        }
      }
      // the row j = -1 of the bands at j0 = 0 reads as zeros
      if (jm < 0)
        for (int u = 2 + lpos; u < L0; u += kBandLoadLanes) s[u] = (T)0;
    };
    // plane q travels in register set (q - k0 + 1) % PD
    static_assert(PD == 4, "the prologue below assumes four planes in flight");
    issue(k0 - 1, buf[0], eb[0], tr[0], fas[0]);
    issue(k0, buf[1], eb[1], tr[1], fas[1]);
    issue(k0 + 1, buf[2], eb[2], tr[2], fas[2]);
    issue(k0 + 2, buf[3], eb[3], tr[3], fas[3]);
    commit(k0 - 1, buf[0], eb[0], tr[0], fas[0]);
    issue(k0 + 3, buf[0], eb[0], tr[0], fas[0]);
    commit(k0, buf[1], eb[1], tr[1], fas[1]);
    issue(k0 + 4, buf[1], eb[1], tr[1], fas[1]);
    commit(k0 + 1, buf[2], eb[2], tr[2], fas[2]);
    issue(k0 + 5, buf[2], eb[2], tr[2], fas[2]);
    lds_barrier();
    // Step k commits plane k + 2 and issues plane k + 2 + PD.
    auto lstep = [&](int k, int set) {
      commit(k + 2, buf[set], eb[set], tr[set], fas[set]);
      issue(k + 2 + PD, buf[set], eb[set], tr[set], fas[set]);
      lds_barrier();
    };
    // whole rounds of PD steps, without exits in between (the compute waves
    // meet the extra barriers of the last round idle)
    for (int k = k0; k < k1; k += PD) {
      lstep(k, 3);
      lstep(k + 1, 0);
      lstep(k + 2, 1);
      lstep(k + 3, 2);
    }
    return;
  }

  // ------------------------------------------------------ compute waves --
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  constexpr bool R32 = OP == OP_RESID32 || OP == OP_RESID32X;
  constexpr bool ADD = OP == OP_JACOBIADD;
  constexpr bool SWEEP = OP == OP_JACOBI || OP == OP_RESID || R32 || ADD;
  const __amdgpu_buffer_rsrc_t ry32 =
      make_rsrc(R32 ? a.y32 + cell * a.stride : (float*)a.y, R32 ? a.stride * 4 : 0);
  const __amdgpu_buffer_rsrc_t ref =
      make_rsrc(OP == OP_RESID32X ? a.efirst + cell * a.stride : (float*)a.y,
                OP == OP_RESID32X ? a.stride * 4 : 0);
  const __amdgpu_buffer_rsrc_t rb =
      make_rsrc(SWEEP ? (const T*)a.b + cell * a.stride : (const T*)a.x, SWEEP ? bytes : 0);
  // OP_JACOBIADD: the FP64 iterate (byte offset of a point = 2 x its FP32 one)
  const __amdgpu_buffer_rsrc_t ru =
      make_rsrc(ADD ? a.uadd + cell * a.stride : (double*)a.y, ADD ? a.stride * 8 : 0);
  // omega D^-1 at the cell's interior points (as the tile kernel forms it)
  const T omega_invd = SWEEP ? (T)(a.omega * a.nscale * a.cls[cell * 16].inv_diag_unit) : (T)0;
  double nsq = 0.0;  // |r|^2 of the points this wave finishes
  const T w0 = wc[0], w1 = wc[1], w2 = wc[2], w3 = wc[3], w4 = wc[4], w5 = wc[5],
          w6 = wc[6], w7 = wc[7], w8 = wc[8], w9 = wc[9], w10 = wc[10],
          w11 = wc[11], w12 = wc[12], w13 = wc[13], w14 = wc[14];
  struct Two { T a, b; };  // the values at columns A and A + 1 of one row
  auto rd2 = [&](int e) { return Two{ring[e], ring[e + 1]}; };
  // One output row at columns A (a) and A + 1 (b) from its seven neighbour
  // rows (dj, dk).  Interior weights are the same on every lane, and a lane
  // shift is linear: the i + 1 terms of b (offsets 1, 8, 10, 13) are formed
  // at the next lane's a column and the i - 1 terms of a (offsets 2, 7, 9,
  // 14) at the previous lane's b column, each shifted once.
  auto row_interior = [&](const Two& xc, const Two& xjp, const Two& xjm, const Two& xkp,
                          const Two& xjmkp, const Two& xkm, const Two& xjpkm, T& oa, T& ob) {
    const T ta = fma(w13, xjmkp.a, fma(w10, xkm.a, fma(w8, xjm.a, w1 * xc.a)));
    const T tb = fma(w14, xjpkm.b, fma(w9, xkp.b, fma(w7, xjp.b, w2 * xc.b)));
    T sa = fma(w13, xjmkp.b, fma(w10, xkm.b, fma(w8, xjm.b, w1 * xc.b)));
    T sb = fma(w14, xjpkm.a, fma(w9, xkp.a, fma(w7, xjp.a, w2 * xc.a)));
    sa = fma(w0, xc.a, sa);     sb = fma(w0, xc.b, sb);
    sa = fma(w3, xjp.a, sa);    sb = fma(w3, xjp.b, sb);
    sa = fma(w4, xjm.a, sa);    sb = fma(w4, xjm.b, sb);
    sa = fma(w5, xkp.a, sa);    sb = fma(w5, xkp.b, sb);
    sa = fma(w6, xkm.a, sa);    sb = fma(w6, xkm.b, sb);
    sa = fma(w11, xjmkp.a, sa); sb = fma(w11, xjmkp.b, sb);
    sa = fma(w12, xjpkm.a, sa); sb = fma(w12, xjpkm.b, sb);
    oa = sa + lane_prev(tb);
    ob = sb + lane_next(ta);
  };
  // The same with per-lane class stencils W (faces j = 0 and k = 0).
  auto row_special = [&](const T* W, const Two& xc, const Two& xjp, const Two& xjm,
                         const Two& xkp, const Two& xjmkp, const Two& xkm, const Two& xjpkm,
                         T& oa, T& ob) {
    T a = W[0] * xc.a, b = W[0] * xc.b;
    a = fma(W[1], xc.b, a);                 b = fma(W[1], lane_next(xc.a), b);
    a = fma(W[2], lane_prev(xc.b), a);      b = fma(W[2], xc.a, b);
    a = fma(W[3], xjp.a, a);                b = fma(W[3], xjp.b, b);
    a = fma(W[4], xjm.a, a);                b = fma(W[4], xjm.b, b);
    a = fma(W[5], xkp.a, a);                b = fma(W[5], xkp.b, b);
    a = fma(W[6], xkm.a, a);                b = fma(W[6], xkm.b, b);
    a = fma(W[7], lane_prev(xjp.b), a);     b = fma(W[7], xjp.a, b);
    a = fma(W[8], xjm.b, a);                b = fma(W[8], lane_next(xjm.a), b);
    a = fma(W[9], lane_prev(xkp.b), a);     b = fma(W[9], xkp.a, b);
    a = fma(W[10], xkm.b, a);               b = fma(W[10], lane_next(xkm.a), b);
    a = fma(W[11], xjmkp.a, a);             b = fma(W[11], xjmkp.b, b);
    a = fma(W[12], xjpkm.a, a);             b = fma(W[12], xjpkm.b, b);
    a = fma(W[13], xjmkp.b, a);             b = fma(W[13], lane_next(xjmkp.a), b);
    a = fma(W[14], lane_prev(xjpkm.b), a);  b = fma(W[14], xjpkm.a, b);
    oa = a;
    ob = b;
  };
  auto compute = [&](int k) {
    const int L0 = n - jm - k + 1;
    const int rmax = R < L0 - 1 ? R : L0 - 1;  // output rows 1 .. rmax
    if (rmax < 1) return;
    // Output rows are taken in pairs (2p + 1, 2p + 2).  The lanes run over
    // the concatenation of the pairs' first rows (each with its pad
    // columns): pair p starts there at E(p) = p b - p^2, b = L0 + 2.
    const int b = L0 + 2;
    const int npair = (rmax + 1) >> 1;
    const int Etot = __mul24(npair, b - npair);
    const int sk = slot(k), skp = slot(k + 1), skm = slot(k - 1);
    // main-block element of image position U in output row r: Kc + U - 4 r
    const int Kc = tet32(n - 1) - tet32(n - 1 - k) - 1 + j0 * (n - 1 - k) -
                   ((j0 * (j0 - 1)) >> 1) - bstart(1, L0) + 3;
    const int nch = (Etot + 123) / 124;
    // One chunk: lanes 1 .. 62 output columns A, A + 1 of the rows r and
    // r + 1 (up to 248 points).  SPECIAL chunks may hold points of the faces
    // j = 0 (row 1 of the band j0 = 0) or k = 0 and take per-lane class
    // stencils; the others take the cell's interior stencil.
    auto chunk = [&](int ch, auto special) {
      constexpr bool SPECIAL = decltype(special)::value;
      const int ur = 124 * ch - 2 + 2 * lane;
      const int u = ur < 0 ? 0 : (ur > Etot - 1 ? Etot - 1 : ur);
      int Ep;
      const int p = bpair(u, b, Ep);
      const int r = 2 * p + 1, c = u - Ep;
      const int A = bstart(r, L0) + c;
      const int v = L0 - r + 2;  // positions of image row r
      // main-block points only (2 <= c <= L_r - 1); the row ends are the
      // face points computed below.  Row r + 1 is one point shorter.
      const bool out = lane >= 1 && lane <= 62 && ur == u;
      const bool two = out && r + 1 <= rmax;
      const int Lr = L0 - r;
      const unsigned sz = (unsigned)sizeof(T);
      const unsigned e1 = (unsigned)(Kc + A - 4 * r) * sz;
      const unsigned e2 = e1 + (unsigned)(v - 4) * sz;
      const bool st1a = out && c >= 2 && c <= Lr - 1, st1b = out && c >= 1 && c <= Lr - 2;
      const bool st2a = two && c >= 2 && c <= Lr - 2, st2b = two && c >= 1 && c <= Lr - 3;
      // sweeps: b at the four points, two 16-byte loads issued before the
      // LDS reads (a pair's second value is read even where only the first
      // is used: it is the next main-block element, inside the cell block)
      u32x4 bv1 = {0u, 0u, 0u, 0u}, bv2 = {0u, 0u, 0u, 0u};
      if constexpr (SWEEP) {
        bv1 = __builtin_amdgcn_raw_buffer_load_b128(rb, (st1a || st1b) ? e1 : HT_OOB, 0, 0);
        bv2 = __builtin_amdgcn_raw_buffer_load_b128(rb, (st2a || st2b) ? e2 : HT_OOB, 0, 0);
      }
      // OP_JACOBIADD: u at the four points (two FP64 pairs)
      u32x4 uv1 = {0u, 0u, 0u, 0u}, uv2 = {0u, 0u, 0u, 0u};
      if constexpr (ADD) {
        uv1 = __builtin_amdgcn_raw_buffer_load_b128(ru, (st1a || st1b) ? 2 * e1 : HT_OOB, 0, 0);
        uv2 = __builtin_amdgcn_raw_buffer_load_b128(ru, (st2a || st2b) ? 2 * e2 : HT_OOB, 0, 0);
      }
      // ten rows (dj, dk) at columns A, A + 1: plane k rows r - 1 .. r + 2,
      // plane k + 1 rows r - 1 .. r + 1, plane k - 1 rows r .. r + 2
      const int q0 = sk + A, q1 = q0 + v, q2 = q1 + v - 1, qm = q0 - v - 1;
      const int p0 = skp + A - r, p1 = p0 + v - 1, pm = p0 - v;
      const int m0 = skm + A + r, m1 = m0 + v + 1, m2 = m1 + v;
      const Two K0 = rd2(q0), K1 = rd2(q1), K2 = rd2(q2), Km = rd2(qm);
      const Two P0 = rd2(p0), P1 = rd2(p1), Pm = rd2(pm);
      const Two M0 = rd2(m0), M1 = rd2(m1), M2 = rd2(m2);
      T a1, b1, a2, b2;
      if (!SPECIAL) {
        row_interior(K0, K1, Km, P0, Pm, M0, M1, a1, b1);
        row_interior(K1, K2, K0, P1, P0, M1, M2, a2, b2);
      } else {
        const int kb = (k == 0) << 2;
        row_special(wtab + 15 * (((jm + r == 0) << 1) | kb), K0, K1, Km, P0, Pm, M0, M1, a1, b1);
        row_special(wtab + 15 * kb, K1, K2, K0, P1, P0, M1, M2, a2, b2);
      }
      if constexpr (SWEEP) {
        // Points on the faces j = 0 (row 1 of the band j0 = 0) and k = 0
        // keep their partial row for the exchange; the others are finished:
        // r = b - A u, and the Jacobi update u + omega D^-1 r or r itself.
        const bool surf1 = SPECIAL && ((jm + r == 0) || k == 0);
        const bool surf2 = SPECIAL && k == 0;
        const T* b1v = reinterpret_cast<const T*>(&bv1);
        const T* b2v = reinterpret_cast<const T*>(&bv2);
        auto fin = [&](T acc, T xc, T bval, bool st, bool surf, unsigned e) {
          const T rr = bval - acc;
          nsq += (st && !surf) ? (double)rr * (double)rr : 0.0;
          if constexpr (R32) {
            // finished points: the FP32 residual (element offset = e / 2)
            // and, fused, the next correction's first sweep in FP32 as the
            // separate zero-guess sweep forms it (FP32 factor times FP32
            // residual); the face points' FP64 partial rows are stored below
            const unsigned f = (st && !surf) ? e >> 1 : HT_OOB;
            bstore((float)rr, ry32, f);
            if constexpr (OP == OP_RESID32X) bstore((float)omega_invd * (float)rr, ref, f);
            return acc;
          }
          return surf ? acc : ((OP == OP_JACOBI || ADD) ? fma(omega_invd, rr, xc) : rr);
        };
        a1 = fin(a1, K0.a, b1v[0], st1a, surf1, e1);
        b1 = fin(b1, K0.b, b1v[1], st1b, surf1, e1 + sz);
        a2 = fin(a2, K1.a, b2v[0], st2a, surf2, e2);
        b2 = fin(b2, K1.b, b2v[1], st2b, surf2, e2 + sz);
        if constexpr (R32) {
          // only the face points keep an FP64 partial row
          if constexpr (SPECIAL) {
            bstore(a1, ry, st1a && surf1 ? e1 : HT_OOB);
            bstore(b1, ry, st1b && surf1 ? e1 + sz : HT_OOB);
            bstore(a2, ry, st2a && surf2 ? e2 : HT_OOB);
            bstore(b2, ry, st2b && surf2 ? e2 + sz : HT_OOB);
          }
          return;
        }
        if constexpr (ADD) {
          // finished points: u += e_new in FP64; face points: partial rows
          const double* u1 = reinterpret_cast<const double*>(&uv1);
          const double* u2 = reinterpret_cast<const double*>(&uv2);
          bstore(u1[0] + (double)a1, ru, st1a && !surf1 ? 2 * e1 : HT_OOB);
          bstore(u1[1] + (double)b1, ru, st1b && !surf1 ? 2 * (e1 + sz) : HT_OOB);
          bstore(u2[0] + (double)a2, ru, st2a && !surf2 ? 2 * e2 : HT_OOB);
          bstore(u2[1] + (double)b2, ru, st2b && !surf2 ? 2 * (e2 + sz) : HT_OOB);
          if constexpr (SPECIAL) {
            bstore(a1, ry, st1a && surf1 ? e1 : HT_OOB);
            bstore(b1, ry, st1b && surf1 ? e1 + sz : HT_OOB);
            bstore(a2, ry, st2a && surf2 ? e2 : HT_OOB);
            bstore(b2, ry, st2b && surf2 ? e2 + sz : HT_OOB);
          }
          return;
        }
      }
      // no branches: the chunk stays one basic block
      bstore(a1, ry, st1a ? e1 : HT_OOB);
      bstore(b1, ry, st1b ? e1 + sz : HT_OOB);
      bstore(a2, ry, st2a ? e2 : HT_OOB);
      bstore(b2, ry, st2b ? e2 + sz : HT_OOB);
    };
    // chunks before nspec may touch row 1 of the band j0 = 0 (pair 0, whose
    // first row ends below E(1) = b - 1); on the plane k = 0 every chunk is
    // special
    const int nspec = k == 0 ? nch : (j0 == 0 ? min(nch, (b - 1 + 123) / 124) : 0);
    int ch = wave;
    for (; ch < nspec; ch += kBandComputeWaves) chunk(ch, std::true_type{});
    for (; ch < nch; ch += kBandComputeWaves) chunk(ch, std::false_type{});
    // Row ends (faces i = 0 and i + j + k = n) of the output rows: lane q < R
    // takes the first point of row q + 1, lane R + q its last point.  The
    // wave with the fewest chunks of this plane does it.
    if (wave == (nch & (kBandComputeWaves - 1))) {
      const bool s1 = lane >= R;
      const int r0 = (s1 ? lane - R : lane) + 1;
      const bool ok = lane < 2 * R && r0 <= rmax && (!s1 || L0 - r0 >= 2);
      const int r = ok ? r0 : 1;
      const int Lr = L0 - r, v = Lr + 2;
      const int c = (ok && s1) ? Lr : 1;
      const int U = bstart(r, L0) + c;
      const int j = jm + r;
      const int cls = (c == 1) | ((j == 0) << 1) | ((k == 0) << 2) | ((c == Lr) << 3);
      const T* W = wtab + cls * 15;
      T s = W[0] * ring[sk + U];
      s = fma(W[1], ring[sk + U + 1], s);
      s = fma(W[2], ring[sk + U - 1], s);
      s = fma(W[3], ring[sk + U + v], s);
      s = fma(W[4], ring[sk + U - v - 1], s);
      s = fma(W[5], ring[skp + U - r], s);
      s = fma(W[6], ring[skm + U + r], s);
      s = fma(W[7], ring[sk + U + v - 1], s);
      s = fma(W[8], ring[sk + U - v], s);
      s = fma(W[9], ring[skp + U - r - 1], s);
      s = fma(W[10], ring[skm + U + r + 1], s);
      s = fma(W[11], ring[skp + U - r - v], s);
      s = fma(W[12], ring[skm + U + r + v + 1], s);
      s = fma(W[13], ring[skp + U - r - v + 1], s);
      s = fma(W[14], ring[skm + U + r + v], s);
      const int el = s1 ? off_s1 + tri32(n) - tri32(n - k) + j
                        : off_s0 + tri32(n + 1) - tri32(n + 1 - k) + j;
      bstore(s, ry, ok ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB);
    }
  };
  lds_barrier();  // the load waves' first three planes
  const int kend = k0 + (k1 - k0 + PD - 1) / PD * PD;  // the load waves' rounds
  for (int k = k0; k < kend; ++k) {
    if (k < k1) compute(k);
    lds_barrier();
  }
  if constexpr (SWEEP) {
    nsq = wave_sum(nsq);
    if (lane == 0) a.partials[wb * kBandComputeWaves + wave] = nsq;
  }
}

template <typename T>
static void launch_band_t(int op, const BandArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(((a.nblocks + 7) / 8) * 8));
  switch (op) {
    case OP_APPLY:
      hipLaunchKernelGGL((k_band<T, OP_APPLY>), grid, dim3(kBandThreads), 0, s, a);
      break;
    case OP_JACOBI:
      hipLaunchKernelGGL((k_band<T, OP_JACOBI>), grid, dim3(kBandThreads), 0, s, a);
      break;
    case OP_RESID:
      hipLaunchKernelGGL((k_band<T, OP_RESID>), grid, dim3(kBandThreads), 0, s, a);
      break;
    case OP_JACOBIADD:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((k_band<T, OP_JACOBIADD>), grid, dim3(kBandThreads), 0, s, a);
        break;
      }
      throw Error{HT_ERR_ARG, "band kernel: the sweep added to u is an FP32 operation"};
    case OP_RESID32:
    case OP_RESID32X:
      if constexpr (sizeof(T) == 8) {
        if (op == OP_RESID32)
          hipLaunchKernelGGL((k_band<T, OP_RESID32>), grid, dim3(kBandThreads), 0, s, a);
        else
          hipLaunchKernelGGL((k_band<T, OP_RESID32X>), grid, dim3(kBandThreads), 0, s, a);
        break;
      }
      throw Error{HT_ERR_ARG, "band kernel: the FP32-output residual is an FP64 operation"};
    default: throw Error{HT_ERR_ARG, "band kernel: unsupported operation"};
  }
}

void launch_band(int dtype, int op, const BandArgs& a, hipStream_t s) {
  if (a.nblocks <= 0) return;
  if (dtype == HT_F64) launch_band_t<double>(op, a, s);
  else launch_band_t<float>(op, a, s);
}

}  // namespace ht
