// Band stencil kernel (gfx950, wave64): the P1 operator y = A x over every
// macro-cell's closure with the planes staged in LDS.
//
// The tile kernel (kernels.hip) gives each wave a fixed (64 i x J rows)
// tile; rows of the index polytope have every length from 1 to n + 1
// (Section 3.2), so many of its lanes fall past the row ends and its loads
// and stores touch short, unaligned pieces of several rows.  Here a
// workgroup owns a band of whole rows of one cell, and
//   * loads each plane of the band once, as one contiguous run of the main
//     block plus the band's face entries, into an LDS image (band.hpp);
//   * assigns each lane two consecutive image positions, so a wave's 124
//     outputs are consecutive closure points, possibly spanning several
//     rows, and its stores form one contiguous run of the main block;
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

// Image row of position U, 0 <= U < D(rows), rows <= L0 + 1: the largest r
// with D(r) <= U, i.e. the floor of the smaller root t of D(r) = U.  The
// radicand and its terms are integers below 2^24, exact in FP32, and the
// hardware square root is within 1 ulp, so t is known to within 5e-4; the
// estimate biased down by 1e-3 is floor(t) or floor(t) - 1, and one
// comparison settles which.  Returns r and D(r).
__device__ __forceinline__ int brow(int U, int L0, int& Dr) {
  const float b = (float)(2 * L0 + 5);
  const float x = fmaxf(fmaf(-8.0f, (float)U, b * b), 0.0f);
  int r = (int)fmaf(b - __builtin_amdgcn_sqrtf(x), 0.5f, -1e-3f);
  r = r < 0 ? 0 : r;
  const int d0 = bstart(r, L0), d1 = d0 + (L0 - r) + 2;  // D(r), D(r + 1)
  const bool up = d1 <= U;
  Dr = up ? d1 : d0;
  return up ? r + 1 : r;
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
__global__ __launch_bounds__(kBandThreads) void k_band(BandArgs a) {
  constexpr int CAP = BandCap<T>::value;
  constexpr int NL = CAP / kBandLoadLanes;  // image values per load lane
  constexpr int PD = kBandDepth;            // planes in flight per load lane
  __shared__ T ring[kBandSlots * CAP];
  __shared__ T wtab[16 * 15];
  // XCD-aware block order: block b runs on XCD b % 8; each XCD gets a
  // contiguous run of (cell, item) work, so concurrent bands of one cell
  // share an L2.
  const int64_t nb = a.nblocks;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t wb = (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
  if (wb >= nb) return;
  const int64_t cell = wb / a.nitems;
  const int2 it = a.items[wb % a.nitems];
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
    // Plane q of the band: load lane t holds image positions t + m kBandLoadLanes.
    // Row r of the image is closure row jm + r: its first point (i = 0) is
    // in S0, its last (i = e) in S1, the others in the main block, where
    // consecutive rows follow each other (the main-block element of image
    // position U in row r is mq + U - 4 r).  Every plane issues the same
    // NL loads per lane (out-of-range ones return zero without touching
    // memory), so the wait for the oldest plane is a fixed count.
    const __amdgpu_buffer_rsrc_t rx = make_rsrc((const T*)a.x + cell * a.stride, bytes);
    const int lw = wave - kBandComputeWaves;
    T buf[PD][NL];
    // Row of each held position and the start of that row, at the last
    // plane issued.  From one plane to the next every row loses one point,
    // so a position moves down by at most one row as long as the rows stay
    // longer than the row indices (L0 > 2 R + 1); below that, and at the
    // first plane, the row comes from the closed form.
    int rs[NL], ds[NL];
#pragma unroll
    for (int m = 0; m < NL; ++m) rs[m] = ds[m] = 0;
    const int qfirst = k0 > 0 ? k0 - 1 : 0;
    auto issue = [&](int q, T (&b)[NL]) {
      const int L0 = n - jm - q + 1;
      const int rows = (L0 < 0 || q > k1) ? 0 : (R + 2 < L0 + 1 ? R + 2 : L0 + 1);
      const int size = bstart(rows, L0);
      const bool plane_ok = q >= 0 && q <= n;
      const bool incr = q > qfirst && L0 > 2 * R + 1;
      const int s0b = off_s0 + tri32(n + 1) - tri32(n + 1 - q) + jm;
      const int s1b = off_s1 + tri32(n) - tri32(n - q) + jm;
      const int mq = tet32(n - 1) - tet32(n - 1 - q) - 2 + jm * (n - 1 - q) -
                     ((jm * (jm - 1)) >> 1);
#pragma unroll
      for (int m = 0; m < NL; ++m) {
        const int U0 = m * kBandLoadLanes + lw * 64;
        unsigned off = HT_OOB;
        if (plane_ok && U0 < size) {  // uniform
          const int U = U0 + lane;
          int r, Dr;
          if (incr) {
            r = rs[m];
            Dr = ds[m] - r;
            const int nx = Dr + (L0 - r) + 2;
            const bool up = U >= nx;
            r += up ? 1 : 0;
            Dr = up ? nx : Dr;
          } else {
            r = brow(U < size ? U : size - 1, L0, Dr);
          }
          rs[m] = r;
          ds[m] = Dr;
          const int c = U - Dr, Lr = L0 - r;
          const bool end = c == 1 || c == Lr;
          const int el = end ? (c == 1 ? s0b : s1b) + r : mq + U - 4 * r;
          const bool data = jm + r >= 0 && c >= 1 && c <= Lr && U < size;
          off = data ? (unsigned)el * (unsigned)sizeof(T) : HT_OOB;
        }
        bload(b[m], rx, off);
      }
    };
    // Every held value is written, past the image end too (those slot
    // positions are never read as data): each register set is then consumed
    // in full before it is reloaded, and the wait for it counts only the
    // younger planes' loads.
    auto commit = [&](int q, const T (&b)[NL]) {
      T* s = ring + slot(q);
#pragma unroll
      for (int m = 0; m < NL; ++m) s[m * kBandLoadLanes + lw * 64 + lane] = b[m];
    };
    // plane q travels in register set (q - k0 + 1) % PD
    static_assert(PD == 4, "the prologue below assumes four planes in flight");
    issue(k0 - 1, buf[0]);
    issue(k0, buf[1]);
    issue(k0 + 1, buf[2]);
    issue(k0 + 2, buf[3]);
    commit(k0 - 1, buf[0]);
    issue(k0 + 3, buf[0]);
    commit(k0, buf[1]);
    issue(k0 + 4, buf[1]);
    commit(k0 + 1, buf[2]);
    issue(k0 + 5, buf[2]);
    lds_barrier();
    // Step k commits plane k + 2 and issues plane k + 2 + PD.  The commit is
    // unconditional (past k1 it fills a slot no later step reads), so every
    // path through the loop consumes the same loads in the same order.
    auto lstep = [&](int k, T (&b)[NL]) {
      commit(k + 2, b);
      issue(k + 2 + PD, b);
      lds_barrier();
    };
    // whole rounds of PD steps, without exits in between (the compute waves
    // meet the extra barriers of the last round idle)
    for (int k = k0; k < k1; k += PD) {
      lstep(k, buf[3]);
      lstep(k + 1, buf[0]);
      lstep(k + 2, buf[1]);
      lstep(k + 3, buf[2]);
    }
    return;
  }

  // ------------------------------------------------------ compute waves --
  const __amdgpu_buffer_rsrc_t ry = make_rsrc((T*)a.y + cell * a.stride, bytes);
  const T w0 = wc[0], w1 = wc[1], w2 = wc[2], w3 = wc[3], w4 = wc[4], w5 = wc[5],
          w6 = wc[6], w7 = wc[7], w8 = wc[8], w9 = wc[9], w10 = wc[10],
          w11 = wc[11], w12 = wc[12], w13 = wc[13], w14 = wc[14];
  auto compute = [&](int k) {
    const int L0 = n - jm - k + 1;
    const int rmax = R < L0 - 1 ? R : L0 - 1;  // output rows 1 .. rmax
    if (rmax < 1) return;
    const int Ub = bstart(1, L0), Ue = bstart(rmax + 1, L0);
    const int sk = slot(k), skp = slot(k + 1), skm = slot(k - 1);
    // main-block element of image position U in output row r: Kc + U - 4 r
    const int Kc = tet32(n - 1) - tet32(n - 1 - k) - 1 + j0 * (n - 1 - k) -
                   ((j0 * (j0 - 1)) >> 1) - Ub + 3;
    // Two consecutive image positions per lane, A = P + 2 lane and B = A + 1:
    // a wave covers 128 positions, of which lanes 1 .. 62 output 124.  B is
    // A's i + 1 neighbour in the same row (unless A is the row's last pad
    // column, whose pair is not output), so the i +- 1 terms need one lane
    // shift per point pair instead of two per point, and each row's two
    // values come from one paired LDS read.
    // The pair grid starts at G = Ub or Ub - 1 so that A always maps to an
    // even main-block element: a pair inside a row is then one aligned
    // two-value store, and a wave's stores cover whole cache lines.
    const int G = Ub - ((Kc + Ub) & 1);
    const int nch = (Ue - G + 123) / 124;
    // One chunk: the 124 outputs of lanes 1 .. 62.  SPECIAL chunks may hold
    // points of the faces j = 0 (row 1 of the band j0 = 0) or k = 0 and take
    // per-lane class stencils; the others take the cell's interior stencil.
    auto chunk = [&](int ch, auto special) {
      constexpr bool SPECIAL = decltype(special)::value;
      const int P = G + 124 * ch - 2;
      const int Ar = P + 2 * lane;
      const int A = Ar < Ub ? Ub : (Ar > Ue - 1 ? Ue - 1 : Ar);
      int Dr;
      const int r = brow(A, L0, Dr);
      const int c = A - Dr, Lr = L0 - r, v = Lr + 2;
      // the seven rows (dj, dk) at the columns of A and B
      const int e0 = sk + A, e1 = sk + A + v, e2 = sk + A - v - 1;
      const int e3 = skp + A - r, e4 = skp + A - r - v;
      const int e5 = skm + A + r, e6 = skm + A + r + v + 1;
      const T xcA = ring[e0], xcB = ring[e0 + 1];          // ( 0,  0)
      const T xjpA = ring[e1], xjpB = ring[e1 + 1];        // (+1,  0)
      const T xjmA = ring[e2], xjmB = ring[e2 + 1];        // (-1,  0)
      const T xkpA = ring[e3], xkpB = ring[e3 + 1];        // ( 0, +1)
      const T xjmkpA = ring[e4], xjmkpB = ring[e4 + 1];    // (-1, +1)
      const T xkmA = ring[e5], xkmB = ring[e5 + 1];        // ( 0, -1)
      const T xjpkmA = ring[e6], xjpkmB = ring[e6 + 1];    // (+1, -1)
      T accA, accB;
      if (!SPECIAL) {
        // Interior weights are the same on every lane, and a lane shift is
        // linear: the i + 1 terms of B (offsets 1, 8, 10, 13) are formed at
        // A's column of the next lane and the i - 1 terms of A (offsets 2,
        // 7, 9, 14) at B's column of the previous lane, each shifted once.
        const T tA = fma(w13, xjmkpA, fma(w10, xkmA, fma(w8, xjmA, w1 * xcA)));
        const T tB = fma(w14, xjpkmB, fma(w9, xkpB, fma(w7, xjpB, w2 * xcB)));
        accA = fma(w13, xjmkpB, fma(w10, xkmB, fma(w8, xjmB, w1 * xcB)));
        accB = fma(w14, xjpkmA, fma(w9, xkpA, fma(w7, xjpA, w2 * xcA)));
        accA = fma(w0, xcA, accA); accB = fma(w0, xcB, accB);
        accA = fma(w3, xjpA, accA); accB = fma(w3, xjpB, accB);
        accA = fma(w4, xjmA, accA); accB = fma(w4, xjmB, accB);
        accA = fma(w5, xkpA, accA); accB = fma(w5, xkpB, accB);
        accA = fma(w6, xkmA, accA); accB = fma(w6, xkmB, accB);
        accA = fma(w11, xjmkpA, accA); accB = fma(w11, xjmkpB, accB);
        accA = fma(w12, xjpkmA, accA); accB = fma(w12, xjpkmB, accB);
        accA += lane_prev(tB);
        accB += lane_next(tA);
      } else {
        const int cls = ((jm + r == 0) << 1) | ((k == 0) << 2);
        const T* W = wtab + cls * 15;
        T a = W[0] * xcA, b = W[0] * xcB;
        a = fma(W[1], xcB, a);              b = fma(W[1], lane_next(xcA), b);
        a = fma(W[2], lane_prev(xcB), a);   b = fma(W[2], xcA, b);
        a = fma(W[3], xjpA, a);             b = fma(W[3], xjpB, b);
        a = fma(W[4], xjmA, a);             b = fma(W[4], xjmB, b);
        a = fma(W[5], xkpA, a);             b = fma(W[5], xkpB, b);
        a = fma(W[6], xkmA, a);             b = fma(W[6], xkmB, b);
        a = fma(W[7], lane_prev(xjpB), a);  b = fma(W[7], xjpA, b);
        a = fma(W[8], xjmB, a);             b = fma(W[8], lane_next(xjmA), b);
        a = fma(W[9], lane_prev(xkpB), a);  b = fma(W[9], xkpA, b);
        a = fma(W[10], xkmB, a);            b = fma(W[10], lane_next(xkmA), b);
        a = fma(W[11], xjmkpA, a);          b = fma(W[11], xjmkpB, b);
        a = fma(W[12], xjpkmA, a);          b = fma(W[12], xjpkmB, b);
        a = fma(W[13], xjmkpB, a);          b = fma(W[13], lane_next(xjmkpA), b);
        a = fma(W[14], lane_prev(xjpkmB), a); b = fma(W[14], xjpkmA, b);
        accA = a;
        accB = b;
      }
      // main-block points only (2 <= c <= Lr - 1); the row ends are the
      // face points computed below
      const bool out = lane >= 1 && lane <= 62 && Ar == A;
      const bool stA = out && c >= 2 && c <= Lr - 1;
      const bool stB = out && A + 1 <= Ue - 1 && c + 1 >= 2 && c + 1 <= Lr - 1;
      const unsigned el = (unsigned)(Kc + A - 4 * r) * (unsigned)sizeof(T);
      // no branches: the chunk stays one basic block, which lets the
      // scheduler overlap two chunks
      bstore2(accA, accB, ry, stA && stB ? el : HT_OOB);
      bstore(accA, ry, stA && !stB ? el : HT_OOB);
      bstore(accB, ry, stB && !stA ? el + (unsigned)sizeof(T) : HT_OOB);
    };
    // chunks before nspec may touch row 1 of the band j0 = 0 (positions
    // below D(2) = Ub + L0 + 1); on the plane k = 0 every chunk is special
    const int nspec = k == 0 ? nch
                      : (j0 == 0 ? min(nch, (Ub + L0 + 3 - G + 123) / 124) : 0);
    int ch = wave;
    for (; ch < nspec; ch += kBandComputeWaves) chunk(ch, std::true_type{});
    // two independent chunks per iteration, so that the LDS reads of one
    // overlap the arithmetic of the other
    for (; ch + kBandComputeWaves < nch; ch += 2 * kBandComputeWaves) {
      chunk(ch, std::false_type{});
      chunk(ch + kBandComputeWaves, std::false_type{});
    }
    if (ch < nch) chunk(ch, std::false_type{});
    // Row ends (faces i = 0 and i + j + k = n) of the output rows: lane q < R
    // takes the first point of row q + 1, lane R + q its last point.
    if (wave == (k & (kBandComputeWaves - 1))) {
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
}

template <typename T>
static void launch_band_t(int op, const BandArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(((a.nblocks + 7) / 8) * 8));
  switch (op) {
    case OP_APPLY:
      hipLaunchKernelGGL((k_band<T, OP_APPLY>), grid, dim3(kBandThreads), 0, s, a);
      break;
    default: throw Error{HT_ERR_ARG, "band kernel: unsupported operation"};
  }
}

void launch_band(int dtype, int op, const BandArgs& a, hipStream_t s) {
  if (a.nblocks <= 0) return;
  if (dtype == HT_F64) launch_band_t<double>(op, a, s);
  else launch_band_t<float>(op, a, s);
}

}  // namespace ht
