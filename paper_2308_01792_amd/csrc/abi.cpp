// C ABI of the hytet library: argument checking, device upload, launch
// sequencing of operators, V-cycles, iterative refinement and graphs.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <sstream>
#include <tuple>

#include "hytet_impl.hpp"
#include "p2.hpp"
#include "kernels.hpp"
#include "band.hpp"
#include "scratch.hpp"
#include "vcoef.hpp"

struct ht_mesh;
namespace ht {
// A batch: the problems' meshes laid side by side as one disjoint mesh
// (problems sorted by finest level, descending) plus the bookkeeping of the
// per-problem norms.
struct Batch {
  int nprob = 0;
  std::vector<int> order;         // merged problem -> caller index
  std::vector<int> level;         // finest level per merged problem
  std::vector<int64_t> ndofs;     // unknowns per merged problem
  int lmax = 0, lmin = 0;         // range of finest levels
  std::vector<int> pd0, pd1;      // per level: problems whose finest level it is
  std::vector<int64_t> part_off;  // per level: start of its norm partials
  int64_t part_size = 0;
  double* d_part = nullptr;
  int64_t* d_lo = nullptr;        // per merged problem: partial range
  int64_t* d_hi = nullptr;
  double* d_norm2 = nullptr;      // per merged problem
  double* h_norm2 = nullptr;      // pinned copy
};
}  // namespace ht

// Tuned tile shape of the sweep operations at one (level, dtype).
struct SweepShape {
  int J;
  bool in_i;
  int seg;
};

struct ht_mesh {
  ht::Mesh m;
  // (level, J) -> tile list on the device
  // (level, J, waves side by side in i) -> tile list on the device
  // (level, J, waves in i, planes per march segment; 0 = unsegmented)
  std::map<std::tuple<int, int, bool, int>, std::pair<int2*, int64_t>> tiles;
  // level -> walk tiles (64 i x 8 rows) for the transfer / elementwise kernels
  std::map<int, std::pair<int2*, int64_t>> walk_tiles;
  std::map<std::pair<int, int>, int> tuned_J;  // (level, dtype) -> J
  // (level, dtype) -> band-kernel work items of one cell (absent where no
  // band fits the LDS image capacity)
  std::map<std::pair<int, int>, std::pair<int2*, int64_t>> band_items;
  // (level, dtype) -> the band kernel's row table (make_band_rowtab)
  std::map<std::pair<int, int>, uint8_t*> band_rowtab;
  // (level, dtype) -> (J, waves side by side in i) of the sweep operations
  std::map<std::pair<int, int>, SweepShape> tuned_sweep;
  std::map<int, double> lambda_max;            // level -> estimate
  // (fine level, J) -> P2 k-march segments; fine level -> P2 face runs
  std::map<std::pair<int, int>, std::pair<int2*, int64_t>> p2_tiles;
  std::map<int, std::pair<int2*, int64_t>> p2_runs;
  std::map<int, std::pair<int2*, int64_t>> p2_face_tiles;
  // P2 level -> subgroup rows (g, k, j, element offset) of one cell
  std::map<int, std::pair<int4*, int64_t>> p2_pack_rows;
  bool capturing = false;
};

namespace ht {

static thread_local std::string g_last_error;
void set_error(int code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}

static int guard(const std::function<void()>& f) {
  try {
    f();
    return HT_OK;
  } catch (const Error& e) {
    set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error(HT_ERR_OOM, "host allocation failed");
    return HT_ERR_OOM;
  } catch (const std::exception& e) {
    set_error(HT_ERR_ARG, e.what());
    return HT_ERR_ARG;
  } catch (...) {
    set_error(HT_ERR_ARG, "unknown error");
    return HT_ERR_ARG;
  }
}

static void check_level(const Mesh& m, int level) {
  if (level < m.min_level || level > m.max_level)
    throw Error{HT_ERR_LEVEL, "level " + std::to_string(level) +
                                  " outside [" + std::to_string(m.min_level) +
                                  ", " + std::to_string(m.max_level) + "]"};
}
static void check_dtype(int dtype) {
  if (dtype != HT_F64 && dtype != HT_F32)
    throw Error{HT_ERR_ARG, "dtype must be HT_F64 or HT_F32"};
}
static void check_ptr(const void* p, const char* what) {
  if (!p) throw Error{HT_ERR_ARG, std::string(what) + " is NULL"};
  if (reinterpret_cast<uintptr_t>(p) % 256)
    throw Error{HT_ERR_ARG, std::string(what) + " is not 256-byte aligned"};
}
static size_t esize(int dtype) { return dtype == HT_F64 ? 8 : 4; }
// Address of the first slot of cell c0 in a level vector.
template <typename P>
static P* at_cell(P* v, int64_t c0, int level, int dtype) {
  return v ? (P*)((const char*)v + c0 * make_layout(level).stride * (int64_t)esize(dtype)) : v;
}

// Slots of a level vector: the cells of the problems present on the level.
int64_t level_slots(const Mesh& m, int level) {
  return m.act_cells[level] * make_layout(level).stride;
}

template <typename T>
static T* dalloc(size_t count, bool zero = true) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{HT_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                " bytes failed"};
  }
  if (zero) HT_CHECK_HIP(hipMemset(p, 0, count * sizeof(T)));
  return (T*)p;
}
template <typename T>
static T* upload(const std::vector<T>& v) {
  T* p = dalloc<T>(v.size(), false);
  if (!v.empty())
    HT_CHECK_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

static const int kJ[] = {4, 8, 16};
// untuned tile rows: 4 keeps the FP64 stencil kernels at three waves per SIMD
static const int kDefaultJ = 4;

// Tile groups of the stencil kernel: 62 output i x (kCellWaves x J rows),
// or (62 kCellWaves) i x J rows when the waves sit side by side in i.
// Planes per march segment of the stencil kernel's tiles: splitting a column
// into segments (each reloads two planes) evens out the work per wave;
// measured at level 8, 64 suits the stacked arrangement, 32 the side-by-side
// one.
static int march_segment(bool in_i) { return in_i ? 32 : 64; }
// segment lengths the autotuner tries for the sweeps (the shortest bounds the
// norm partials a launch may need)
static const int kSegs[] = {32, 64, 128};

// Tiles (i0, j0) of one cell; with seg > 0 (the stencil kernel) each tile is
// split into march segments of seg planes (i0, j0 | k0 << 16).
static std::vector<int2> make_tiles(int n, int J, bool in_i, int seg = 0) {
  std::vector<int2> t;
  const int GJ = in_i ? J : kCellWaves * J, GI = in_i ? 62 * kCellWaves : 62;
  for (int tj = 0; GJ * tj <= n; ++tj)
    for (int ti = 0; GI * ti + GJ * tj <= n; ++ti) {
      const int kcol = seg > 0 ? n - GI * ti - GJ * tj : 0;
      for (int k0 = 0; k0 <= kcol; k0 += (seg > 0 ? seg : 1)) t.push_back(make_int2(GI * ti, GJ * tj | (k0 << 16)));
    }
  return t;
}

// Walk tiles of one cell: (i0, j0 | k0 << 16), 64 i x 8 rows, planes k0 ..
// k0 + kWalkSeg - 1 up to n - i0 - j0; consecutive tiles are the segments of
// one column.
static std::vector<int2> make_walk_tiles(int n) {
  std::vector<int2> t;
  for (int tj = 0; 8 * tj <= n; ++tj)
    for (int ti = 0; 64 * ti + 8 * tj <= n; ++ti)
      for (int k0 = 0; k0 <= n - 64 * ti - 8 * tj; k0 += kWalkSeg)
        t.push_back(make_int2(64 * ti, (8 * tj) | (k0 << 16)));
  return t;
}

static int64_t partials_needed(const ht_mesh* h, int level) {
  const Mesh& m = h->m;
  const int n = 1 << level;
  int64_t cell_blocks = 0;
  for (int J : kJ)
    for (bool in_i : {false, true})
      cell_blocks = std::max<int64_t>(cell_blocks, kCellWaves * m.nc * (int64_t)make_tiles(n, J, in_i, kSegs[0]).size());
  // exchange blocks (exch_args): per face, per edge, then the vertices
  const int64_t exch_blocks = m.n_faces * ((n_tri(n - 2) + 256 * kExchFacePts - 1) / (256 * kExchFacePts)) +
                              m.n_edges * ((std::max(n - 1, 0) + 255) / 256) +
                              (m.n_verts + 255) / 256;
  const int64_t elem_blocks = m.nc * (int64_t)make_walk_tiles(n).size();
  return std::max(cell_blocks + exch_blocks, elem_blocks) + 512;
}

void ensure_uploaded_h(ht_mesh* h) {
  Mesh& m = h->m;
  if (m.uploaded) return;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    throw Error{HT_ERR_STATE, "no HIP device available"};
  }
  HT_CHECK_HIP(hipGetDevice(&m.device));
  m.d_cls = upload(m.cls);
  std::vector<DevPrim> dp(m.prims.size());
  std::vector<DevInc> di;
  for (size_t p = 0; p < m.prims.size(); ++p) {
    const Prim& P = m.prims[p];
    if (P.inc.size() > 32000)
      throw Error{HT_ERR_MESH, "too many cells around one primitive"};
    dp[p].inc_begin = (int32_t)di.size();
    dp[p].inc_count = (int16_t)P.inc.size();
    dp[p].dim = (int8_t)P.dim;
    dp[p].boundary = P.boundary ? 1 : 0;
    dp[p].inv_diag_unit = P.boundary ? 0.0 : 1.0 / P.diag_unit;
    // The exchange numbers a face's interior points with the face's second
    // vertex as the fast coordinate.  Faces take their vertices in the order
    // (other, fast, slow) of the first incident cell's storage: along S0 and
    // S1 rows j is fast and k slow; along the M rows of the faces j = 0 and
    // k = 0, i is fast.  That cell's copy is then read and written in
    // contiguous runs.  All incidences follow the same vertex order.
    int perm[3] = {0, 1, 2};
    if (P.dim == 2 && !P.inc.empty()) {
      const Incidence& I0 = P.inc[0];
      const int q = 6 - I0.lv[0] - I0.lv[1] - I0.lv[2];  // vertex opposite the face
      static const int order[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
      for (int mm = 0; mm < 3; ++mm)
        for (int v = 0; v < 3; ++v)
          if (I0.lv[v] == order[q][mm]) perm[mm] = v;
    }
    for (const Incidence& I : P.inc) {
      DevInc d;
      d.cell = I.cell;
      for (int mm = 0; mm < 3; ++mm) d.lv[mm] = I.lv[perm[mm]];
      d.cls = I.cls;
      di.push_back(d);
    }
  }
  m.d_prim = upload(dp);
  m.d_inc = upload(di);
  std::vector<double> cx(m.nc * 12);
  std::vector<int8_t> co(m.nc * 4);
  for (int64_t c = 0; c < m.nc; ++c) {
    int ord[4] = {0, 1, 2, 3};
    std::sort(ord, ord + 4, [&](int a, int b) { return m.cells[c].gv[a] < m.cells[c].gv[b]; });
    for (int q = 0; q < 4; ++q) {
      co[4 * c + q] = (int8_t)ord[q];
      for (int a = 0; a < 3; ++a) cx[12 * c + 3 * q + a] = m.xyz[3 * m.cells[c].gv[ord[q]] + a];
    }
  }
  m.d_cell_xyz = upload(cx);
  m.d_cell_order = upload(co);
  m.d_w64.assign(m.max_level + 1, nullptr);
  m.d_w32.assign(m.max_level + 1, nullptr);
  m.d_kc64.assign(m.max_level + 1, nullptr);
  m.d_kc32.assign(m.max_level + 1, nullptr);
  m.d_p2w64.assign(m.max_level + 1, nullptr);
  m.d_p2w32.assign(m.max_level + 1, nullptr);
  int64_t pcap = 0;
  for (int l = m.min_level; l <= m.max_level; ++l) {
    std::vector<double> w;
    level_scaled_stencils(m, l, w);
    std::vector<float> wf(w.begin(), w.end());
    m.d_w64[l] = upload(w);
    m.d_w32[l] = upload(wf);
    for (int J : kJ)
      for (bool in_i : {false, true}) {
        auto t = make_tiles(1 << l, J, in_i, march_segment(in_i));
        h->tiles[{l, J, in_i, march_segment(in_i)}] = {upload(t), (int64_t)t.size()};
      }
    {
      auto t = make_walk_tiles(1 << l);
      h->walk_tiles[l] = {upload(t), (int64_t)t.size()};
    }
    for (int dt : {HT_F64, HT_F32}) {
      std::vector<int2> it;
      if (make_band_items(1 << l, band_cap(dt == HT_F64), kBandMinRows, it)) {
        h->band_items[{l, dt}] = {upload(it), (int64_t)it.size()};
        std::vector<uint8_t> tab;
        make_band_rowtab(l, band_cap(dt == HT_F64), (int)esize(dt), it, tab);
        h->band_rowtab[{l, dt}] = upload(tab);
      }
    }
    pcap = std::max(pcap, partials_needed(h, l));
  }
  m.d_partials = dalloc<double>(pcap);
  m.partials_cap = pcap;
  m.d_scalar = dalloc<double>(16);
  HT_CHECK_HIP(hipHostMalloc((void**)&m.h_scalar, 16 * sizeof(double), hipHostMallocDefault));
  HT_CHECK_HIP(hipStreamCreateWithFlags(&m.capture_stream, hipStreamNonBlocking));
  m.work64.assign(m.max_level + 1, LevelWork{});
  m.work32.assign(m.max_level + 1, LevelWork{});
  m.uploaded = true;
}

// --------------------------------------------------------- profiling ----
struct Prof {
  ht_mesh* h;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Prof(ht_mesh* h_, const char* n, hipStream_t s_) : h(h_), name(n), s(s_) {
    if (h->m.profiling && !h->capturing) {
      HT_CHECK_HIP(hipEventCreate(&a));
      HT_CHECK_HIP(hipEventCreate(&b));
      HT_CHECK_HIP(hipEventRecord(a, s));
    }
  }
  ~Prof() {
    if (a) {
      (void)hipEventRecord(b, s);
      h->m.prof.push_back({name, a, b});
    }
  }
};

static void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{HT_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

// -------------------------------------------------------- operators -----
// Tile rows of the apply; 0 selects the band kernel (band.hip), the FP64
// default wherever its LDS image fits (measured faster than every tile
// shape in FP64 at level 8, slower in FP32, where tile rows 4 stay the
// default).  The autotuner times both.
static bool has_band(const ht_mesh* h, int level, int dtype) {
  (void)h;
  // a function of (level, dtype) only: tabulated once
  static const std::vector<std::array<bool, 2>> ok = [] {
    std::vector<std::array<bool, 2>> t(kBandMaxLevel + 1);
    std::vector<int2> it;
    for (int l = 0; l <= kBandMaxLevel; ++l)
      for (int d = 0; d < 2; ++d)
        t[l][d] = make_band_items(1 << l, band_cap(d == HT_F64), kBandMinRows, it);
    return t;
  }();
  return level >= 0 && level <= kBandMaxLevel && ok[level][dtype == HT_F64 ? 0 : 1];
}
static int choose_J(ht_mesh* h, int level, int dtype) {
  auto it = h->tuned_J.find({level, dtype});
  if (it != h->tuned_J.end()) return it->second;
  return has_band(h, level, dtype) ? 0 : kDefaultJ;
}

// Tile shape of a stencil launch: rows per wave and wave arrangement.  The
// apply and the restriction stack the waves in j with the tuned J; the
// sweep operations use their own tuned shape, by default four rows with the
// waves side by side in i where all four have points on the longest rows
// (n >= 187, measured faster there) and stacked in j below.
struct Shape {
  int J;          // rows per wave of the tile kernel; 0 = the band kernel
  bool in_i;
  int seg;        // planes per march segment
};
// operations the band kernel runs
static bool band_op(int op) {
  return op == OP_APPLY || op == OP_JACOBI || op == OP_RESID || op == OP_RESID32 ||
         op == OP_RESID32X || op == OP_JACOBIADD;
}
// untuned sweeps use the band kernel from this level on (measured at level 8:
// Jacobi 4.22 against 4.94 ms in FP64, 2.49 against 2.78 ms in FP32); below,
// where the kernels are short, the tile kernel
static const int kBandSweepLevel = 7;
static Shape choose_shape(ht_mesh* h, int level, int dtype, int op) {
  if (op == OP_APPLY) return Shape{choose_J(h, level, dtype), false, march_segment(false)};
  const bool in_i = (1 << level) >= 62 * (kCellWaves - 1) + 1;
  // the sweep that adds its result to an FP64 iterate exists on the band
  // kernel only; it replaces a sweep plus a separate update pass, so it runs
  // there whatever shape the other sweeps take
  if (op == OP_JACOBIADD)
    return (level >= kBandSweepLevel && has_band(h, level, dtype))
               ? Shape{0, in_i, march_segment(in_i)}
               : Shape{kDefaultJ, in_i, march_segment(in_i)};
  if (!op_is_sweep(op)) {
    const int J = choose_J(h, level, dtype);
    return Shape{J == 0 ? kDefaultJ : J, false, march_segment(false)};
  }
  auto it = h->tuned_sweep.find({level, dtype});
  if (it != h->tuned_sweep.end()) {
    // the band kernel (J = 0) runs the Jacobi sweep and the residual; the
    // other sweep operations take the default tile shape then
    if (it->second.J != 0 || band_op(op))
      return Shape{it->second.J, it->second.in_i, it->second.seg};
  } else if (band_op(op) && level >= kBandSweepLevel && has_band(h, level, dtype)) {
    return Shape{0, in_i, march_segment(in_i)};
  }
  return Shape{kDefaultJ, in_i, march_segment(in_i)};
}
// Segmented tiles of a shape, uploaded on first use (never under graph
// capture: the defaults exist from set-up, and the autotuner and the shape
// setters create the others before any launch uses them).
static const std::pair<int2*, int64_t>& seg_tiles(ht_mesh* h, int level, int J, bool in_i,
                                                  int seg) {
  auto it = h->tiles.find({level, J, in_i, seg});
  if (it == h->tiles.end()) {
    auto t = make_tiles(1 << level, J, in_i, seg);
    it = h->tiles.emplace(std::make_tuple(level, J, in_i, seg),
                          std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  return it->second;
}

// Stencil-kernel arguments over the cells of R: every per-cell array is
// addressed from the range's first cell.
static const void* level_weights(ht_mesh* h, int level, int dtype) {
  return dtype == HT_F64 ? (const void*)h->m.d_w64[level] : (const void*)h->m.d_w32[level];
}
static CellArgs cell_args(ht_mesh* h, int level, int dtype, const Shape& sh,
                          const void* x, void* y, const void* b, double omega,
                          const Range& R) {
  Mesh& m = h->m;
  const CellLayout L = make_layout(level);
  CellArgs a{};
  a.x = at_cell(x, R.c0, level, dtype);
  a.y = at_cell(y, R.c0, level, dtype);
  a.b = at_cell(b, R.c0, level, dtype);
  a.w = (const char*)level_weights(h, level, dtype) + R.c0 * 240 * (int64_t)esize(dtype);
  a.cls = m.d_cls + 16 * R.c0;
  a.partials = m.d_partials;
  auto& t = h->tiles.at({level, sh.J, sh.in_i, sh.seg});
  a.waves_in_i = sh.in_i ? 1 : 0;
  a.kseg = sh.seg;
  a.tiles = t.first;
  a.ntiles = t.second;
  a.nblocks = (R.c1 - R.c0) * t.second;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.n = L.n;
  a.omega = omega;
  a.nscale = (double)L.n;
  return a;
}

// Band-kernel arguments over the cells of R.
static BandArgs band_args(ht_mesh* h, int level, int dtype, const void* x, void* y,
                          const Range& R, const void* b = nullptr, double omega = 0.0,
                          double* partials = nullptr) {
  const CellLayout L = make_layout(level);
  BandArgs a{};
  a.x = at_cell(x, R.c0, level, dtype);
  a.y = at_cell(y, R.c0, level, dtype);
  a.b = at_cell(b, R.c0, level, dtype);
  a.cls = h->m.d_cls + 16 * R.c0;
  a.partials = partials;
  a.omega = omega;
  a.nscale = (double)L.n;
  a.w = (const char*)level_weights(h, level, dtype) + R.c0 * 240 * (int64_t)esize(dtype);
  const auto& it = h->band_items.at({level, dtype});
  a.items = it.first;
  a.rtab = h->band_rowtab.at({level, dtype});
  a.nitems = it.second;
  a.nblocks = (R.c1 - R.c0) * it.second;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.n = L.n;
  return a;
}

// Exchange arguments over the shared primitives of R; vectors and weights
// stay absolute (incidences name absolute cells).
static ExchArgs exch_args(ht_mesh* h, int level, void* y, const void* u,
                          const void* b, double omega, double* partials,
                          const Range& R) {
  Mesh& m = h->m;
  const CellLayout L = make_layout(level);
  const int n = L.n;
  ExchArgs a{};
  a.y = y; a.u = u; a.b = b;
  a.prim = m.d_prim; a.inc = m.d_inc;
  a.partials = partials;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.n = n;
  a.n_faces = R.f1 - R.f0; a.n_edges = R.e1 - R.e0;
  a.prim_f0 = R.f0;
  a.prim_e0 = m.n_faces + R.e0;
  a.prim_v0 = m.n_faces + m.n_edges + R.v0;
  a.face_pts = n_tri(n - 2);
  a.face_end = a.n_faces * a.face_pts;
  a.edge_end = a.face_end + a.n_edges * std::max(n - 1, 0);
  a.total = a.edge_end + (R.v1 - R.v0);
  a.bpf = (a.face_pts + 256 * kExchFacePts - 1) / (256 * kExchFacePts);
  a.bpe = (std::max(n - 1, 0) + 255) / 256;
  a.fblk = a.n_faces * a.bpf;
  a.eblk = a.n_edges * a.bpe;
  a.nverts = R.v1 - R.v0;
  a.nblocks = a.fblk + a.eblk + (a.nverts + 255) / 256;
  a.omega = omega;
  a.nscale = (double)n;
  return a;
}

// One operator pass (cell kernel + ghost exchange).  For OP_RESID,
// OP_RESID32 and OP_JACOBI the norm of b - A x (x: the operand) lands in
// m.d_scalar[slot] (device) when want_norm.  OP_RESID32 (FP64 only) delivers
// the residual in the FP32 vector y32 and uses y as FP64 scratch.
// Norm partials of one residual / Jacobi pass over R: one per stencil-kernel
// wave plus one per exchange block.
static int64_t pass_partials(ht_mesh* h, int level, int dtype, int op, const Range& R);

// Extra output of the fused refinement passes: the first zero-guess sweep
// of the next correction (OP_RESID32X), the FP64 iterate that the last sweep
// of a correction is added to (OP_JACOBIADD).
struct Fuse {
  void* efirst = nullptr;
  double* uadd = nullptr;
};

static void op_pass(ht_mesh* h, int level, int dtype, int op, const void* x,
                    void* y, const void* b, double omega, hipStream_t s,
                    bool want_norm, int scalar_slot, const Range& R,
                    void* y32 = nullptr, double* partials = nullptr,
                    double* norm_dst = nullptr, const Fuse* fuse = nullptr) {
  Mesh& m = h->m;
  if (R.empty()) return;
  if (!partials) partials = m.d_partials;
  if (!norm_dst) norm_dst = m.d_scalar + scalar_slot;
  const Shape sh = choose_shape(h, level, dtype, op);
  if (sh.J == 0 && band_op(op)) {
    BandArgs ba = band_args(h, level, dtype, x, y, R, b, omega, partials);
    ba.y32 = (float*)at_cell(y32, R.c0, level, HT_F32);
    if (fuse) ba.efirst = (float*)at_cell(fuse->efirst, R.c0, level, HT_F32);
    if (fuse) ba.uadd = (double*)at_cell(fuse->uadd, R.c0, level, HT_F64);
    const bool res = op == OP_RESID || op == OP_RESID32 || op == OP_RESID32X;
    {
      Prof p(h, op == OP_APPLY ? "cell_apply" : res ? "cell_residual" : "cell_jacobi", s);
      launch_band(dtype, op, ba, s);
      check_launch();
    }
    ExchArgs ea = exch_args(h, level, y, (op == OP_JACOBI || op == OP_JACOBIADD) ? x : nullptr,
                            b, omega, partials + kBandComputeWaves * ba.nblocks, R);
    if (res) ea.u = x;
    ea.y32 = y32;
    if (fuse) ea.efirst = fuse->efirst;
    if (fuse) ea.uadd = fuse->uadd;
    if (ea.total > 0) {
      Prof p(h, "exchange", s);
      launch_exchange(dtype, op, ea, s);
      check_launch();
    }
    if (op != OP_APPLY && want_norm) {
      const int64_t cnt = kBandComputeWaves * ba.nblocks + ea.nblocks;
      Prof p(h, "norm_sum", s);
      launch_sum_partials(partials, cnt, norm_dst, true, s);
      check_launch();
    }
    return;
  }
  if (op == OP_JACOBIADD)
    throw Error{HT_ERR_STATE, "the sweep added to the iterate runs on the band kernel only"};
  CellArgs ca = cell_args(h, level, dtype, sh, x, y, b, omega, R);
  ca.y32 = at_cell(y32, R.c0, level, HT_F32);
  ca.partials = partials;
  if (fuse) ca.efirst = at_cell(fuse->efirst, R.c0, level, HT_F32);
  {
    const bool res = op == OP_RESID || op == OP_RESID32 || op == OP_RESID32X;
    Prof p(h, op == OP_APPLY ? "cell_apply" : res ? "cell_residual" : "cell_jacobi", s);
    launch_cell(dtype, op, sh.J, ca, s);
    check_launch();
  }
  ExchArgs ea = exch_args(h, level, y, op == OP_JACOBI ? x : nullptr, b, omega,
                          partials + kCellWaves * ca.nblocks, R);
  if (op == OP_RESID || op == OP_RESID32 || op == OP_RESID32X) ea.u = x;
  ea.y32 = y32;
  if (fuse) ea.efirst = fuse->efirst;
  if (ea.total > 0) {
    Prof p(h, "exchange", s);
    launch_exchange(dtype, op, ea, s);
    check_launch();
  }
  if ((op == OP_RESID || op == OP_RESID32 || op == OP_RESID32X || op == OP_JACOBI) &&
      want_norm) {
    const int64_t cnt = kCellWaves * ca.nblocks + ea.nblocks;
    Prof p(h, "norm_sum", s);
    launch_sum_partials(partials, cnt, norm_dst, true, s);
    check_launch();
  }
}

static int64_t pass_partials(ht_mesh* h, int level, int dtype, int op, const Range& R) {
  const Shape sh = choose_shape(h, level, dtype, op);
  const ExchArgs ea = exch_args(h, level, nullptr, nullptr, nullptr, 0.0, nullptr, R);
  if (sh.J == 0 && band_op(op))
    return kBandComputeWaves * band_args(h, level, dtype, nullptr, nullptr, R).nblocks +
           ea.nblocks;
  const CellArgs ca = cell_args(h, level, dtype, sh, nullptr, nullptr, nullptr, 0.0, R);
  return kCellWaves * ca.nblocks + ea.nblocks;
}

static void op_pass(ht_mesh* h, int level, int dtype, int op, const void* x,
                    void* y, const void* b, double omega, hipStream_t s,
                    bool want_norm = false, int scalar_slot = 0) {
  op_pass(h, level, dtype, op, x, y, b, omega, s, want_norm, scalar_slot,
          full_range(h->m));
}

// ------------------------------------------- variable coefficient -------
// Tile rows of the div(k grad) kernel: two rows per wave keep the planes of
// x and k and the 24 micro-cell sums within the register file.
static const int kVcoefJ = 2;

// Level-scaled couplings of the six shapes per cell, K_t / (4 n): the 1/4
// turns the sum of k over a micro-cell's vertices into their mean, and the
// micro-cells of level l are the unit shapes scaled by 1/n.
static const void* vcoef_couplings(ht_mesh* h, int level, int dtype) {
  Mesh& m = h->m;
  if (!m.d_kc64[level]) {
    const double sc = 1.0 / (4.0 * (double)(1 << level));
    std::vector<double> k(m.nc * kVcoefPerCell);
    for (int64_t c = 0; c < m.nc; ++c)
      for (int t = 0; t < 6; ++t)
        for (int p = 0; p < 6; ++p) k[c * kVcoefPerCell + 6 * t + p] = m.cells[c].shape_k[t][p] * sc;
    std::vector<float> kf(k.begin(), k.end());
    m.d_kc64[level] = upload(k);
    m.d_kc32[level] = upload(kf);
  }
  return dtype == HT_F64 ? (const void*)m.d_kc64[level] : (const void*)m.d_kc32[level];
}

// Unsegmented tiles for the variable-coefficient kernel, cached under -J so
// that they never mix with the stencil kernel's segmented tiles.
// Planes per march segment of the variable-coefficient kernel: a column of
// tiles near i0 = j0 = 0 spans all n + 1 planes, one near the apex a few.
static const int kVcoefSeg = 32;
static const std::pair<int2*, int64_t>& tiles_of(ht_mesh* h, int level, int J) {
  auto it = h->tiles.find({level, -J, false, kVcoefSeg});
  if (it == h->tiles.end()) {
    auto t = make_tiles(1 << level, J, false, kVcoefSeg);
    it = h->tiles.emplace(std::make_tuple(level, -J, false, kVcoefSeg),
                          std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  return it->second;
}

// One march of the variable-coefficient kernel in `mode` over all cells;
// VC_APPLY and VC_STORED are followed by the exchange, which sums the
// partial rows (zero at Dirichlet points).
static void vcoef_pass(ht_mesh* h, int level, int dtype, int mode,
                       const void* kappa, const void* x, void* rows, void* y,
                       hipStream_t s) {
  Mesh& m = h->m;
  const CellLayout L = make_layout(level);
  VCellArgs a{};
  a.x = x; a.kappa = kappa; a.y = y; a.w = rows;
  if (mode != VC_STORED) a.kc = vcoef_couplings(h, level, dtype);
  const auto& t = tiles_of(h, level, kVcoefJ);
  a.tiles = t.first;
  a.ntiles = t.second;
  a.nblocks = m.nc * t.second;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.n = L.n;
  a.kseg = kVcoefSeg;
  {
    Prof p(h, mode == VC_APPLY ? "cell_divkgrad" : mode == VC_STORED ? "cell_stored" : "assemble", s);
    launch_vcell(dtype, mode, kVcoefJ, a, s);
    check_launch();
  }
  if (mode == VC_ASSEMBLE) return;
  ExchArgs ea = exch_args(h, level, y, nullptr, nullptr, 0.0, m.d_partials, full_range(m));
  if (ea.total > 0) {
    Prof p(h, "exchange", s);
    launch_exchange(dtype, OP_APPLY, ea, s);
    check_launch();
  }
}

// Stored rows of one cell are addressed by 32-bit byte offsets.
static void check_stored_level(int level, int dtype) {
  if (15 * make_layout(level).stride * (int64_t)esize(dtype) >= (int64_t)1 << 31)
    throw Error{HT_ERR_LEVEL, "stored rows of one cell exceed 2 GiB at this level"};
}

// ------------------------------------------------------------- P2 --------
// Bulk P2 kernel: k-march segments of p2_march_rows() rows (five planes of
// J + 4 rows in a register ring); measured at P2 level 7: J = 2 in FP64,
// J = 4 in FP32, 40-plane segments.
static int p2_march_rows(int dtype) { return dtype == HT_F64 ? 2 : 4; }
static const int kP2MarchSeg = 40;  // planes per march segment, multiple of 10

// Level-scaled P2 stencils of every cell, K / 2^l at P2 level l.
static const void* p2_weights(ht_mesh* h, int level, int dtype) {
  Mesh& m = h->m;
  if (m.p2_unit.empty()) {
    std::vector<double> u(m.nc * (int64_t)kP2PerCell);
    parallel_for(m.nc, [&](int64_t a, int64_t b) {
      for (int64_t c = a; c < b; ++c) {
        double X[4][3];
        for (int q = 0; q < 4; ++q)
          for (int d = 0; d < 3; ++d) X[q][d] = m.xyz[3 * m.cells[c].gv[q] + d];
        p2_cell_weights(X, u.data() + c * kP2PerCell);
      }
    }, 8);
    m.p2_unit.swap(u);
  }
  if (!m.d_p2w64[level]) {
    const double sc = std::ldexp(1.0, -level);
    std::vector<double> w(m.p2_unit.size());
    for (size_t t = 0; t < w.size(); ++t) w[t] = m.p2_unit[t] * sc;
    std::vector<float> wf(w.begin(), w.end());
    m.d_p2w64[level] = upload(w);
    m.d_p2w32[level] = upload(wf);
  }
  return dtype == HT_F64 ? (const void*)m.d_p2w64[level] : (const void*)m.d_p2w32[level];
}

// k-march segments of one cell at fine n: (j0 | k0 << 16, i0) for rows
// j0 .. j0 + J - 1, points i0 + 2 .. i0 + 125 and planes k0 .. k0 + seg - 1
// up to the last plane where row j0 has a point 1 <= i <= e - 1.
static std::vector<int2> make_p2_columns(int n, int J, int seg) {
  // segment-major: the waves of a workgroup, and neighbouring workgroups,
  // march the same planes over neighbouring rows and share their halo rows
  // in cache
  std::vector<int2> t;
  for (int k0 = 0; k0 <= n - 2; k0 += seg)
    for (int j0 = 0; n - j0 >= 2; j0 += J)
      for (int i0 = -2; i0 + 2 <= n - j0 - 1; i0 += kP2TileI) {
        const int kcol = n - j0 - std::max(2, i0 + 3);
        if (k0 <= kcol) t.push_back(make_int2(j0 | (k0 << 16), i0));
      }
  return t;
}
// Face work of one cell (faces i = 0, side 0, and i = n - j - k, side 1):
//   face tiles (k0 | side << 16, jb): the points of the rows
//     1 <= j <= n - k - 1 of the planes k0 .. k0 + kP2FaceK - 1, rows
//     jb .. jb + kP2FaceRows - 1, which share one boundary class per plane;
//   edge runs (side << 16 | s << 17 | edge << 19, k0): the 64 points
//     k = k0 + 2 lane + s of the edge j = 0 (edge 0) or, on face i = 0, of
//     the edge j = n - k with k < n (edge 1), each with its own class.
static std::vector<int2> make_p2_face_tiles(int n) {
  std::vector<int2> t;
  for (int side = 0; side < 2; ++side)
    for (int k0 = 0; k0 <= n - 2; k0 += kP2FaceK)
      for (int jb = 0; jb <= n - k0 - 1; jb += kP2FaceRows)
        t.push_back(make_int2(k0 | (side << 16), jb));
  return t;
}
static std::vector<int2> make_p2_edge_runs(int n) {
  std::vector<int2> t;
  for (int side = 0; side < 2; ++side)
    for (int edge = 0; edge < (side == 0 ? 2 : 1); ++edge) {
      const int kmax = side == 0 ? (edge ? n - 1 : n) : n - 1;
      for (int k0 = 0; k0 <= kmax; k0 += 128)
        for (int s = 0; s < 2 && k0 + s <= kmax; ++s)
          t.push_back(make_int2((side << 16) | (s << 17) | (edge << 19), k0));
    }
  return t;
}

// y = A_P2 x at P2 level `level` (vectors in the layout of level + 1): bulk
// and face kernels, then the exchange of the finer level, which sums the
// partial rows of shared points and zeroes Dirichlet rows.
static void p2_pass(ht_mesh* h, int level, int dtype, const void* x, void* y,
                    hipStream_t s) {
  Mesh& m = h->m;
  const int lf = level + 1;
  const CellLayout L = make_layout(lf);
  const int J = p2_march_rows(dtype);
  auto tiles = h->p2_tiles.find({lf, J});
  if (tiles == h->p2_tiles.end()) {
    auto t = make_p2_columns(L.n, J, kP2MarchSeg);
    tiles = h->p2_tiles.emplace(std::make_pair(lf, J),
                                std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  auto runs = h->p2_runs.find(lf);
  if (runs == h->p2_runs.end()) {
    auto t = make_p2_edge_runs(L.n);
    runs = h->p2_runs.emplace(lf, std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  auto ftiles = h->p2_face_tiles.find(lf);
  if (ftiles == h->p2_face_tiles.end()) {
    auto t = make_p2_face_tiles(L.n);
    ftiles = h->p2_face_tiles.emplace(lf, std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  P2Args a{};
  a.x = x; a.y = y;
  a.w = p2_weights(h, level, dtype);
  a.tiles = tiles->second.first;
  a.ntiles = tiles->second.second;
  a.nblk = (a.ntiles + 3) / 4;
  a.ftiles = ftiles->second.first;
  a.nftiles = ftiles->second.second;
  a.runs = runs->second.first;
  a.nruns = runs->second.second;
  a.nfblk = (a.nruns + 3) / 4;
  a.nc = m.nc;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.n = L.n;
  a.kseg = kP2MarchSeg;
  {
    P2Args b = a;  // bulk kernel only
    b.nfblk = 0;
    b.nftiles = 0;
    Prof p(h, "cell_p2", s);
    launch_p2(dtype, J, b, s);
    check_launch();
  }
  {
    P2Args f = a;  // face kernel only
    f.nblk = 0;
    Prof p(h, "face_p2", s);
    launch_p2(dtype, J, f, s);
    check_launch();
  }
  ExchArgs ea = exch_args(h, lf, y, nullptr, nullptr, 0.0, m.d_partials, full_range(m));
  if (ea.total > 0) {
    Prof p(h, "exchange", s);
    launch_exchange(dtype, OP_APPLY, ea, s);
    check_launch();
  }
}

// Subgroup rows of one cell at P2 level `level`: (g, k, j, offset of subgroup
// g's array for one component), subgroups in the order vertex, x, y, z, xy,
// xz, yz, xyz with widths 2^l + 1, 2^l (six times), 2^l - 1.
static std::vector<int4> make_p2_pack_rows(int level) {
  std::vector<int4> t;
  const int n = 1 << level;
  int64_t off = 0;
  for (int g = 0; g < 8; ++g) {
    const int w = g == 0 ? n + 1 : (g == 7 ? n - 1 : n);
    for (int k = 0; k < w; ++k)
      for (int j = 0; j < w - k; ++j) t.push_back(make_int4(g, k, j, (int)off));
    off += n_tet(w);
  }
  return t;
}

static void p2_pack_pass(ht_mesh* h, int level, int dtype, int m, int layout,
                         const void* lattice, void* arrays, bool unpack,
                         hipStream_t s) {
  Mesh& m_ = h->m;
  const int lf = level + 1;
  const CellLayout L = make_layout(lf);
  auto rows = h->p2_pack_rows.find(level);
  if (rows == h->p2_pack_rows.end()) {
    auto t = make_p2_pack_rows(level);
    rows = h->p2_pack_rows.emplace(level, std::make_pair(upload(t), (int64_t)t.size())).first;
  }
  P2PackArgs a{};
  a.lattice = lattice;
  a.arrays = arrays;
  a.rows = rows->second.first;
  a.nrows = rows->second.second;
  a.nc = m_.nc;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.comp_stride = level_slots(m_, lf);
  a.cell_elems = (int64_t)m * n_tet(L.n + 1);
  a.n = L.n;
  a.m = m;
  a.soa = layout == HT_LAYOUT_SOA;
  a.unpack = unpack;
  Prof p(h, unpack ? "p2_unpack" : "p2_pack", s);
  launch_p2_pack(dtype, a, s);
  check_launch();
}

static void exch_only(ht_mesh* h, int level, int dtype, int op, void* v,
                      double fill, hipStream_t s) {
  ExchArgs ea = exch_args(h, level, v, nullptr, nullptr, 0.0, h->m.d_partials,
                          full_range(h->m));
  if (ea.total == 0) return;
  ea.fill = fill;
  Prof p(h, op == OP_SYNC ? "sync" : "fill", s);
  launch_exchange(dtype, op, ea, s);
  check_launch();
}

// Elementwise-kernel arguments over the cells of R (vectors must be given
// at_cell(v, R.c0, ...) by the caller).
static ElemArgs elem_args(ht_mesh* h, int level, const Range& R) {
  Mesh& m = h->m;
  const CellLayout L = make_layout(level);
  ElemArgs a{};
  a.cls = m.d_cls + 16 * R.c0;
  a.partials = m.d_partials;
  a.cell_xyz = m.d_cell_xyz + 12 * R.c0;
  a.cell_order = m.d_cell_order + 4 * R.c0;
  a.ncells = R.c1 - R.c0;
  a.n = L.n;
  a.stride = L.stride; a.off_s0 = L.off_s0; a.off_s1 = L.off_s1;
  a.nscale = (double)L.n;
  auto& t = h->walk_tiles.at(level);
  a.tiles = t.first;
  a.ntiles = t.second;
  a.nblocks = a.ncells * t.second;
  return a;
}
static ElemArgs elem_args(ht_mesh* h, int level) {
  return elem_args(h, level, full_range(h->m));
}

static void flat(ht_mesh* h, int level, int dto, int dti, int fop, void* out,
                 const void* in, hipStream_t s) {
  FlatArgs a{out, in, level_slots(h->m, level)};
  if (a.count == 0) return;
  Prof p(h, "flat", s);
  launch_flat(dto, dti, fop, a, s);
  check_launch();
}

// flat over the cells of R only
static void flat_range(ht_mesh* h, int level, int dto, int dti, int fop,
                       void* out, const void* in, hipStream_t s, const Range& R) {
  FlatArgs a{at_cell(out, R.c0, level, dto), at_cell(in, R.c0, level, dti),
             (R.c1 - R.c0) * make_layout(level).stride};
  if (a.count == 0) return;
  Prof p(h, "flat", s);
  launch_flat(dto, dti, fop, a, s);
  check_launch();
}

static void zero_guess_sweep(ht_mesh* h, int level, int dtype, double omega,
                             void* u, const void* b, hipStream_t s,
                             const Range& R) {
  if (R.empty()) return;
  ElemArgs a = elem_args(h, level, R);
  a.out = at_cell(u, R.c0, level, dtype);
  a.in0 = at_cell(b, R.c0, level, dtype);
  a.alpha = omega;
  Prof p(h, "zero_guess", s);
  launch_elem(dtype, EOP_ZERO_GUESS, a, s);
  check_launch();
}

static void restrict_pass(ht_mesh* h, int fine, int dtype, const void* rf,
                          void* rc, hipStream_t s, const Range& R) {
  Mesh& m = h->m;
  if (R.empty()) return;
  const CellLayout Lc = make_layout(fine - 1);
  const Shape sh = choose_shape(h, fine, dtype, OP_RESTRICT);
  CellArgs ca = cell_args(h, fine, dtype, sh, rf, nullptr, nullptr, 0.0, R);
  ca.y = at_cell(rc, R.c0, fine - 1, dtype);
  ca.stride_out = Lc.stride;
  ca.off_s0_out = Lc.off_s0;
  ca.off_s1_out = Lc.off_s1;
  {
    Prof p(h, "restrict", s);
    launch_cell(dtype, OP_RESTRICT, sh.J, ca, s);
    check_launch();
  }
  ExchArgs ea = exch_args(h, fine - 1, rc, nullptr, nullptr, 0.0, m.d_partials, R);
  if (ea.total == 0) return;
  Prof p(h, "exchange", s);
  launch_exchange(dtype, OP_RESTRICT, ea, s);
  check_launch();
}

static void prolong_pass(ht_mesh* h, int coarse, int dtype, const void* ec,
                         void* uf, hipStream_t s, const Range& R) {
  Mesh& m = h->m;
  if (R.empty()) return;
  const CellLayout Lf = make_layout(coarse + 1), Lc = make_layout(coarse);
  XferArgs a{};
  a.src = at_cell(ec, R.c0, coarse, dtype);
  a.dst = at_cell(uf, R.c0, coarse + 1, dtype);
  a.cls = m.d_cls + 16 * R.c0;
  a.ncells = R.c1 - R.c0;
  a.nf = Lf.n; a.nc_ = Lc.n;
  a.stride_f = Lf.stride; a.off_s0_f = Lf.off_s0; a.off_s1_f = Lf.off_s1;
  a.stride_c = Lc.stride; a.off_s0_c = Lc.off_s0; a.off_s1_c = Lc.off_s1;
  {
    auto& t = h->walk_tiles.at(coarse + 1);
    a.tiles = t.first; a.ntiles = t.second; a.nblocks = a.ncells * t.second;
  }
  Prof p(h, "prolongate", s);
  launch_prolong(dtype, a, s);
  check_launch();
}

static CoarseSolver& coarse_solver(ht_mesh* h, int level) {
  Mesh& m = h->m;
  auto it = m.coarse.find(level);
  if (it != m.coarse.end()) return it->second;
  CoarseSolver& cs = m.coarse[level];
  build_coarse_solver(m, level, cs);
  cs.d_inv = upload(cs.inv);
  cs.d_owner = upload(cs.owner_slot);
  cs.d_copy_ptr = upload(cs.copy_ptr);
  cs.d_copy_slot = upload(cs.copy_slot);
  cs.d_blk_dof = upload(cs.blk_dof);
  cs.d_blk_inv = upload(cs.blk_inv);
  cs.d_row_blk = upload(cs.row_blk);
  cs.d_rhs = dalloc<double>(std::max<int64_t>(cs.ndof, 1));
  return cs;
}

// u_I = A_II^-1 b_I, Dirichlet slots of u untouched (assumed zero data).
static void coarse_fast(ht_mesh* h, int level, int dtype, const void* b,
                        void* u, hipStream_t s) {
  CoarseSolver& cs = coarse_solver(h, level);
  CoarseArgs a{b, u, cs.d_inv, cs.d_owner, cs.d_copy_ptr, cs.d_copy_slot,
               cs.d_blk_dof, cs.d_blk_inv, cs.d_row_blk, cs.d_rhs, cs.ndof};
  Prof p(h, "coarse_solve", s);
  launch_coarse(dtype, a, s);
  check_launch();
}

static LevelWork& work(ht_mesh* h, int level, int dtype) {
  Mesh& m = h->m;
  LevelWork& w = (dtype == HT_F64 ? m.work64 : m.work32)[level];
  if (!w.t) {
    const size_t n = level_slots(m, level) * esize(dtype);
    w.u = dalloc<char>(n);
    w.b = dalloc<char>(n);
    w.t = dalloc<char>(n);
  }
  return w;
}

// Weighted Jacobi sweeps between two buffers; returns the buffer holding the
// result (cur or other).
static void* sweeps(ht_mesh* h, int level, int dtype, double omega, int count,
                    void* cur, void* other, const void* b, hipStream_t s) {
  for (int k = 0; k < count; ++k) {
    op_pass(h, level, dtype, OP_JACOBI, cur, other, b, omega, s);
    std::swap(cur, other);
  }
  return cur;
}

static void* smooth(ht_mesh* h, int level, int dtype, const ht_cycle_opts& o,
                    int count, void* cur, void* other, const void* b,
                    hipStream_t s);
static double norm_of(ht_mesh* h, int level, int dtype, const void* a,
                      const void* b, hipStream_t s, bool sq);

// Whether the last sweep of an FP32 correction on `level` can add its result
// to an FP64 iterate (OP_JACOBIADD runs on the band kernel).
static bool can_add_last_sweep(ht_mesh* h, int level, const ht_cycle_opts& o) {
  return o.smoother == HT_SMOOTH_JACOBI && o.nu2 > 0 && level > o.coarse_level &&
         choose_shape(h, level, HT_F32, OP_JACOBIADD).J == 0;
}

// V(nu1, nu2) on `level`: iterate in u (or t), returns the buffer with the
// new iterate.  zero_guess: the incoming iterate is zero.  first_done: the
// first pre-smoothing sweep has already been made from u into t.  uadd (FP32
// cycles where can_add_last_sweep holds): the last post-smoothing sweep adds
// its result to this FP64 vector instead of storing it; the returned buffer
// is then the one that sweep would have written, and holds scratch.
static void* vcycle_impl(ht_mesh* h, int level, int dtype,
                         const ht_cycle_opts& o, void* u, void* t,
                         const void* b, bool zero_guess, hipStream_t s,
                         bool first_done = false, double* uadd = nullptr) {
  if (level == o.coarse_level) {
    coarse_fast(h, level, dtype, b, u, s);
    return u;
  }
  void* cur = first_done ? t : u;
  void* other = first_done ? u : t;
  int todo = first_done ? o.nu1 - 1 : o.nu1;
  if (zero_guess) {
    if (todo > 0 && o.smoother == HT_SMOOTH_JACOBI) {
      zero_guess_sweep(h, level, dtype, o.omega, cur, b, s, full_range(h->m));
      --todo;
    } else {
      flat(h, level, dtype, dtype, FOP_ZERO, cur, nullptr, s);
    }
  }
  cur = smooth(h, level, dtype, o, todo, cur, other, b, s);
  other = (cur == u) ? t : u;
  op_pass(h, level, dtype, OP_RESID, cur, other, b, 0.0, s);
  LevelWork& wc = work(h, level - 1, dtype);
  restrict_pass(h, level, dtype, other, wc.b, s, full_range(h->m));
  void* ec = vcycle_impl(h, level - 1, dtype, o, wc.u, wc.t, wc.b, true, s);
  prolong_pass(h, level - 1, dtype, ec, cur, s, full_range(h->m));
  if (!uadd) return smooth(h, level, dtype, o, o.nu2, cur, other, b, s);
  if (dtype != HT_F32 || !can_add_last_sweep(h, level, o))
    throw Error{HT_ERR_STATE, "the last sweep cannot be added to the iterate here"};
  cur = smooth(h, level, dtype, o, o.nu2 - 1, cur, other, b, s);
  other = (cur == u) ? t : u;
  Fuse F;
  F.uadd = uadd;
  op_pass(h, level, dtype, OP_JACOBIADD, cur, other, b, o.omega, s, false, 0,
          full_range(h->m), nullptr, nullptr, nullptr, &F);
  return other;
}

static void check_cycle(const Mesh& m, int level, const ht_cycle_opts* o) {
  if (!o) throw Error{HT_ERR_ARG, "cycle options are NULL"};
  if (o->coarse_level < m.min_level || o->coarse_level > level)
    throw Error{HT_ERR_LEVEL, "coarse_level outside [min_level, level]"};
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 > 64)
    throw Error{HT_ERR_ARG, "sweep counts must be in [0, 64]"};
  if (o->smoother != HT_SMOOTH_JACOBI && o->smoother != HT_SMOOTH_CHEBYSHEV)
    throw Error{HT_ERR_ARG, "unknown smoother"};
  if (o->smoother == HT_SMOOTH_JACOBI && !(o->omega > 0.0 && o->omega < 2.0))
    throw Error{HT_ERR_ARG, "omega must lie in (0, 2)"};
  if (o->smoother == HT_SMOOTH_CHEBYSHEV && (o->degree < 1 || o->degree > 16))
    throw Error{HT_ERR_ARG, "Chebyshev degree must be in [1, 16]"};
}

// ----------------------------------------------------- Chebyshev smoother
// Largest eigenvalue of D^-1 A by power iteration (estimate cached per
// level).  Runs eagerly with two scratch vectors: call it before capture.
static double lambda_max_of(ht_mesh* h, int level, hipStream_t s) {
  auto it = h->lambda_max.find(level);
  if (it != h->lambda_max.end()) return it->second;
  Mesh& m = h->m;
  const size_t bytes = level_slots(m, level) * sizeof(double);
  double* v = dalloc<double>(level_slots(m, level));
  double* w = dalloc<double>(level_slots(m, level));
  double lam = 0.0;
  try {
    ElemArgs a = elem_args(h, level);
    a.out = v;
    a.alpha = std::ldexp(1.0, -level);
    launch_elem(HT_F64, EOP_PROBE, a, s);
    check_launch();
    double vn = norm_of(h, level, HT_F64, v, v, s, true);
    for (int it2 = 0; it2 < 20; ++it2) {
      op_pass(h, level, HT_F64, OP_APPLY, v, w, nullptr, 0.0, s);
      // w <- D^-1 w (the zero-guess sweep with weight 1), in place
      ElemArgs z = elem_args(h, level);
      z.out = w;
      z.in0 = w;
      z.alpha = 1.0;
      launch_elem(HT_F64, EOP_ZERO_GUESS, z, s);
      check_launch();
      const double wn = norm_of(h, level, HT_F64, w, w, s, true);
      lam = vn > 0 ? wn / vn : 0.0;
      vn = wn;
      std::swap(v, w);
    }
  } catch (...) {
    (void)hipFree(v);
    (void)hipFree(w);
    throw;
  }
  HT_CHECK_HIP(hipStreamSynchronize(s));
  (void)hipFree(v);
  (void)hipFree(w);
  (void)bytes;
  h->lambda_max[level] = lam;
  return lam;
}

// Everything the smoother needs on levels (coarse, level]: eigenvalue
// estimates and direction vectors.  Before any capture.
static void prepare_smoother(ht_mesh* h, int level, int dtype,
                             const ht_cycle_opts& o, hipStream_t s) {
  if (o.smoother != HT_SMOOTH_CHEBYSHEV) return;
  for (int l = o.coarse_level + 1; l <= level; ++l) {
    lambda_max_of(h, l, s);
    LevelWork& w = work(h, l, dtype);
    if (!w.d) w.d = dalloc<char>(level_slots(h->m, l) * esize(dtype));
  }
}

// One Chebyshev step (cell kernel + exchange): d <- c1 d + c2 D^-1 (b - A x),
// y = x + d.
static void cheb_pass(ht_mesh* h, int level, int dtype, const void* x, void* y,
                      const void* b, void* d, double c1, double c2,
                      hipStream_t s) {
  Mesh& m = h->m;
  const Range R = full_range(m);
  const Shape sh = choose_shape(h, level, dtype, OP_CHEB);
  CellArgs ca = cell_args(h, level, dtype, sh, x, y, b, 1.0, R);
  ca.d = at_cell(d, R.c0, level, dtype);
  ca.c1 = c1;
  ca.c2 = c2;
  {
    Prof p(h, "cell_chebyshev", s);
    launch_cell(dtype, OP_CHEB, sh.J, ca, s);
    check_launch();
  }
  ExchArgs ea = exch_args(h, level, y, x, b, 1.0, m.d_partials + kCellWaves * ca.nblocks, R);
  ea.d = d;
  ea.c1 = c1;
  ea.c2 = c2;
  if (ea.total > 0) {
    Prof p(h, "exchange", s);
    launch_exchange(dtype, OP_CHEB, ea, s);
    check_launch();
  }
}

// `count` smoother applications between two buffers; returns the buffer
// holding the result.
static void* smooth(ht_mesh* h, int level, int dtype, const ht_cycle_opts& o,
                    int count, void* cur, void* other, const void* b,
                    hipStream_t s) {
  if (o.smoother == HT_SMOOTH_JACOBI)
    return sweeps(h, level, dtype, o.omega, count, cur, other, b, s);
  const double beta = 1.1 * h->lambda_max.at(level), alpha = beta / 8.0;
  const double theta = 0.5 * (beta + alpha), delta = 0.5 * (beta - alpha);
  const double sigma = theta / delta;
  void* d = work(h, level, dtype).d;
  for (int app = 0; app < count; ++app) {
    double rho_prev = 1.0 / sigma;
    for (int k = 0; k < o.degree; ++k) {
      double c1 = 0.0, c2 = 1.0 / theta;
      if (k > 0) {
        const double rho = 1.0 / (2.0 * sigma - rho_prev);
        c1 = rho * rho_prev;
        c2 = 2.0 * rho / delta;
        rho_prev = rho;
      }
      cheb_pass(h, level, dtype, cur, other, b, d, c1, c2, s);
      std::swap(cur, other);
    }
  }
  return cur;
}

// Top-level V-cycle on caller buffers (u, b).
static void vcycle_top(ht_mesh* h, int level, int dtype, const ht_cycle_opts& o,
                       void* u, const void* b, bool zero_guess, hipStream_t s) {
  LevelWork& w = work(h, level, dtype);
  void* res = vcycle_impl(h, level, dtype, o, u, w.t, b, zero_guess, s);
  if (res != u) flat(h, level, dtype, dtype, FOP_COPY, u, res, s);
}

static double read_scalar(ht_mesh* h, int slot, hipStream_t s) {
  Mesh& m = h->m;
  HT_CHECK_HIP(hipMemcpyAsync(m.h_scalar + slot, m.d_scalar + slot, sizeof(double),
                              hipMemcpyDeviceToHost, s));
  HT_CHECK_HIP(hipStreamSynchronize(s));
  return m.h_scalar[slot];
}

static double norm_of(ht_mesh* h, int level, int dtype, const void* a,
                      const void* b, hipStream_t s, bool sq) {
  ElemArgs ea = elem_args(h, level);
  ea.in0 = a; ea.in1 = b;
  {
    Prof p(h, "dot", s);
    launch_elem(dtype, EOP_DOT, ea, s);
    check_launch();
  }
  launch_sum_partials(h->m.d_partials, ea.nblocks, h->m.d_scalar + 1, sq, s);
  check_launch();
  return read_scalar(h, 1, s);
}

// Capture `body` into a graph cached under `key` and launch it on s.
static void run_graph(ht_mesh* h, const std::string& key,
                      const std::function<void(hipStream_t)>& body,
                      hipStream_t s) {
  Mesh& m = h->m;
  auto it = m.graphs.find(key);
  if (it == m.graphs.end()) {
    hipGraph_t g = nullptr;
    h->capturing = true;
    HT_CHECK_HIP(hipStreamBeginCapture(m.capture_stream, hipStreamCaptureModeRelaxed));
    try {
      body(m.capture_stream);
    } catch (...) {
      hipGraph_t dummy;
      (void)hipStreamEndCapture(m.capture_stream, &dummy);
      h->capturing = false;
      throw;
    }
    HT_CHECK_HIP(hipStreamEndCapture(m.capture_stream, &g));
    h->capturing = false;
    GraphEntry ge;
    HT_CHECK_HIP(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
    HT_CHECK_HIP(hipGraphDestroy(g));
    it = m.graphs.emplace(key, ge).first;
  }
  HT_CHECK_HIP(hipGraphLaunch(it->second.exec, s));
}


// ------------------------------------------------------------- batch ----
// Per-problem squared norms of (which = 0) the residual b - A u or (1) b at
// each problem's finest level, into bt.d_norm2 and its pinned copy.
static void batch_norms(ht_mesh* h, Batch& bt, int which, hipStream_t s) {
  Mesh& m = h->m;
  for (int l = bt.lmax; l >= bt.lmin; --l) {
    if (bt.pd1[l] <= bt.pd0[l]) continue;
    const Range D = problem_range(m, bt.pd0[l], bt.pd1[l]);
    LevelWork& w = work(h, l, HT_F64);
    const void* v = w.b;
    if (which == 0) {
      op_pass(h, l, HT_F64, OP_RESID, w.u, w.t, w.b, 0.0, s, false, 0, D);
      v = w.t;
    }
    ElemArgs a = elem_args(h, l, D);
    a.in0 = a.in1 = at_cell(v, D.c0, l, HT_F64);
    a.partials = bt.d_part + bt.part_off[l];
    Prof p(h, "dot", s);
    launch_elem(HT_F64, EOP_DOT, a, s);
    check_launch();
  }
  SegArgs sa{bt.d_part, bt.d_lo, bt.d_hi, bt.d_norm2, bt.nprob};
  launch_seg_sum(sa, s);
  check_launch();
  HT_CHECK_HIP(hipMemcpyAsync(bt.h_norm2, bt.d_norm2, bt.nprob * sizeof(double),
                              hipMemcpyDeviceToHost, s));
}

// One V-cycle over absolute levels in `dtype`.  On level l the problems
// [0, pd1[l]) are active: those with a finer finest level carry a coarse
// correction (zero initial guess, right-hand side restricted from l + 1),
// those whose finest level is l carry their iterate.  A correction cycle
// (the FP32 cycle of the refinement) starts every problem from zero: there
// each problem's right-hand side at its finest level is its FP64 residual
// rounded to FP32.  The result is left in work(l).u.
static void batch_level(ht_mesh* h, Batch& bt, int l, const ht_cycle_opts& o,
                        int dtype, bool correction, hipStream_t s) {
  Mesh& m = h->m;
  LevelWork& w = work(h, l, dtype);
  if (l == o.coarse_level) {
    coarse_fast(h, l, dtype, w.b, w.u, s);
    return;
  }
  const int pz = correction ? bt.pd1[l] : bt.pd0[l];
  const Range A = problem_range(m, 0, bt.pd1[l]);
  const Range C = problem_range(m, 0, pz);          // zero initial guess
  const Range D = problem_range(m, pz, bt.pd1[l]);  // iterate carried
  void* cur = w.u;
  void* oth = w.t;
  int todo = o.nu1;
  if (todo > 0) {
    zero_guess_sweep(h, l, dtype, o.omega, oth, w.b, s, C);
    op_pass(h, l, dtype, OP_JACOBI, cur, oth, w.b, o.omega, s, false, 0, D);
    std::swap(cur, oth);
    --todo;
  } else {
    flat_range(h, l, dtype, dtype, FOP_ZERO, cur, nullptr, s, C);
  }
  for (; todo > 0; --todo) {
    op_pass(h, l, dtype, OP_JACOBI, cur, oth, w.b, o.omega, s, false, 0, A);
    std::swap(cur, oth);
  }
  op_pass(h, l, dtype, OP_RESID, cur, oth, w.b, 0.0, s, false, 0, A);
  LevelWork& wc = work(h, l - 1, dtype);
  restrict_pass(h, l, dtype, oth, wc.b, s, A);
  batch_level(h, bt, l - 1, o, dtype, correction, s);
  prolong_pass(h, l - 1, dtype, wc.u, cur, s, A);
  for (int k = 0; k < o.nu2; ++k) {
    op_pass(h, l, dtype, OP_JACOBI, cur, oth, w.b, o.omega, s, false, 0, A);
    std::swap(cur, oth);
  }
  if (cur != w.u) flat_range(h, l, dtype, dtype, FOP_COPY, w.u, cur, s, A);
}

}  // namespace ht

struct ht_batch {
  ht_mesh* mesh = nullptr;  // the disjoint union of the problems
  ht::Batch bt;
};

using namespace ht;

// ================================================================= ABI ====
extern "C" {

const char* ht_last_error(void) { return g_last_error.c_str(); }
int ht_version(void) { return 1; }
int64_t ht_index_tw(int64_t w, int64_t i, int64_t j, int64_t k) {
  return t_w(w, i, j, k);
}

int ht_mesh_create(const double* xyz, int64_t nv, const int64_t* cells,
                   int64_t nc, int min_level, int max_level, ht_mesh** out) {
  return guard([&] {
    if (!out) throw Error{HT_ERR_ARG, "out is NULL"};
    *out = nullptr;
    auto h = std::make_unique<ht_mesh>();
    build_mesh(h->m, xyz, nv, cells, nc, min_level, max_level);
    *out = h.release();
  });
}

int ht_mesh_destroy(ht_mesh* h) {
  return guard([&] {
    if (!h) return;
    Mesh& m = h->m;
    if (m.uploaded) {
      (void)hipDeviceSynchronize();
      for (auto& kv : m.graphs) (void)hipGraphExecDestroy(kv.second.exec);
      for (auto& kv : h->tiles) (void)hipFree(kv.second.first);
      for (auto& kv : h->walk_tiles) (void)hipFree(kv.second.first);
      for (auto& kv : h->band_items) (void)hipFree(kv.second.first);
      for (auto& kv : h->band_rowtab) (void)hipFree(kv.second);
      for (auto* p : m.d_w64) if (p) (void)hipFree(p);
      for (auto* p : m.d_w32) if (p) (void)hipFree(p);
      for (auto* p : m.d_kc64) if (p) (void)hipFree(p);
      for (auto* p : m.d_kc32) if (p) (void)hipFree(p);
      for (auto* p : m.d_p2w64) if (p) (void)hipFree(p);
      for (auto* p : m.d_p2w32) if (p) (void)hipFree(p);
      for (auto& kv : h->p2_tiles) (void)hipFree(kv.second.first);
      for (auto& kv : h->p2_runs) (void)hipFree(kv.second.first);
      for (auto& kv : h->p2_face_tiles) (void)hipFree(kv.second.first);
      for (auto& kv : h->p2_pack_rows) (void)hipFree(kv.second.first);
      for (auto* list : {&m.work64, &m.work32})
        for (auto& w : *list) {
          (void)hipFree(w.u); (void)hipFree(w.b); (void)hipFree(w.t); (void)hipFree(w.d);
        }
      for (auto& kv : m.coarse) {
        (void)hipFree(kv.second.d_inv); (void)hipFree(kv.second.d_owner);
        (void)hipFree(kv.second.d_copy_ptr); (void)hipFree(kv.second.d_copy_slot);
        (void)hipFree(kv.second.d_blk_dof); (void)hipFree(kv.second.d_blk_inv);
        (void)hipFree(kv.second.d_row_blk);
        (void)hipFree(kv.second.d_rhs);
      }
      for (auto& e : m.prof) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
      (void)hipFree(m.d_cls); (void)hipFree(m.d_prim); (void)hipFree(m.d_inc);
      (void)hipFree(m.d_cell_xyz); (void)hipFree(m.d_cell_order);
      (void)hipFree(m.d_partials); (void)hipFree(m.d_scalar);
      (void)hipHostFree(m.h_scalar);
      (void)hipStreamDestroy(m.capture_stream);
    }
    delete h;
  });
}

int ht_mesh_query(const ht_mesh* h, int level, ht_level_info* info) {
  return guard([&] {
    if (!h || !info) throw Error{HT_ERR_ARG, "NULL argument"};
    const Mesh& m = h->m;
    check_level(m, level);
    const CellLayout L = make_layout(level);
    const int n = L.n;
    info->n_slots = m.nc * L.stride;
    info->cell_stride = L.stride;
    info->n_cells = m.nc;
    info->n_faces = m.n_faces;
    info->n_edges = m.n_edges;
    info->n_vertices = m.n_verts;
    int64_t uniq = m.nc * n_tet(n - 3), dofs = uniq;
    for (const Prim& p : m.prims) {
      const int64_t pts = p.dim == 2 ? n_tri(n - 2) : (p.dim == 1 ? std::max(n - 1, 0) : 1);
      uniq += pts;
      if (!p.boundary) dofs += pts;
    }
    info->n_unique = uniq;
    info->n_dofs = dofs;
  });
}

int ht_vertex_keys(const ht_mesh* h, int level, int64_t first, int64_t count,
                   int64_t* keys, uint8_t* flags) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    const int64_t ns = level_slots(h->m, level);
    if (first < 0 || count < 0 || first + count > ns)
      throw Error{HT_ERR_ARG, "slot range out of bounds"};
    parallel_for(count, [&](int64_t lo, int64_t hi) {
      for (int64_t s = lo; s < hi; ++s) {
        int64_t k[8];
        uint8_t f;
        slot_key(h->m, level, first + s, k, &f);
        if (keys) std::memcpy(keys + 8 * s, k, sizeof(k));
        if (flags) flags[s] = f;
      }
    });
  });
}

int ht_vertex_coords(const ht_mesh* h, int level, int64_t first, int64_t count,
                     double* xyz) {
  return guard([&] {
    if (!h || !xyz) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    const int64_t ns = level_slots(h->m, level);
    if (first < 0 || count < 0 || first + count > ns)
      throw Error{HT_ERR_ARG, "slot range out of bounds"};
    parallel_for(count, [&](int64_t lo, int64_t hi) {
      for (int64_t s = lo; s < hi; ++s) slot_coords(h->m, level, first + s, xyz + 3 * s);
    });
  });
}

int ht_slot_index(const ht_mesh* h, int level, int64_t cell, int i, int j,
                  int k, int64_t* slot) {
  return guard([&] {
    if (!h || !slot) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    const CellLayout L = make_layout(level);
    if (cell < 0 || cell >= h->m.nc || i < 0 || j < 0 || k < 0 || i + j + k > L.n)
      throw Error{HT_ERR_ARG, "index outside the cell closure"};
    *slot = cell * L.stride + slot_in_cell(L, i, j, k);
  });
}

int ht_cell_stencils(const ht_mesh* h, int level, double* out) {
  return guard([&] {
    if (!h || !out) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    std::vector<double> w;
    level_scaled_stencils(h->m, level, w);
    std::memcpy(out, w.data(), w.size() * sizeof(double));
  });
}

int ht_p2_offsets(int* len, int* d) {
  return guard([&] {
    if (!len || !d) throw Error{HT_ERR_ARG, "NULL argument"};
    for (int p = 0; p < kP2Parities; ++p) {
      len[p] = kP2Off.len[p];
      for (int t = 0; t < kP2MaxOffsets; ++t)
        for (int c = 0; c < 3; ++c) d[(p * kP2MaxOffsets + t) * 3 + c] = kP2Off.d[p][t][c];
    }
  });
}

int ht_p2_stencils(const ht_mesh* h, int level, double* out) {
  return guard([&] {
    if (!h || !out) throw Error{HT_ERR_ARG, "NULL argument"};
    if (level < 0) throw Error{HT_ERR_LEVEL, "P2 level must be >= 0"};
    check_level(h->m, level + 1);
    const Mesh& m = h->m;
    const double sc = std::ldexp(1.0, -level);
    for (int64_t c = 0; c < m.nc; ++c) {
      double X[4][3];
      for (int q = 0; q < 4; ++q)
        for (int d = 0; d < 3; ++d) X[q][d] = m.xyz[3 * m.cells[c].gv[q] + d];
      double* w = out + c * kP2PerCell;
      p2_cell_weights(X, w);
      for (int t = 0; t < kP2PerCell; ++t) w[t] *= sc;
    }
  });
}

int ht_vertex_coords_device(ht_mesh* h, int level, int dtype, void* xyz_dev,
                            ht_stream stream) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_dtype(dtype);
    check_ptr(xyz_dev, "xyz_dev");
    ensure_uploaded_h(h);
    ElemArgs a = elem_args(h, level);
    a.out = xyz_dev;
    a.alpha = std::ldexp(1.0, -level);
    launch_elem(dtype, EOP_COORDS, a, (hipStream_t)stream);
    check_launch();
  });
}

int ht_slot_flags_device(ht_mesh* h, int level, uint8_t* flags_dev,
                         ht_stream stream) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_ptr(flags_dev, "flags_dev");
    ensure_uploaded_h(h);
    HT_CHECK_HIP(hipMemsetAsync(flags_dev, HT_SLOT_PAD, level_slots(h->m, level),
                                (hipStream_t)stream));
    ElemArgs a = elem_args(h, level);
    a.out = flags_dev;
    launch_elem(HT_F64, EOP_FLAGS, a, (hipStream_t)stream);
    check_launch();
  });
}

#define HT_DEV_PROLOGUE(level, dtype)      \
  if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"}; \
  check_level(h->m, level);                \
  check_dtype(dtype);                      \
  ensure_uploaded_h(h);                    \
  hipStream_t s = (hipStream_t)stream;

int ht_sync(ht_mesh* h, int level, int dtype, void* v, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(v, "v");
    exch_only(h, level, dtype, OP_SYNC, v, 0.0, s);
  });
}

int ht_fill_dirichlet(ht_mesh* h, int level, int dtype, void* v, double value,
                      ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(v, "v");
    exch_only(h, level, dtype, OP_FILL, v, value, s);
  });
}

int ht_lumped_mass(ht_mesh* h, int level, int dtype, void* mvec, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(mvec, "m");
    ElemArgs a = elem_args(h, level);
    a.out = mvec;
    a.nscale = std::ldexp(1.0, -3 * level);
    launch_elem(dtype, EOP_MASS, a, s);
    check_launch();
  });
}

int ht_norm(ht_mesh* h, int level, int dtype, const void* v, double* norm,
            ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(v, "v");
    if (!norm) throw Error{HT_ERR_ARG, "norm is NULL"};
    *norm = norm_of(h, level, dtype, v, v, s, true);
  });
}

int ht_dot(ht_mesh* h, int level, int dtype, const void* a, const void* b,
           double* dot, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(a, "a");
    check_ptr(b, "b");
    if (!dot) throw Error{HT_ERR_ARG, "dot is NULL"};
    *dot = norm_of(h, level, dtype, a, b, s, false);
  });
}

int ht_copy(ht_mesh* h, int level, int dtype, const void* src, void* dst,
            ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(src, "src");
    check_ptr(dst, "dst");
    flat(h, level, dtype, dtype, FOP_COPY, dst, src, s);
  });
}

int ht_apply(ht_mesh* h, int level, int dtype, const void* x, void* y,
             ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(x, "x");
    check_ptr(y, "y");
    if (x == y) throw Error{HT_ERR_ARG, "x and y must not alias"};
    op_pass(h, level, dtype, OP_APPLY, x, y, nullptr, 0.0, s);
  });
}

int ht_apply_divkgrad(ht_mesh* h, int level, int dtype, const void* kappa,
                      const void* x, void* y, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(kappa, "kappa");
    check_ptr(x, "x");
    check_ptr(y, "y");
    if (y == x || y == kappa) throw Error{HT_ERR_ARG, "y must not alias x or kappa"};
    vcoef_pass(h, level, dtype, VC_APPLY, kappa, x, nullptr, y, s);
  });
}

int ht_assemble_divkgrad(ht_mesh* h, int level, int dtype, const void* kappa,
                         void* rows, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(kappa, "kappa");
    check_ptr(rows, "rows");
    check_stored_level(level, dtype);
    vcoef_pass(h, level, dtype, VC_ASSEMBLE, kappa, nullptr, rows, nullptr, s);
  });
}

int ht_apply_stored(ht_mesh* h, int level, int dtype, const void* rows,
                    const void* x, void* y, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(rows, "rows");
    check_ptr(x, "x");
    check_ptr(y, "y");
    if (y == x) throw Error{HT_ERR_ARG, "y must not alias x"};
    check_stored_level(level, dtype);
    vcoef_pass(h, level, dtype, VC_STORED, nullptr, x, const_cast<void*>(rows), y, s);
  });
}

int ht_apply_p2(ht_mesh* h, int level, int dtype, const void* x, void* y,
                ht_stream stream) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    if (level < 0) throw Error{HT_ERR_LEVEL, "P2 level must be >= 0"};
    HT_DEV_PROLOGUE(level + 1, dtype);
    check_ptr(x, "x");
    check_ptr(y, "y");
    if (y == x) throw Error{HT_ERR_ARG, "y must not alias x"};
    p2_pass(h, level, dtype, x, y, s);
  });
}

static void check_pack(ht_mesh* h, int level, int m, int layout) {
  if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
  if (level < 0) throw Error{HT_ERR_LEVEL, "P2 level must be >= 0"};
  if (m < 1 || m > 64) throw Error{HT_ERR_ARG, "components per node must be 1 .. 64"};
  if (layout != HT_LAYOUT_AOS && layout != HT_LAYOUT_SOA)
    throw Error{HT_ERR_ARG, "layout must be HT_LAYOUT_AOS or HT_LAYOUT_SOA"};
}

int ht_p2_pack(ht_mesh* h, int level, int dtype, int m, int layout,
               const void* lattice, void* arrays, ht_stream stream) {
  return guard([&] {
    check_pack(h, level, m, layout);
    HT_DEV_PROLOGUE(level + 1, dtype);
    check_ptr(lattice, "lattice");
    check_ptr(arrays, "arrays");
    p2_pack_pass(h, level, dtype, m, layout, lattice, arrays, false, s);
  });
}

int ht_p2_unpack(ht_mesh* h, int level, int dtype, int m, int layout,
                 const void* arrays, void* lattice, ht_stream stream) {
  return guard([&] {
    check_pack(h, level, m, layout);
    HT_DEV_PROLOGUE(level + 1, dtype);
    check_ptr(lattice, "lattice");
    check_ptr(arrays, "arrays");
    p2_pack_pass(h, level, dtype, m, layout, lattice, const_cast<void*>(arrays), true, s);
  });
}

int ht_residual(ht_mesh* h, int level, int dtype, const void* u, const void* b,
                void* r, double* norm, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(u, "u");
    check_ptr(b, "b");
    check_ptr(r, "r");
    if (r == u || r == b) throw Error{HT_ERR_ARG, "r must not alias u or b"};
    op_pass(h, level, dtype, OP_RESID, u, r, b, 0.0, s, norm != nullptr, 0);
    if (norm) *norm = read_scalar(h, 0, s);
  });
}

int ht_residual_noalloc(ht_mesh* h, int level, int dtype, const void* u,
                        const void* b, void* r, double* norm_dev, ht_stream stream) {
  // No std::function and no allocation on the success path: the checks,
  // the scratch lookup and the launches only.
  try {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_dtype(dtype);
    if (!h->m.uploaded)
      throw Error{HT_ERR_STATE, "the mesh is not on the device yet: call a device "
                                "entry point (e.g. ht_apply) once before, since "
                                "uploading it allocates"};
    check_ptr(u, "u");
    check_ptr(b, "b");
    check_ptr(r, "r");
    if (r == u || r == b) throw Error{HT_ERR_ARG, "r must not alias u or b"};
    const Range R = full_range(h->m);
    const int64_t need = pass_partials(h, level, dtype, OP_RESID, R) + 256;
    if (need > kNoAllocScratch)
      throw Error{HT_ERR_ARG, "level too large for the allocation-free residual: its norm "
                              "partials need " + std::to_string(need) + " values, the "
                              "scratch holds " + std::to_string((long long)kNoAllocScratch)};
    double* p = noalloc_scratch();
    op_pass(h, level, dtype, OP_RESID, u, r, b, 0.0, (hipStream_t)stream,
            norm_dev != nullptr, 0, R, nullptr, p, norm_dev);
    return HT_OK;
  } catch (const Error& e) {
    set_error(e.code, e.msg);
    return e.code;
  } catch (...) {
    set_error(HT_ERR_ARG, "unknown error");
    return HT_ERR_ARG;
  }
}

int ht_smooth_jacobi(ht_mesh* h, int level, int dtype, double omega, int nsw,
                     void* u, const void* b, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(u, "u");
    check_ptr(b, "b");
    if (nsw < 0) throw Error{HT_ERR_ARG, "sweeps must be >= 0"};
    LevelWork& w = work(h, level, dtype);
    void* res = sweeps(h, level, dtype, omega, nsw, u, w.t, b, s);
    if (res != u) flat(h, level, dtype, dtype, FOP_COPY, u, res, s);
  });
}

int ht_restrict(ht_mesh* h, int fine_level, int dtype, const void* rf, void* rc,
                ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(fine_level, dtype);
    check_level(h->m, fine_level - 1);
    check_ptr(rf, "r_fine");
    check_ptr(rc, "r_coarse");
    restrict_pass(h, fine_level, dtype, rf, rc, s, full_range(h->m));
  });
}

int ht_prolongate_add(ht_mesh* h, int coarse_level, int dtype, const void* ec,
                      void* uf, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(coarse_level, dtype);
    check_level(h->m, coarse_level + 1);
    check_ptr(ec, "e_coarse");
    check_ptr(uf, "u_fine");
    prolong_pass(h, coarse_level, dtype, ec, uf, s, full_range(h->m));
  });
}

int ht_coarse_solve(ht_mesh* h, int level, int dtype, const void* b, void* u,
                    ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_ptr(b, "b");
    check_ptr(u, "u");
    // rhs = b - A u_B (u with its interior zeroed), then u_I = A_II^-1 rhs
    LevelWork& w = work(h, level, dtype);
    flat(h, level, dtype, dtype, FOP_COPY, w.u, u, s);
    ElemArgs a = elem_args(h, level);
    a.out = w.u;
    launch_elem(dtype, EOP_ZERO_INTERIOR, a, s);
    check_launch();
    op_pass(h, level, dtype, OP_RESID, w.u, w.t, b, 0.0, s);
    coarse_fast(h, level, dtype, w.t, u, s);
  });
}

int ht_vcycle(ht_mesh* h, int level, int dtype, const ht_cycle_opts* o, void* u,
              const void* b, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    check_cycle(h->m, level, o);
    check_ptr(u, "u");
    check_ptr(b, "b");
    if (level == o->coarse_level) {
      if (ht_coarse_solve(h, level, dtype, b, u, stream) != HT_OK)
        throw Error{HT_ERR_HIP, g_last_error};
      return;
    }
    prepare_smoother(h, level, dtype, *o, s);
    vcycle_top(h, level, dtype, *o, u, b, false, s);
  });
}

int ht_solve(ht_mesh* h, int level, const ht_solve_opts* o, void* u,
             const void* b, ht_solve_stats* st, ht_stream stream) {
  int rc = guard([&] {
    HT_DEV_PROLOGUE(level, HT_F64);
    if (!o || !st) throw Error{HT_ERR_ARG, "NULL options or stats"};
    check_cycle(h->m, level, &o->cyc);
    check_ptr(u, "u");
    check_ptr(b, "b");
    if (o->max_cycles < 0 || o->max_cycles > 256)
      throw Error{HT_ERR_ARG, "max_cycles must be in [0, 256]"};
    if (o->precision != HT_PREC_F64 && o->precision != HT_PREC_MIXED)
      throw Error{HT_ERR_ARG, "precision must be HT_PREC_F64 or HT_PREC_MIXED"};
    if (level == o->cyc.coarse_level && o->precision == HT_PREC_MIXED)
      throw Error{HT_ERR_ARG, "mixed precision needs level > coarse_level"};
    std::memset(st, 0, sizeof(*st));
    auto t0 = std::chrono::steady_clock::now();
    const double bnorm = norm_of(h, level, HT_F64, b, b, s, true);
    const double scale = bnorm > 0 ? 1.0 / bnorm : 1.0;
    LevelWork& w64 = work(h, level, HT_F64);
    const bool mixed = o->precision == HT_PREC_MIXED;
    LevelWork* w32 = mixed ? &work(h, level, HT_F32) : nullptr;
    // Fused refinement (Jacobi smoother): the FP64 residual pass, which
    // rounds the residual to FP32 as the next right-hand side, also writes
    // the next correction's first zero-guess sweep (into ffirst), so the
    // FP32 V-cycle starts after that sweep.  (Adding the correction to u
    // inside the same pass was measured slower: the stencil kernel loads
    // each row of u more than once, and every load would read e too.)
    const bool fused = mixed && o->cyc.smoother == HT_SMOOTH_JACOBI && o->cyc.nu1 > 0;
    void* ffirst = fused ? w32->t : nullptr;   // holds the first sweep
    void* fother = fused ? w32->u : nullptr;
    // the V-cycle started from a done first sweep in its t buffer ends in t
    // after an even number of further sweeps
    const bool e_in_t = ((o->cyc.nu1 - 1 + o->cyc.nu2) % 2) == 0;
    // the last sweep of each correction adds its result to u (no update pass)
    double* uadd = mixed && can_add_last_sweep(h, level, o->cyc) ? (double*)u : nullptr;
    // residual of the initial iterate (mixed: delivered in FP32 as the
    // right-hand side of the first correction)
    if (fused) {
      Fuse F;
      F.efirst = ffirst;
      op_pass(h, level, HT_F64, OP_RESID32X, u, w64.t, b, o->cyc.omega, s, true, 0,
              full_range(h->m), w32->b, nullptr, nullptr, &F);
    } else if (mixed) {
      op_pass(h, level, HT_F64, OP_RESID32, u, w64.t, b, 0.0, s, true, 0,
              full_range(h->m), w32->b);
    } else {
      op_pass(h, level, HT_F64, OP_RESID, u, w64.t, b, 0.0, s, true, 0);
    }
    double rel = read_scalar(h, 0, s) * scale;
    st->res_history[0] = rel;
    int k = 0;
    // FP64 cycles: the first Jacobi sweep of the next cycle (out of place,
    // u -> t) also yields |b - A u| of the iterate it starts from, so each
    // cycle's graph ends with that sweep instead of a separate residual
    // pass; when the norm meets the tolerance the sweep is discarded and u
    // is the result.
    const bool lag = !mixed && o->cyc.nu1 > 0 && level > o->cyc.coarse_level &&
                     o->cyc.smoother == HT_SMOOTH_JACOBI;
    auto first_sweep = [&](hipStream_t ss) {
      op_pass(h, level, HT_F64, OP_JACOBI, u, w64.t, b, o->cyc.omega, ss, true, 0);
      HT_CHECK_HIP(hipMemcpyAsync(h->m.h_scalar, h->m.d_scalar, sizeof(double),
                                  hipMemcpyDeviceToHost, ss));
    };
    auto step = [&](hipStream_t ss) {
      if (lag) {
        void* res = vcycle_impl(h, level, HT_F64, o->cyc, u, w64.t, b, false, ss, true);
        if (res != u) flat(h, level, HT_F64, HT_F64, FOP_COPY, u, res, ss);
        first_sweep(ss);
        return;
      }
      if (fused) {
        void* e = vcycle_impl(h, level, HT_F32, o->cyc, fother, ffirst, w32->b, false,
                              ss, true, uadd);
        if (e != (e_in_t ? ffirst : fother))
          throw Error{HT_ERR_STATE, "refinement: correction not in the expected buffer"};
        if (!uadd) flat(h, level, HT_F64, HT_F32, FOP_ADD, u, e, ss);
        Fuse F;
        F.efirst = e == w32->u ? w32->t : w32->u;
        op_pass(h, level, HT_F64, OP_RESID32X, u, w64.t, b, o->cyc.omega, ss, true, 0,
                full_range(h->m), w32->b, nullptr, nullptr, &F);
      } else if (!mixed) {
        vcycle_top(h, level, HT_F64, o->cyc, u, b, false, ss);
        op_pass(h, level, HT_F64, OP_RESID, u, w64.t, b, 0.0, ss, true, 0);
      } else {
        // FP32 correction of the FP64 residual (rounded to FP32 in w32->b),
        // FP64 update, FP64 residual of the new iterate rounded to FP32
        void* e = vcycle_impl(h, level, HT_F32, o->cyc, w32->u, w32->t, w32->b, true, ss,
                              false, uadd);
        if (!uadd) flat(h, level, HT_F64, HT_F32, FOP_ADD, u, e, ss);
        op_pass(h, level, HT_F64, OP_RESID32, u, w64.t, b, 0.0, ss, true, 0,
                full_range(h->m), w32->b);
      }
      HT_CHECK_HIP(hipMemcpyAsync(h->m.h_scalar, h->m.d_scalar, sizeof(double),
                                  hipMemcpyDeviceToHost, ss));
    };
    std::ostringstream key;
    key << "solve:" << level << ':' << o->precision << ':' << o->cyc.nu1 << ':'
        << o->cyc.nu2 << ':' << o->cyc.omega << ':' << o->cyc.coarse_level << ':'
        << o->cyc.smoother << ':' << o->cyc.degree << ':' << u << ':' << b;
    // all allocations and host setup happen before any capture
    coarse_solver(h, o->cyc.coarse_level);
    for (int l = o->cyc.coarse_level; l <= level; ++l) {
      work(h, l, HT_F64);
      if (mixed) work(h, l, HT_F32);
    }
    prepare_smoother(h, level, mixed ? HT_F32 : HT_F64, o->cyc, s);
    if (lag && rel > o->rel_tol && k < o->max_cycles && std::isfinite(rel)) {
      first_sweep(s);
      HT_CHECK_HIP(hipStreamSynchronize(s));
    }
    // stagnation: three cycles in a row without a new minimum of the residual
    double best = rel;
    int kbest = 0;
    bool stagnated = false;
    while (rel > o->rel_tol && k < o->max_cycles && std::isfinite(rel)) {
      if (!fused) {
        if (o->use_graph) run_graph(h, key.str(), step, s);
        else step(s);
      } else {
        // the FP32 buffers' roles may alternate: one graph per assignment
        std::ostringstream fk;
        fk << key.str() << ':' << ffirst;
        if (o->use_graph) run_graph(h, fk.str(), step, s);
        else step(s);
        void* e = e_in_t ? ffirst : fother;
        ffirst = e == w32->u ? w32->t : w32->u;
        fother = e;
      }
      HT_CHECK_HIP(hipStreamSynchronize(s));
      rel = h->m.h_scalar[0] * scale;
      ++k;
      st->res_history[k] = rel;
      if (rel < best) {
        best = rel;
        kbest = k;
      } else if (rel > o->rel_tol && k - kbest >= 3) {
        stagnated = true;
        break;
      }
    }
    st->cycles = k;
    st->rel_res = rel;
    st->converged = rel <= o->rel_tol;
    st->stagnated = stagnated;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!st->converged)
      throw Error{HT_ERR_NOT_CONVERGED,
                  std::string(stagnated ? "stagnated: " : "") + "relative residual " +
                      std::to_string(rel) + " after " + std::to_string(k) + " cycles"};
  });
  return rc;
}

int ht_lambda_max(ht_mesh* h, int level, double* lambda, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, HT_F64);
    if (!lambda) throw Error{HT_ERR_ARG, "lambda is NULL"};
    *lambda = lambda_max_of(h, level, s);
  });
}

int ht_set_lambda_max(ht_mesh* h, int level, double lambda) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    if (!(lambda > 0.0) || !std::isfinite(lambda))
      throw Error{HT_ERR_ARG, "lambda must be positive and finite"};
    // captured cycles hold the Chebyshev coefficients of the old value
    if (h->m.uploaded) (void)hipDeviceSynchronize();
    for (auto& kv : h->m.graphs) (void)hipGraphExecDestroy(kv.second.exec);
    h->m.graphs.clear();
    h->lambda_max[level] = lambda;
  });
}

int ht_fmg(ht_mesh* h, int level, const ht_cycle_opts* o, int cycles, void* u,
           const void* b, double* rel_res, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, HT_F64);
    check_cycle(h->m, level, o);
    check_ptr(u, "u");
    check_ptr(b, "b");
    if (cycles < 1 || cycles > 64) throw Error{HT_ERR_ARG, "cycles must be in [1, 64]"};
    const int lc = o->coarse_level;
    // set-up before capture: workspace and the coarse solver
    coarse_solver(h, lc);
    for (int l = lc; l <= level; ++l) work(h, l, HT_F64);
    prepare_smoother(h, level, HT_F64, *o, s);
    auto body = [&](hipStream_t ss) {
      const Range R = full_range(h->m);
      // right-hand sides of the coarser levels: b_{l-1} = R b_l
      const void* bl = b;
      for (int l = level; l > lc; --l) {
        restrict_pass(h, l, HT_F64, bl, work(h, l - 1, HT_F64).b, ss, R);
        bl = work(h, l - 1, HT_F64).b;
      }
      if (level == lc) {
        flat(h, lc, HT_F64, HT_F64, FOP_ZERO, u, nullptr, ss);
        coarse_fast(h, lc, HT_F64, b, u, ss);
        return;
      }
      LevelWork& w0 = work(h, lc, HT_F64);
      flat(h, lc, HT_F64, HT_F64, FOP_ZERO, w0.u, nullptr, ss);
      coarse_fast(h, lc, HT_F64, w0.b, w0.u, ss);
      // upwards: interpolate, then V-cycles on each level
      for (int l = lc + 1; l <= level; ++l) {
        LevelWork& wl = work(h, l, HT_F64);
        void* ul = l == level ? u : wl.u;
        const void* rl = l == level ? b : wl.b;
        flat(h, l, HT_F64, HT_F64, FOP_ZERO, ul, nullptr, ss);
        prolong_pass(h, l - 1, HT_F64, work(h, l - 1, HT_F64).u, ul, ss, R);
        for (int c = 0; c < cycles; ++c) vcycle_top(h, l, HT_F64, *o, ul, rl, false, ss);
      }
    };
    std::ostringstream key;
    key << "fmg:" << level << ':' << o->nu1 << ':' << o->nu2 << ':' << o->omega << ':'
        << lc << ':' << o->smoother << ':' << o->degree << ':' << cycles << ':' << u
        << ':' << b;
    run_graph(h, key.str(), body, s);
    if (rel_res) {
      const double bn = norm_of(h, level, HT_F64, b, b, s, true);
      op_pass(h, level, HT_F64, OP_RESID, u, work(h, level, HT_F64).t, b, 0.0, s, true, 0);
      const double rn = read_scalar(h, 0, s);
      *rel_res = bn > 0 ? rn / bn : rn;
    }
  });
}

int ht_batch_create(ht_mesh* const* meshes, const int* levels, int n,
                    ht_batch** out) {
  return guard([&] {
    if (!out || !meshes || !levels || n < 1)
      throw Error{HT_ERR_ARG, "need n >= 1 meshes, levels and out"};
    *out = nullptr;
    for (int p = 0; p < n; ++p) {
      if (!meshes[p]) throw Error{HT_ERR_ARG, "mesh " + std::to_string(p) + " is NULL"};
      check_level(meshes[p]->m, levels[p]);
    }
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return levels[a] > levels[b]; });
    std::vector<double> xyz;
    std::vector<int64_t> cells, cell_begin{0};
    std::vector<int> fin;
    int lo = 10;
    for (int q : order) {
      const Mesh& src = meshes[q]->m;
      const int64_t voff = (int64_t)xyz.size() / 3;
      xyz.insert(xyz.end(), src.xyz.begin(), src.xyz.end());
      for (const Cell& c : src.cells)
        for (int k = 0; k < 4; ++k) cells.push_back(c.gv[k] + voff);
      cell_begin.push_back(cell_begin.back() + src.nc);
      fin.push_back(levels[q]);
      lo = std::min(lo, src.min_level);
    }
    auto B = std::make_unique<ht_batch>();
    B->mesh = new ht_mesh();
    Mesh& m = B->mesh->m;
    build_mesh(m, xyz.data(), (int64_t)xyz.size() / 3, cells.data(),
               (int64_t)cells.size() / 4, lo, fin.front());
    set_problems(m, cell_begin, fin);
    Batch& bt = B->bt;
    bt.nprob = n;
    bt.order = order;
    bt.level = fin;
    bt.lmax = fin.front();
    bt.lmin = fin.back();
    bt.pd0.assign(bt.lmax + 2, 0);
    bt.pd1.assign(bt.lmax + 2, 0);
    for (int l = 0; l <= bt.lmax + 1; ++l) {
      int a = 0, b = 0;
      while (a < n && fin[a] > l) ++a;
      while (b < n && fin[b] >= l) ++b;
      bt.pd0[l] = a;
      bt.pd1[l] = b;
    }
    for (int p = 0; p < n; ++p) {
      ht_level_info li;
      if (ht_mesh_query(meshes[order[p]], fin[p], &li) != HT_OK)
        throw Error{HT_ERR_ARG, g_last_error};
      bt.ndofs.push_back(li.n_dofs);
    }
    *out = B.release();
  });
}

int ht_batch_destroy(ht_batch* B) {
  return guard([&] {
    if (!B) return;
    Batch& bt = B->bt;
    if (bt.d_part) {
      (void)hipDeviceSynchronize();
      (void)hipFree(bt.d_part); (void)hipFree(bt.d_lo); (void)hipFree(bt.d_hi);
      (void)hipFree(bt.d_norm2); (void)hipHostFree(bt.h_norm2);
    }
    ht_mesh_destroy(B->mesh);
    delete B;
  });
}

static void autotune_level(ht_mesh* h, int level, int dtype, const char* cache_path,
                           int* rows, hipStream_t s);
static void drop_graphs(ht_mesh* h);

int ht_batch_mesh(ht_batch* B, ht_mesh** mesh) {
  return guard([&] {
    if (!B || !mesh) throw Error{HT_ERR_ARG, "NULL argument"};
    *mesh = B->mesh;
  });
}

int ht_batch_autotune(ht_batch* B, const char* cache_path, ht_stream stream) {
  return guard([&] {
    if (!B) throw Error{HT_ERR_ARG, "batch is NULL"};
    ht_mesh* h = B->mesh;
    ensure_uploaded_h(h);
    hipStream_t s = (hipStream_t)stream;
    for (int l = h->m.min_level; l <= B->bt.lmax; ++l)
      for (int dt : {HT_F64, HT_F32}) autotune_level(h, l, dt, cache_path, nullptr, s);
    drop_graphs(h);
  });
}

int ht_batch_query(const ht_batch* B, int* n_problems, int64_t* n_dofs,
                   int64_t* n_cells) {
  return guard([&] {
    if (!B) throw Error{HT_ERR_ARG, "batch is NULL"};
    if (n_problems) *n_problems = B->bt.nprob;
    if (n_dofs) {
      int64_t t = 0;
      for (int64_t d : B->bt.ndofs) t += d;
      *n_dofs = t;
    }
    if (n_cells) *n_cells = B->mesh->m.nc;
  });
}

int ht_batch_solve(ht_batch* B, const ht_solve_opts* o, void* const* u,
                   const void* const* b, ht_solve_stats* st, ht_stream stream) {
  return guard([&] {
    if (!B || !o || !u || !b || !st) throw Error{HT_ERR_ARG, "NULL argument"};
    ht_mesh* h = B->mesh;
    Mesh& m = h->m;
    Batch& bt = B->bt;
    const int P = bt.nprob;
    if (o->precision != HT_PREC_F64 && o->precision != HT_PREC_MIXED)
      throw Error{HT_ERR_ARG, "precision must be HT_PREC_F64 or HT_PREC_MIXED"};
    const bool mixed = o->precision == HT_PREC_MIXED;
    if (o->cyc.smoother != HT_SMOOTH_JACOBI)
      throw Error{HT_ERR_ARG, "batch solves use the Jacobi smoother"};
    if (o->max_cycles < 0 || o->max_cycles > 256)
      throw Error{HT_ERR_ARG, "max_cycles must be in [0, 256]"};
    check_cycle(m, bt.lmax, &o->cyc);
    if (o->cyc.coarse_level > bt.lmin)
      throw Error{HT_ERR_LEVEL, "coarse_level above the finest level of a problem"};
    for (int q = 0; q < P; ++q) {
      check_ptr(u[q], "u[p]");
      check_ptr(b[q], "b[p]");
    }
    ensure_uploaded_h(h);
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    // set-up before any capture: workspace, coarse solver, norm tables
    coarse_solver(h, o->cyc.coarse_level);
    for (int l = o->cyc.coarse_level; l <= bt.lmax; ++l) {
      work(h, l, HT_F64);
      if (mixed) work(h, l, HT_F32);
    }
    if (!bt.d_part) {
      bt.part_off.assign(bt.lmax + 1, 0);
      int64_t off = 0;
      std::vector<int64_t> lo(P), hi(P);
      for (int l = bt.lmax; l >= bt.lmin; --l) {
        bt.part_off[l] = off;
        if (bt.pd1[l] <= bt.pd0[l]) continue;
        const int64_t nw = h->walk_tiles.at(l).second;
        const int64_t cbase = m.pcell[bt.pd0[l]];
        for (int p = bt.pd0[l]; p < bt.pd1[l]; ++p) {
          lo[p] = off + (m.pcell[p] - cbase) * nw;
          hi[p] = off + (m.pcell[p + 1] - cbase) * nw;
        }
        off += (m.pcell[bt.pd1[l]] - cbase) * nw;
      }
      bt.part_size = off;
      bt.d_part = dalloc<double>(std::max<int64_t>(off, 1));
      bt.d_lo = upload(lo);
      bt.d_hi = upload(hi);
      bt.d_norm2 = dalloc<double>(P);
      HT_CHECK_HIP(hipHostMalloc((void**)&bt.h_norm2, P * sizeof(double),
                                 hipHostMallocDefault));
    }
    // a problem's vector is the run of slots of its cells on its finest level
    auto seg = [&](int p, void* v) {
      return at_cell(v, m.pcell[p], bt.level[p], HT_F64);
    };
    auto seg_bytes = [&](int p) {
      return (size_t)((m.pcell[p + 1] - m.pcell[p]) * make_layout(bt.level[p]).stride * 8);
    };
    for (int p = 0; p < P; ++p) {
      LevelWork& w = work(h, bt.level[p], HT_F64);
      HT_CHECK_HIP(hipMemcpyAsync(seg(p, w.u), u[bt.order[p]], seg_bytes(p),
                                  hipMemcpyDeviceToDevice, s));
      HT_CHECK_HIP(hipMemcpyAsync(seg(p, w.b), b[bt.order[p]], seg_bytes(p),
                                  hipMemcpyDeviceToDevice, s));
    }
    batch_norms(h, bt, 1, s);
    HT_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<double> scale(P);
    for (int p = 0; p < P; ++p) {
      const double bn = std::sqrt(bt.h_norm2[p]);
      scale[p] = bn > 0 ? 1.0 / bn : 1.0;
    }
    // mixed: each problem's FP64 residual (left in work(l).t by the norms
    // at its finest level l) rounded to FP32, the right-hand side of the
    // next correction cycle
    auto residuals_to_f32 = [&](hipStream_t ss) {
      for (int l = bt.lmax; l >= bt.lmin; --l) {
        if (bt.pd1[l] <= bt.pd0[l]) continue;
        flat_range(h, l, HT_F32, HT_F64, FOP_COPY, work(h, l, HT_F32).b,
                   work(h, l, HT_F64).t, ss, problem_range(m, bt.pd0[l], bt.pd1[l]));
      }
    };
    batch_norms(h, bt, 0, s);
    if (mixed) residuals_to_f32(s);
    HT_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<ht_solve_stats> ps(P);
    for (auto& x : ps) std::memset(&x, 0, sizeof(x));
    std::vector<char> done(P, 0);
    int open = P;
    auto copy_out = [&](int p) {
      LevelWork& w = work(h, bt.level[p], HT_F64);
      HT_CHECK_HIP(hipMemcpyAsync(u[bt.order[p]], seg(p, w.u), seg_bytes(p),
                                  hipMemcpyDeviceToDevice, s));
    };
    // a problem is frozen (copied out) at the first cycle that meets rel_tol
    // ... or at the third cycle in a row without a new minimum of its
    // residual (stagnation, as in ht_solve)
    std::vector<double> best(P, HUGE_VAL);
    std::vector<int> kbest(P, 0);
    auto record = [&](int k) {
      for (int p = 0; p < P; ++p) {
        if (done[p]) continue;
        const double rel = std::sqrt(bt.h_norm2[p]) * scale[p];
        ps[p].res_history[k] = rel;
        ps[p].cycles = k;
        ps[p].rel_res = rel;
        bool stop = rel <= o->rel_tol || !std::isfinite(rel);
        if (rel < best[p]) {
          best[p] = rel;
          kbest[p] = k;
        } else if (!stop && k - kbest[p] >= 3) {
          ps[p].stagnated = 1;
          stop = true;
        }
        if (stop) {
          ps[p].converged = rel <= o->rel_tol;
          done[p] = 1;
          --open;
          copy_out(p);
        }
      }
    };
    record(0);
    std::ostringstream key;
    key << "batch:" << o->precision << ':' << o->cyc.nu1 << ':' << o->cyc.nu2
        << ':' << o->cyc.omega << ':' << o->cyc.coarse_level;
    auto step = [&](hipStream_t ss) {
      if (!mixed) {
        batch_level(h, bt, bt.lmax, o->cyc, HT_F64, false, ss);
        batch_norms(h, bt, 0, ss);
        return;
      }
      // FP32 correction cycle, FP64 update u += c at every problem's finest
      // level, FP64 residuals and norms, residuals rounded to FP32
      batch_level(h, bt, bt.lmax, o->cyc, HT_F32, true, ss);
      for (int l = bt.lmax; l >= bt.lmin; --l) {
        if (bt.pd1[l] <= bt.pd0[l]) continue;
        flat_range(h, l, HT_F64, HT_F32, FOP_ADD, work(h, l, HT_F64).u,
                   work(h, l, HT_F32).u, ss, problem_range(m, bt.pd0[l], bt.pd1[l]));
      }
      batch_norms(h, bt, 0, ss);
      residuals_to_f32(ss);
    };
    int k = 0;
    while (open > 0 && k < o->max_cycles) {
      if (o->use_graph) run_graph(h, key.str(), step, s);
      else step(s);
      HT_CHECK_HIP(hipStreamSynchronize(s));
      ++k;
      record(k);
    }
    for (int p = 0; p < P; ++p)
      if (!done[p]) copy_out(p);
    HT_CHECK_HIP(hipStreamSynchronize(s));
    const double sec =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int failed = 0;
    for (int p = 0; p < P; ++p) {
      ps[p].seconds = sec;
      failed += !ps[p].converged;
      st[bt.order[p]] = ps[p];
    }
    if (failed)
      throw Error{HT_ERR_NOT_CONVERGED, std::to_string(failed) + " of " +
                                            std::to_string(P) + " problems did not converge"};
  });
}

int ht_set_tile_rows(ht_mesh* h, int level, int dtype, int rows) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_dtype(dtype);
    if (rows != 4 && rows != 8 && rows != 16 && !(rows == 0 && has_band(h, level, dtype)))
      throw Error{HT_ERR_ARG, "tile rows must be 4, 8 or 16, or 0 (band kernel) where "
                              "its LDS image fits the level"};
    h->tuned_J[{level, dtype}] = rows;
  });
}

int ht_get_tile_rows(const ht_mesh* h, int level, int dtype, int* rows) {
  return guard([&] {
    if (!h || !rows) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    check_dtype(dtype);
    *rows = choose_J(const_cast<ht_mesh*>(h), level, dtype);
  });
}

int ht_set_sweep_shape(ht_mesh* h, int level, int dtype, int rows, int waves_in_i) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_dtype(dtype);
    if (rows != 4 && rows != 8 && rows != 16 && !(rows == 0 && has_band(h, level, dtype)))
      throw Error{HT_ERR_ARG, "tile rows must be 4, 8 or 16 (or 0 where a band fits)"};
    if (waves_in_i != 0 && waves_in_i != 1)
      throw Error{HT_ERR_ARG, "waves_in_i must be 0 or 1"};
    auto it = h->tuned_sweep.find({level, dtype});
    const int seg = it != h->tuned_sweep.end() ? it->second.seg : march_segment(waves_in_i != 0);
    if (h->m.uploaded && rows > 0) seg_tiles(h, level, rows, waves_in_i != 0, seg);
    h->tuned_sweep[{level, dtype}] = {rows, waves_in_i != 0, seg};
  });
}

int ht_get_sweep_shape(const ht_mesh* h, int level, int dtype, int* rows,
                       int* waves_in_i) {
  return guard([&] {
    if (!h || !rows || !waves_in_i) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    check_dtype(dtype);
    const Shape sh = choose_shape(const_cast<ht_mesh*>(h), level, dtype, OP_JACOBI);
    *rows = sh.J;
    *waves_in_i = sh.in_i ? 1 : 0;
  });
}

int ht_set_march_segment(ht_mesh* h, int level, int dtype, int planes) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    check_level(h->m, level);
    check_dtype(dtype);
    if (std::find(std::begin(kSegs), std::end(kSegs), planes) == std::end(kSegs))
      throw Error{HT_ERR_ARG, "march segment must be 32, 64 or 128 planes"};
    const Shape sh = choose_shape(h, level, dtype, OP_JACOBI);
    if (h->m.uploaded && sh.J > 0) seg_tiles(h, level, sh.J, sh.in_i, planes);
    h->tuned_sweep[{level, dtype}] = {sh.J, sh.in_i, planes};
  });
}

int ht_get_march_segment(const ht_mesh* h, int level, int dtype, int* planes) {
  return guard([&] {
    if (!h || !planes) throw Error{HT_ERR_ARG, "NULL argument"};
    check_level(h->m, level);
    check_dtype(dtype);
    *planes = choose_shape(const_cast<ht_mesh*>(h), level, dtype, OP_JACOBI).seg;
  });
}

// The cells (and their faces, edges, vertices) present on `level`: all of
// a plain mesh, the problems whose finest level is at least `level` in the
// union mesh of a batch (a prefix of its problems).
static Range level_range(const Mesh& m, int level) {
  int p1 = 0;
  while (p1 < m.nprob && m.pcell[p1 + 1] <= m.act_cells[level]) ++p1;
  return problem_range(m, 0, p1);
}

// Autotuning of one (level, dtype) over the cells present on the level.
static void autotune_level(ht_mesh* h, int level, int dtype, const char* cache_path,
                           int* rows, hipStream_t s) {
  if (!cache_path) {
    const char* env = std::getenv("HT_TUNE_CACHE");
    if (env && *env) cache_path = env;
  }
  // cache: lines "<gfx arch> <level> <dtype> <cells> <stride> v3
  // <apply rows> <sweep rows> <sweep waves in i> <sweep segment>"
  hipDeviceProp_t prop;
  HT_CHECK_HIP(hipGetDeviceProperties(&prop, h->m.device));
  const CellLayout L = make_layout(level);
  const Range R = level_range(h->m, level);
  if (R.c1 <= R.c0) return;  // no cell on this level
  std::ostringstream key;
  key << prop.gcnArchName << ' ' << level << ' ' << dtype << ' ' << (R.c1 - R.c0) << ' '
      << L.stride << " v3";
  auto valid_rows = [](int J) { return J == 4 || J == 8 || J == 16; };
  auto valid_apply = [&](int J) { return valid_rows(J) || (J == 0 && has_band(h, level, dtype)); };
  auto valid_seg = [](int g) { return std::find(std::begin(kSegs), std::end(kSegs), g) != std::end(kSegs); };
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (std::fgets(line, sizeof line, f)) {
        const std::string ln(line), k = key.str() + ' ';
        int J = 0, sJ = 0, sI = -1, sg = 0;
        if (ln.compare(0, k.size(), k) == 0 &&
            std::sscanf(ln.c_str() + k.size(), "%d %d %d %d", &J, &sJ, &sI, &sg) == 4 &&
            valid_apply(J) && valid_apply(sJ) && (sI == 0 || sI == 1) && valid_seg(sg)) {
          if (sJ > 0) seg_tiles(h, level, sJ, sI == 1, sg);
          h->tuned_J[{level, dtype}] = J;
          h->tuned_sweep[{level, dtype}] = {sJ, sI == 1, sg};
          if (rows) *rows = J;
          std::fclose(f);
          return;
        }
      }
      std::fclose(f);
    }
  }
  const size_t bytes = level_slots(h->m, level) * esize(dtype);
  void* x = dalloc<char>(bytes);
  void* y = nullptr;
  void* bv = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool was_profiling = h->m.profiling;
  int best = choose_J(h, level, dtype);
  SweepShape best_sweep{kDefaultJ, true, march_segment(true)};
  auto release = [&] {
    h->m.profiling = was_profiling;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(x); (void)hipFree(y); (void)hipFree(bv);
  };
  try {
    y = dalloc<char>(bytes);
    bv = dalloc<char>(bytes);
    HT_CHECK_HIP(hipEventCreate(&e0));
    HT_CHECK_HIP(hipEventCreate(&e1));
    h->m.profiling = false;
    // mean time of five launches of `pass` after two untimed ones
    auto time_of = [&](const std::function<void()>& pass) {
      for (int rep = 0; rep < 2; ++rep) pass();
      HT_CHECK_HIP(hipEventRecord(e0, s));
      for (int rep = 0; rep < 5; ++rep) pass();
      HT_CHECK_HIP(hipEventRecord(e1, s));
      HT_CHECK_HIP(hipEventSynchronize(e1));
      float ms = 0;
      HT_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    // Every candidate is timed in two rounds and keeps its faster time, so
    // that a clock ramp or a noisy first launch does not decide the choice.
    HT_CHECK_HIP(hipMemsetAsync(x, 0, bytes, s));
    HT_CHECK_HIP(hipMemsetAsync(y, 0, bytes, s));
    HT_CHECK_HIP(hipMemsetAsync(bv, 0, bytes, s));
    const int kRounds = 2;
    // apply: the band kernel, or the tile kernel with J rows per wave and
    // the waves stacked in j
    std::vector<int> cand(std::begin(kJ), std::end(kJ));
    if (has_band(h, level, dtype)) cand.insert(cand.begin(), 0);
    std::vector<float> ms_apply(cand.size(), 1e30f);
    for (int round = 0; round < kRounds; ++round)
      for (size_t c = 0; c < cand.size(); ++c) {
        h->tuned_J[{level, dtype}] = cand[c];
        const float ms = time_of([&] { op_pass(h, level, dtype, OP_APPLY, x, y, nullptr, 0.0, s, false, 0, R); });
        ms_apply[c] = std::min(ms_apply[c], ms);
      }
    best = cand[std::min_element(ms_apply.begin(), ms_apply.end()) - ms_apply.begin()];
    h->tuned_J[{level, dtype}] = best;
    // sweeps: the band kernel, or the tile kernel's rows per wave, wave
    // arrangement and march segment length, on the Jacobi sweep with its
    // own right-hand side (b streams from HBM as in a solve)
    std::vector<SweepShape> scand;
    if (has_band(h, level, dtype)) {
      const bool in_i = (1 << level) >= 62 * (kCellWaves - 1) + 1;
      scand.push_back({0, in_i, march_segment(in_i)});
    }
    for (int J : kJ)
      for (bool in_i : {false, true})
        for (int sg : kSegs) {
          seg_tiles(h, level, J, in_i, sg);
          scand.push_back({J, in_i, sg});
        }
    std::vector<float> ms_sweep(scand.size(), 1e30f);
    for (int round = 0; round < kRounds; ++round)
      for (size_t c = 0; c < scand.size(); ++c) {
        h->tuned_sweep[{level, dtype}] = scand[c];
        const float ms = time_of(
            [&] { op_pass(h, level, dtype, OP_JACOBI, x, y, bv, 2.0 / 3.0, s, false, 0, R); });
        ms_sweep[c] = std::min(ms_sweep[c], ms);
      }
    best_sweep = scand[std::min_element(ms_sweep.begin(), ms_sweep.end()) - ms_sweep.begin()];
  } catch (...) {
    h->tuned_sweep.erase({level, dtype});
    release();
    throw;
  }
  release();
  h->tuned_J[{level, dtype}] = best;
  h->tuned_sweep[{level, dtype}] = best_sweep;
  if (rows) *rows = best;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %d %d %d\n", key.str().c_str(), best, best_sweep.J,
                   best_sweep.in_i ? 1 : 0, best_sweep.seg);
      std::fclose(f);
    }
  }
}

// captured graphs hold the launch shapes of their capture
static void drop_graphs(ht_mesh* h) {
  if (h->m.uploaded) (void)hipDeviceSynchronize();
  for (auto& kv : h->m.graphs) (void)hipGraphExecDestroy(kv.second.exec);
  h->m.graphs.clear();
}

int ht_autotune(ht_mesh* h, int level, int dtype, const char* cache_path,
                int* rows, ht_stream stream) {
  return guard([&] {
    HT_DEV_PROLOGUE(level, dtype);
    autotune_level(h, level, dtype, cache_path, rows, s);
    drop_graphs(h);
  });
}

int ht_profile_enable(ht_mesh* h, int enable) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    h->m.profiling = enable != 0;
  });
}

int ht_profile_reset(ht_mesh* h) {
  return guard([&] {
    if (!h) throw Error{HT_ERR_ARG, "mesh is NULL"};
    (void)hipDeviceSynchronize();
    for (auto& e : h->m.prof) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    h->m.prof.clear();
  });
}

int ht_profile_query(ht_mesh* h, const char* prefix, double* ms, int64_t* launches) {
  return guard([&] {
    if (!h || !prefix || !ms || !launches) throw Error{HT_ERR_ARG, "NULL argument"};
    double tot = 0;
    int64_t cnt = 0;
    const size_t pl = std::strlen(prefix);
    for (auto& e : h->m.prof) {
      if (e.name.compare(0, pl, prefix) != 0) continue;
      HT_CHECK_HIP(hipEventSynchronize(e.b));
      float t = 0;
      HT_CHECK_HIP(hipEventElapsedTime(&t, e.a, e.b));
      tot += t;
      ++cnt;
    }
    *ms = tot;
    *launches = cnt;
  });
}

int ht_selftest_lane_shift(int* mismatches) {
  return guard([&] {
    if (!mismatches) throw Error{HT_ERR_ARG, "NULL argument"};
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
      (void)hipGetLastError();
      throw Error{HT_ERR_STATE, "no HIP device available"};
    }
    int* d = dalloc<int>(128);
    launch_lane_selftest(d, 0);
    check_launch();
    int hbuf[128];
    HT_CHECK_HIP(hipMemcpy(hbuf, d, sizeof(hbuf), hipMemcpyDeviceToHost));
    (void)hipFree(d);
    int bad = 0;
    for (int l = 0; l < 64; ++l) {
      const int prev = l == 0 ? 0 : l;         // value of lane l-1 is l
      const int next = l == 63 ? 0 : l + 2;    // value of lane l+1 is l+2
      bad += hbuf[l] != prev;
      bad += hbuf[64 + l] != next;
    }
    *mismatches = bad;
  });
}

}  // extern "C"
