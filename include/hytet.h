/* hytet -- matrix-free P1 finite elements on regularly refined macro-tetrahedra,
 * for AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The library implements the hot path of Kohl, Bauer, Boehm, Ruede,
 * "Fundamental data structures for matrix-free finite elements on hybrid
 * tetrahedral grids" (arXiv:2308.01792):
 *   - a coarse tetrahedral mesh is turned into a graph of macro-primitives
 *     (cells, faces, edges, vertices; Section 2),
 *   - every macro-cell is refined regularly with the rule of eq. (bey)
 *     (Section 3.1); micro-vertices are addressed by index functions over
 *     tetrahedral polytopes (Section 4),
 *   - the P1 Laplacian a_ij = sum_T int_T grad phi_i . grad phi_j
 *     (Section 5.2.1) is applied matrix-free as a 15-point stencil whose
 *     weights are precomputed once per macro-cell from its geometry,
 *     independent of the level (Section 5.2.3, constant coefficients),
 *   - vectors live on a range of levels and every call names its level
 *     (Section 5.1), which makes geometric multigrid (weighted Jacobi,
 *     restriction, prolongation, V-cycle, iterative refinement) direct.
 *
 * Conventions
 *   Vectors.  A level-l vector is a caller-owned device array of n_slots
 *     elements (ht_mesh_query) of type double (HT_F64) or float (HT_F32),
 *     256-byte aligned.  Slot s holds one copy of one micro-vertex value.
 *     Micro-vertices shared by several macro-cells (on macro-faces, -edges,
 *     -vertices) have one copy per incident cell; exactly one copy is the
 *     owner.  A vector is *consistent* when all copies of every micro-vertex
 *     are equal; inputs must be consistent (ht_sync makes them so) and every
 *     output is consistent.  Padding slots (flag HT_SLOT_PAD) are never read
 *     nor written.
 *   Boundary.  Micro-vertices on macro-faces with a single incident cell are
 *     Dirichlet vertices.  Their input values are boundary data; outputs of
 *     apply/residual/restrict hold 0 there, smoothers and solvers leave them
 *     unchanged.
 *   Keys.  A micro-vertex is identified, independently of the layout, by its
 *     key: the (global macro-vertex id, integer barycentric weight) pairs with
 *     non-zero weight, ascending by id, padded with (-1, 0) to four pairs;
 *     weights sum to 2^level.  Two slots hold the same micro-vertex iff their
 *     keys are equal.
 *   Streams.  ht_stream is a hipStream_t (0 = null stream).  Device calls are
 *     asynchronous on it unless stated otherwise.
 *   Errors.  Every call returns an HT_* status; ht_last_error() describes the
 *     last failure of the calling thread.  Nothing throws or aborts across
 *     the ABI.  A mesh is not thread-safe.
 */
#ifndef HYTET_H
#define HYTET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ht_mesh ht_mesh;
typedef struct ht_batch ht_batch;
typedef void* ht_stream; /* hipStream_t */

enum {
  HT_OK = 0,
  HT_ERR_ARG = 1,            /* null/misaligned pointer, bad option value */
  HT_ERR_MESH = 2,           /* degenerate, duplicated or non-conforming */
  HT_ERR_LEVEL = 3,          /* level outside the mesh's level range */
  HT_ERR_OOM = 4,            /* device allocation failed */
  HT_ERR_HIP = 5,            /* a HIP runtime call failed */
  HT_ERR_NOT_CONVERGED = 6,  /* solver hit max_cycles or diverged */
  HT_ERR_STATE = 7           /* no GPU / call not valid in this state */
};
enum { HT_F64 = 0, HT_F32 = 1 };
enum { HT_PREC_F64 = 0, HT_PREC_MIXED = 1 };
enum { HT_SMOOTH_JACOBI = 0, HT_SMOOTH_CHEBYSHEV = 1 };
enum {
  HT_SLOT_OWNER = 1,     /* the owning copy of its micro-vertex */
  HT_SLOT_GHOST = 2,     /* a further copy of a shared micro-vertex */
  HT_SLOT_DIRICHLET = 4, /* micro-vertex on the domain boundary */
  HT_SLOT_PAD = 8        /* padding, holds no micro-vertex */
};

typedef struct {
  int64_t n_slots;     /* vector length at this level */
  int64_t n_dofs;      /* unique non-Dirichlet micro-vertices (unknowns) */
  int64_t n_unique;    /* unique micro-vertices, boundary included */
  int64_t n_cells, n_faces, n_edges, n_vertices; /* macro-primitives */
  int64_t cell_stride; /* slots per macro-cell block */
} ht_level_info;

typedef struct {
  int nu1, nu2;        /* pre- and post-smoother applications */
  double omega;        /* Jacobi weight, e.g. 2/3 */
  int coarse_level;    /* level solved exactly (dense Cholesky inverse) */
  int smoother;        /* HT_SMOOTH_JACOBI (0) or HT_SMOOTH_CHEBYSHEV */
  int degree;          /* Chebyshev: polynomial degree (stencil passes per
                          application), 1..16; ignored for Jacobi */
} ht_cycle_opts;

typedef struct {
  ht_cycle_opts cyc;
  int precision;       /* HT_PREC_F64 or HT_PREC_MIXED */
  double rel_tol;      /* stop when ||b - A u||_2 <= rel_tol ||b||_2 */
  int max_cycles;      /* <= 256 */
  int use_graph;       /* replay each cycle as a captured hipGraph */
} ht_solve_opts;

typedef struct {
  int cycles;          /* V-cycles (or refinement steps) performed */
  int converged;
  double rel_res;      /* final relative residual (FP64) */
  double seconds;      /* wall time of the solve */
  double res_history[257]; /* relative residual before cycle 0, 1, ... */
  int stagnated;       /* 1: stopped because three cycles in a row brought no
                          new minimum of the residual (rounding floor of the
                          precision reached above rel_tol, or a cycle that
                          does not contract); converged is 0 then */
} ht_solve_stats;

/* ------------------------------------------------------------ general -- */
const char* ht_last_error(void);
int ht_version(void);
/* t_w(i,j,k) of the paper's linearisation of I_tet(w) (Section 4). */
int64_t ht_index_tw(int64_t w, int64_t i, int64_t j, int64_t k);

/* --------------------------------------------------------------- mesh -- */
/* Build the macro-primitive graph (Section 2) of a conforming tetrahedral
 * mesh and the per-cell stencils of every level in [min_level, max_level].
 * xyz: host [nv][3] doubles; cells: host [nc][4] global vertex ids.  The
 * local vertex order of each cell is kept: it selects the inner diagonal of
 * the regular refinement (Section 3.1).  Both arrays are copied.  Host-only:
 * device memory is allocated on the first device call.
 * HT_ERR_MESH for a degenerate cell, repeated vertex, a face shared by more
 * than two cells or an out-of-range id; HT_ERR_LEVEL if the levels are not
 * 0 <= min_level <= max_level <= 10. */
int ht_mesh_create(const double* xyz, int64_t nv, const int64_t* cells,
                   int64_t nc, int min_level, int max_level, ht_mesh** out);
int ht_mesh_destroy(ht_mesh* mesh);
int ht_mesh_query(const ht_mesh* mesh, int level, ht_level_info* info);

/* Keys (int64[count][8]) and/or flags (HT_SLOT_*) of slots
 * [first, first + count) at a level; either output may be NULL.  Host. */
int ht_vertex_keys(const ht_mesh* mesh, int level, int64_t first,
                   int64_t count, int64_t* keys, uint8_t* flags);
/* Coordinates (double[count][3]) of slots [first, first+count).  Host.
 * A micro-vertex with key pairs (g_m, w_m) sits at sum_m w_m X_{g_m} / 2^l. */
int ht_vertex_coords(const ht_mesh* mesh, int level, int64_t first,
                     int64_t count, double* xyz);
/* Same for all slots into device memory xyz_dev[n_slots][3] of dtype. */
int ht_vertex_coords_device(ht_mesh* mesh, int level, int dtype,
                            void* xyz_dev, ht_stream stream);
/* Slot flags for all slots into device memory (uint8[n_slots]). */
int ht_slot_flags_device(ht_mesh* mesh, int level, uint8_t* flags_dev,
                         ht_stream stream);
/* Slot of local index (i,j,k), i+j+k <= 2^level, of macro-cell `cell`. */
int ht_slot_index(const ht_mesh* mesh, int level, int64_t cell, int i, int j,
                  int k, int64_t* slot);
/* Class-partial stencils of every cell at a level: out[nc][16][15] doubles.
 * Class c (bits: i==0, j==0, k==0, i+j+k==n) entry d is the sum of the
 * element-matrix entries of the cell's micro-tets around a point of class c
 * that connect it to offset d (offset order in the documentation). */
int ht_cell_stencils(const ht_mesh* mesh, int level, double* out);

/* Stencil offsets of the P2 operator (ht_apply_p2) on the finer lattice:
 * len[8] offsets per node parity p = (i & 1) | (j & 1) << 1 | (k & 1) << 2
 * and d[8][65][3] their (di, dj, dk), sorted by (dk, dj, di). */
int ht_p2_offsets(int* len, int* d);
/* Class-partial P2 stencils of every cell at P2 level `level`:
 * out[nc][8][16][65] doubles, [parity][boundary class of the fine point]
 * [offset]; entry t is the sum of the P2 element-matrix entries of the
 * cell's micro-tets around such a point that connect it to offset t. */
int ht_p2_stencils(const ht_mesh* mesh, int level, double* out);

/* ------------------------------------------------------- vector ops ---- */
/* Make a vector consistent: every copy takes its owner's value.
 * Section 2 (domain partitioning): each coarse-mesh primitive owns the data
 * of its interior points, and a point on a shared face, edge or vertex is
 * held once by its owning primitive and as a copy by every macro-cell that
 * touches it; this is the exchange from owners to copies.  Works in place on
 * v (n_slots elements of dtype, device memory); asynchronous on `stream`;
 * HT_ERR_LEVEL for a level outside the mesh's range. */
int ht_sync(ht_mesh* mesh, int level, int dtype, void* v, ht_stream stream);
/* Set all Dirichlet slots to `value` (all copies). */
int ht_fill_dirichlet(ht_mesh* mesh, int level, int dtype, void* v,
                      double value, ht_stream stream);
/* Lumped P1 mass m_i = sum_{T contains i} |T|/4 at every slot. */
int ht_lumped_mass(ht_mesh* mesh, int level, int dtype, void* m,
                   ht_stream stream);
/* Euclidean norm over unique non-Dirichlet micro-vertices (synchronises). */
int ht_norm(ht_mesh* mesh, int level, int dtype, const void* v, double* norm,
            ht_stream stream);
/* Dot product over unique non-Dirichlet micro-vertices (synchronises). */
int ht_dot(ht_mesh* mesh, int level, int dtype, const void* a, const void* b,
           double* dot, ht_stream stream);

/* dst = src over all n_slots slots (a plain streaming copy). */
int ht_copy(ht_mesh* mesh, int level, int dtype, const void* src, void* dst,
            ht_stream stream);

/* ------------------------------------------------------------ operators - */
/* y = A x: the P1 Laplacian row sum_j a_ij x_j at every non-Dirichlet
 * micro-vertex (Section 5.2.2), y = 0 at Dirichlet ones.  x and y must not
 * alias. */
int ht_apply(ht_mesh* mesh, int level, int dtype, const void* x, void* y,
             ht_stream stream);
/* y = A_k x for the variable-coefficient operator div(k grad) of the
 * paper's operator catalogue (Section 5.2.1, evaluated element by element):
 * a_ij = sum over micro-tets T of the integral over T of
 * k grad(phi_i) . grad(phi_j), with k the P1 field whose point values are
 * `kappa` (same layout and dtype as x, all copies consistent, e.g. after
 * ht_sync); the linear interpolant of k is integrated exactly, so T
 * contributes the mean of k at its vertices times its element matrix.
 * y = 0 at Dirichlet micro-vertices; Dirichlet values of x act as data.
 * The library keeps per-level couplings (36 values per cell) after the first
 * call on a level.  y must not alias x or kappa. */
int ht_apply_divkgrad(ht_mesh* mesh, int level, int dtype, const void* kappa,
                      const void* x, void* y, ht_stream stream);
/* Stored-stencil variant of the same operator (the paper's grid-aware
 * precomputation, Section 5.2.1): the rows are assembled once and stored in
 * the iteration order instead of a sparse format.
 * ht_assemble_divkgrad writes, for every slot, the 15 entries of its row of
 * A_k (the cell's partial row at shared points) into `rows`, which holds
 * 15 * n_slots elements of `dtype` laid out [cell][offset d][closure slot]
 * (offset order in the documentation; entry 0 is the diagonal).
 * ht_apply_stored computes y = A x from such rows (zero at Dirichlet
 * micro-vertices).  Both reject levels where one cell's rows exceed 2 GiB
 * (HT_ERR_LEVEL). */
int ht_assemble_divkgrad(ht_mesh* mesh, int level, int dtype,
                         const void* kappa, void* rows, ht_stream stream);
int ht_apply_stored(ht_mesh* mesh, int level, int dtype, const void* rows,
                    const void* x, void* y, ht_stream stream);
/* y = A x for the P2 (quadratic Lagrange) Laplacian of P2 level `level`
 * (Section 5.1: one DoF per micro-vertex and one per micro-edge, the vertex
 * and the seven edge subgroups; element matrices of Section 5.2.1).  The P2
 * nodes of level l are the micro-vertices of level l + 1, so x and y are
 * vectors of level l + 1 (n_slots(l + 1) elements of `dtype`, closure
 * layout, consistent copies): the point (i, j, k) of that level is a vertex
 * DoF when i, j, k are all even and otherwise the DoF of the micro-edge whose
 * midpoint it is.  y = 0 at Dirichlet nodes (those on the domain boundary);
 * Dirichlet values of x act as data.  Needs 0 <= level and min_level <=
 * level + 1 <= max_level (HT_ERR_LEVEL).  The library keeps the stencils of
 * each P2 level (8 node parities x 16 boundary classes x 65 offsets per
 * cell) after the first call.  y must not alias x. */
int ht_apply_p2(ht_mesh* mesh, int level, int dtype, const void* x, void* y,
                ht_stream stream);
/* Layouts of the per-cell subgroup arrays of ht_p2_pack / ht_p2_unpack. */
enum { HT_LAYOUT_AOS = 0, HT_LAYOUT_SOA = 1 };
/* Convert P2 functions with m components per node (1 <= m <= 64) between
 * the library's lattice layout and the paper's subgroup arrays (subgroup
 * table; Section 4, AoS and SoA linearisations).
 * `lattice`: m vectors of level + 1 (n_slots(level + 1) elements each, back
 * to back).  `arrays`: per cell, in cell order, m * N_tet(2^(level+1) + 1)
 * elements: the subgroups vertex, x, y, z, xy, xz, yz, xyz one after the
 * other, subgroup g holding the N_tet(w_g) micro-primitives of its polytope
 * (widths 2^level + 1, 2^level six times, 2^level - 1) in t_w order, each
 * with its m DoFs: element m t_w + d (HT_LAYOUT_AOS) or d N_tet(w_g) + t_w
 * (HT_LAYOUT_SOA).  Subgroup g at index (i, j, k) is the point
 * 2 (i, j, k) + s_g of level + 1, s_g = (0,0,0), (1,0,0), (0,1,0), (0,0,1),
 * (1,1,0), (1,0,1), (0,1,1), (1,1,1): the micro-vertex, or the midpoint of
 * the micro-edge of that direction based at (i, j, k).  ht_p2_unpack writes
 * every copy of a shared node from its cell's arrays and leaves padding
 * slots alone.  HT_ERR_LEVEL / HT_ERR_ARG as for ht_apply_p2. */
int ht_p2_pack(ht_mesh* mesh, int level, int dtype, int m, int layout,
               const void* lattice, void* arrays, ht_stream stream);
int ht_p2_unpack(ht_mesh* mesh, int level, int dtype, int m, int layout,
                 const void* arrays, void* lattice, ht_stream stream);
/* r = b - A u (0 at Dirichlet); if norm != NULL, also ||r||_2 over unique
 * non-Dirichlet micro-vertices (synchronises the stream).
 * Section 5.2 (operator design): iterative solvers need only the action of
 * the operator on a vector; the residual is that action (the stencil apply
 * of Section 5.2.2) subtracted from the right-hand side in the same pass.
 * u, b: consistent inputs, r: output, each n_slots elements of dtype in
 * device memory; r must not alias u.  Dirichlet values of u act as data.
 * Asynchronous unless norm != NULL; HT_ERR_LEVEL / HT_ERR_ARG on a bad level
 * or dtype. */
int ht_residual(ht_mesh* mesh, int level, int dtype, const void* u,
                const void* b, void* r, double* norm, ht_stream stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): ht_residual
 * with its scratch, the norm partials, in a fixed device array of the
 * library (4 MiB per GPU, held until the process ends) instead of the
 * mesh's buffers.  The norm, if norm_dev != NULL, is written to that DEVICE
 * address (one FP64 value) without synchronising.  Allocates nothing, on
 * the device or through any library routine.  Requires the mesh to be on
 * the device already (any earlier device call puts it there):
 * HT_ERR_STATE otherwise.  HT_ERR_ARG when the level's partials (one per
 * stencil-kernel wave and exchange block, plus 256) exceed the array:
 * 2^19 values, which covers the 288-cell box at level 8.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU race (order
 * them on one stream).  Arguments and results otherwise as ht_residual. */
int ht_residual_noalloc(ht_mesh* mesh, int level, int dtype, const void* u,
                        const void* b, void* r, double* norm_dev,
                        ht_stream stream);
/* `sweeps` weighted Jacobi sweeps u <- u + omega D^-1 (b - A u).
 * Section 5.2.1: smoothers that need only operator applications and the
 * diagonal suit matrix-free operators (Jacobi, and its Chebyshev
 * acceleration); the diagonal is the stencil's centre weight of Section
 * 5.2.2.  u is updated in place (consistent on exit); b is read; both
 * n_slots elements of dtype in device memory; Dirichlet values of u are
 * kept.  sweeps >= 0 (HT_ERR_ARG otherwise); asynchronous on `stream`. */
int ht_smooth_jacobi(ht_mesh* mesh, int level, int dtype, double omega,
                     int sweeps, void* u, const void* b, ht_stream stream);
/* r_coarse = P^T r_fine (Dirichlet entries of r_fine taken as zero, coarse
 * Dirichlet entries set to zero); P = nested P1 interpolation.
 * Section 5.1: a function holds a coefficient vector on every level of the
 * hierarchy, and the regular refinement of Section 3.1 nests the P1 spaces,
 * so the transfer operators of geometric multigrid are fixed by the mesh.
 * r_fine: n_slots(fine_level) elements, r_coarse: n_slots(fine_level - 1)
 * elements, both dtype in device memory; the output is consistent.
 * HT_ERR_LEVEL unless min_level < fine_level <= max_level. */
int ht_restrict(ht_mesh* mesh, int fine_level, int dtype, const void* r_fine,
                void* r_coarse, ht_stream stream);
/* u_fine += P e_coarse (Dirichlet entries of e_coarse taken as zero).
 * The prolongation of Section 5.1's level hierarchy (P1 interpolation on
 * the refinement of Section 3.1): a new point is the midpoint of a coarse
 * micro-edge and takes the mean of the edge's end values.  e_coarse:
 * n_slots(coarse_level), u_fine: n_slots(coarse_level + 1) elements of
 * dtype in device memory, u_fine updated in place (consistent on exit).
 * HT_ERR_LEVEL unless min_level <= coarse_level < max_level. */
int ht_prolongate_add(ht_mesh* mesh, int coarse_level, int dtype,
                      const void* e_coarse, void* u_fine, ht_stream stream);
/* Exact solve of the interior equations at `level` (dense Cholesky inverse
 * computed on the host at first use), Dirichlet values of u kept.
 * The coarsest level of a multigrid hierarchy (Section 5.1; the paper's
 * remark on the minimum refinement level, Section 3.2, puts it at level 2
 * or above, where every micro-primitive subgroup exists).  b read, u
 * written: n_slots elements of dtype in device memory.  The library keeps
 * the inverse (FP64,
 * one dense block per problem of a batch mesh) per level, so the coarse
 * level must stay small (its memory grows with the square of its unknowns);
 * HT_ERR_MESH if the interior matrix is not positive definite, HT_ERR_LEVEL
 * outside the mesh's range. */
int ht_coarse_solve(ht_mesh* mesh, int level, int dtype, const void* b,
                    void* u, ht_stream stream);
/* One V(nu1, nu2) cycle for A u = b at `level` down to opts->coarse_level.
 * Section 6 runs its solvers as V(1,1) cycles inside full multigrid; the
 * cycle here is the textbook one built from the calls above: nu1 smoothing
 * sweeps, residual, restriction, the cycle (or the coarse solve) one level
 * down from a zero guess, prolongation of the correction, nu2 sweeps.
 * u updated in place, b read: n_slots(level) elements of dtype in device
 * memory, consistent.  The library keeps per-level work vectors and may
 * replay the cycle from a captured HIP graph.  HT_ERR_ARG for negative
 * sweep counts or coarse_level outside [min_level, level]. */
int ht_vcycle(ht_mesh* mesh, int level, int dtype, const ht_cycle_opts* opts,
              void* u, const void* b, ht_stream stream);
/* Solve A u = b (u, b: HT_F64 vectors) from the given u.  HT_PREC_F64 runs
 * FP64 V-cycles; HT_PREC_MIXED runs FP32 V-cycles inside FP64 iterative
 * refinement (FP64 residual, FP64 update, FP64 coarse solve).  Synchronises
 * once per cycle to read the residual norm.
 * Repeats the V-cycle of Section 6's solvers until the relative residual
 * ||b - A u|| / ||b|| falls below opts->rel_tol, or opts->max_cycles
 * cycles have run, or three cycles in a row bring no new minimum of the
 * residual (stats->stagnated; both HT_ERR_NOT_CONVERGED, u holds the last
 * iterate).  u
 * updated in place, b read: n_slots(level) FP64 elements in device memory;
 * stats (host, may be NULL) receives the cycle count, final relative
 * residual, wall time and residual history. */
int ht_solve(ht_mesh* mesh, int level, const ht_solve_opts* opts, void* u,
             const void* b, ht_solve_stats* stats, ht_stream stream);

/* -------------------------------------------------------------- batch -- */
/* Many independent small problems solved together.  The paper's data
 * structures make every problem a set of macro-cells refined in the same way
 * (Sections 2-3), so the problems of a batch are laid side by side as one
 * disjoint mesh and each kernel launch covers every problem that is active
 * on a level: a V-cycle over absolute levels where problem p joins at its
 * own finest level.  One launch sequence (captured as one hipGraph) then
 * serves the whole batch instead of one per problem.
 *
 * ht_batch_create: n meshes and the finest level of each (within that
 * mesh's level range).  The meshes' host descriptions are copied; the
 * meshes themselves are not referenced afterwards and may be destroyed.
 * HT_ERR_ARG for n < 1 or a NULL mesh, HT_ERR_LEVEL for a level outside a
 * mesh's range. */
int ht_batch_create(ht_mesh* const* meshes, const int* levels, int n,
                    ht_batch** out);
int ht_batch_destroy(ht_batch* batch);
/* The batch's union mesh (owned by the batch; valid until ht_batch_destroy),
 * for the tuning queries and setters below. */
int ht_batch_mesh(ht_batch* batch, ht_mesh** mesh);
/* ht_autotune for every level of the batch's union mesh from its lowest
 * level to the largest finest level, in FP64 and FP32, each on the
 * problems present on that level; then drops the batch's captured graphs.
 * cache_path as for ht_autotune.  Synchronises. */
int ht_batch_autotune(ht_batch* batch, const char* cache_path, ht_stream stream);
/* Number of problems, their total unknowns (interior DoFs at each problem's
 * finest level) and total macro-cells; any output may be NULL. */
int ht_batch_query(const ht_batch* batch, int* n_problems, int64_t* n_dofs,
                   int64_t* n_cells);
/* Solve A_p u_p = b_p for every problem p.  u[p], b[p]: HT_F64 device
 * vectors in the layout of mesh p at its finest level (n_slots of
 * ht_mesh_query for that mesh and level); u[p] holds the initial iterate
 * and receives the solution.  Every problem runs V(nu1, nu2) cycles until
 * its own relative residual is <= rel_tol, or until it stagnates as in
 * ht_solve (stats[p].stagnated); its result is the iterate of the cycle at
 * which it stopped (later cycles of the batch do not change it), so it
 * equals what ht_solve computes for that problem alone, up to rounding.  stats: array of n, one per problem.  opts->precision:
 * HT_PREC_F64 (FP64 V-cycles) or HT_PREC_MIXED (FP32-in-FP64 iterative
 * refinement as in ht_solve: FP32 correction cycles of all problems in one
 * batched V-cycle, FP64 residuals, norms and updates).  The Jacobi smoother
 * is required, and opts->cyc.coarse_level must not exceed any problem's
 * finest level.  Synchronises once per cycle.  HT_ERR_NOT_CONVERGED if
 * some problem did not converge (all stats filled, all u[p] written). */
int ht_batch_solve(ht_batch* batch, const ht_solve_opts* opts,
                   void* const* u, const void* const* b, ht_solve_stats* stats,
                   ht_stream stream);

/* Smoothers.  HT_SMOOTH_JACOBI: omega-weighted Jacobi sweeps.
 * HT_SMOOTH_CHEBYSHEV: the Chebyshev iteration of the given degree for the
 * Jacobi-preconditioned system D^-1 A u = D^-1 b on [beta/8, beta] (the
 * paper's large runs accelerate Jacobi with Chebyshev polynomials, Sections
 * 5.2.1 and 6), beta = 1.1 times the estimate of ht_lambda_max.  The
 * estimates are computed once per level on first use (before any graph
 * capture).  ht_lambda_max: 20 power iterations v <- D^-1 A v from
 * v = sin(1000 x + 1700 y + 2300 z) (zero on the boundary); the estimate is
 * |v_20| / |v_19| over the unique non-Dirichlet micro-vertices.  Allocates
 * two scratch vectors; synchronises. */
int ht_lambda_max(ht_mesh* mesh, int level, double* lambda, ht_stream stream);
/* Sets the estimate used at `level` in place of the power iteration (for
 * instance a value computed elsewhere, to run two implementations with one
 * interval).  Host call; drops every captured graph of the mesh.
 * HT_ERR_ARG unless lambda is positive and finite; HT_ERR_LEVEL outside the
 * mesh's level range. */
int ht_set_lambda_max(ht_mesh* mesh, int level, double lambda);

/* Full multigrid (nested iteration) for A u = b at `level` with zero
 * Dirichlet data.  A function lives on every level (Section 5.1), so the
 * right-hand side is carried down by the restriction (b_{l-1} = R b_l),
 * the system at opts->coarse_level is solved exactly, and on each finer
 * level the interpolated coarser solution (P u_{l-1}) starts `cycles`
 * V(nu1, nu2) cycles.  u: HT_F64 output at `level` (overwritten;
 * Dirichlet slots set to 0); b: HT_F64 right-hand side.  rel_res (may be
 * NULL): ||b - A u||_2 / ||b||_2 of the result, which synchronises.  The
 * whole sequence is captured once per (level, opts, cycles, u, b) as a
 * hipGraph and replayed.  HT_ERR_ARG for cycles outside [1, 64]. */
int ht_fmg(ht_mesh* mesh, int level, const ht_cycle_opts* opts, int cycles,
           void* u, const void* b, double* rel_res, ht_stream stream);

/* ------------------------------------------------------------- tuning -- */
/* The tile kernel runs one wavefront per tile of 64 i-points x R rows,
 * marching in k, four wavefronts per workgroup.  R in {4, 8, 16} trades
 * register pressure against halo re-reads.  R = 0 selects the band kernel
 * (whole rows of a cell staged plane by plane in LDS), available up to the
 * level where a band of four rows still fits its LDS image (level 8).
 * ht_set_tile_rows fixes R for the apply and the restriction at (level,
 * dtype) (the restriction takes R = 4 when the apply takes the band
 * kernel); ht_get_tile_rows reports the current choice (default: the band
 * kernel where it is available, else 4). */
int ht_set_tile_rows(ht_mesh* mesh, int level, int dtype, int rows);
int ht_get_tile_rows(const ht_mesh* mesh, int level, int dtype, int* rows);
/* Tile shape of the sweep operations (residual, Jacobi, FP32 residual,
 * Chebyshev step), which also stream b: R rows per wave and the workgroup's
 * arrangement, waves_in_i = 1 for its four waves side by side in i (one
 * contiguous run of 248 points per row), 0 for stacked in j.  R = 0 runs
 * the Jacobi sweep and the residual on the band kernel (the FP32 residual
 * and the Chebyshev step then use R = 4) where it is available.  Default:
 * the band kernel from level 7 on, else R = 4; waves_in_i = 1 from level 8
 * on (0 below).  Results do not depend on the shape (up to rounding). */
int ht_set_sweep_shape(ht_mesh* mesh, int level, int dtype, int rows,
                       int waves_in_i);
int ht_get_sweep_shape(const ht_mesh* mesh, int level, int dtype, int* rows,
                       int* waves_in_i);
/* March segment of the sweep operations: a wavefront's k-march is split
 * into segments of `planes` planes (32, 64 or 128; each segment reloads two
 * planes), which evens out the work per wave.  Default 32 with the waves
 * side by side in i, 64 stacked.  HT_ERR_ARG for another length.  Results
 * do not depend on it. */
int ht_set_march_segment(ht_mesh* mesh, int level, int dtype, int planes);
int ht_get_march_segment(const ht_mesh* mesh, int level, int dtype, int* planes);
/* Autotuner: times the band kernel and every R on the live apply at
 * (level, dtype) on `stream`, and every (R, arrangement, march segment) on
 * the live Jacobi sweep (three scratch vectors are allocated and freed),
 * keeps the fastest of each and returns the apply's choice in *rows (0 =
 * band kernel).  Only the cells present on the level take part (all of a
 * plain mesh; in a batch's union mesh, the problems whose finest level is at
 * least `level`).  With cache_path != NULL (or, when it is NULL, the path in
 * the environment variable HT_TUNE_CACHE if set and not empty) a text cache
 * keyed by (gfx arch, level, dtype, cells, cell stride) is read first and
 * appended to after tuning; ht_batch_autotune reads the same variable.  Captured graphs of the mesh are dropped (they hold the old
 * shapes).  Synchronises. */
int ht_autotune(ht_mesh* mesh, int level, int dtype, const char* cache_path,
                int* rows, ht_stream stream);

/* ---------------------------------------------------------- profiling -- */
/* Record HIP events around every kernel the library launches. */
int ht_profile_enable(ht_mesh* mesh, int enable);
/* Summed device milliseconds and launch count of kernels whose name starts
 * with `prefix` since the last reset (synchronises). */
int ht_profile_query(ht_mesh* mesh, const char* prefix, double* ms,
                     int64_t* launches);
int ht_profile_reset(ht_mesh* mesh);

/* Diagnostics: runs a one-wave kernel that checks the cross-lane shifts the
 * stencil kernel relies on; *mismatches = number of wrong lanes (0 = OK). */
int ht_selftest_lane_shift(int* mismatches);

#ifdef __cplusplus
}
#endif
#endif /* HYTET_H */
