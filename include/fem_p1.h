/*
 * fem_p1.h -- C ABI of the MI355X (gfx950) P1 finite element assembly library.
 *
 * The library assembles the global sparse matrices of P1 Lagrange elements on
 * a 2D triangle mesh, after Cuvelier, Japhet and Scarella, "An efficient way
 * to perform the assembly of finite element matrices in Matlab and Octave"
 * (INRIA RR-8305, 2013):
 *   M    mass            M_ij    = int phi_i phi_j            (eq. MassElem)
 *   Mw   weighted mass   Mw_ij   = int w phi_i phi_j, w P1    (eq. MassWElem)
 *   S    stiffness       S_ij    = int grad phi_i . grad phi_j (eq. StiffMatElem)
 *   K    elasticity      K_ml    = int eps(psi_m)^T C eps(psi_l)
 *                        (linear elasticity section; Hooke's law, Lame
 *                        parameters lambda, mu with lambda + mu > 0)
 *
 * Inputs follow the paper's problem statement (Notations section), 0-based:
 *   q  : [nq][2]  double, vertex coordinates (the paper's 2 x nq array q)
 *   me : [nme][3] int32,  connectivity; me[k][a] is the a-th vertex of
 *                 triangle k (the paper's 3 x nme array me, minus one)
 *   w  : [nq]     double, the weight sampled at the vertices (Tw)
 * Triangle areas are computed from q (the paper passes them in).
 *
 * Output format: CSR (row_ptr, col_idx, values) with rows ascending, columns
 * ascending and unique inside each row.  The pattern is structural: it holds
 * every (i, j) with i and j in a common triangle, including entries whose
 * value happens to be zero (Matlab's sparse() would drop those).  All four
 * matrices share one scalar pattern; the elasticity matrix uses the derived
 * 2 x 2 block layout below.
 *
 * Memory and streams.  Every array argument is a DEVICE pointer unless
 * marked HOST.  The caller owns all memory; the library never allocates
 * device memory.  Every call enqueues work on `stream` (a hipStream_t passed
 * as void*; NULL is the default stream) and returns without waiting, except
 * fem_pattern, which waits once for the number of nonzeros and the mesh
 * checks.  Calls that overlap on the same output buffers race.
 *
 * Errors.  Every function returns a fem_status.  Argument checks run on the
 * host before anything is enqueued; mesh checks (indices in range, distinct
 * vertices per triangle) run on the device inside fem_pattern.  On error,
 * fem_last_error() returns a message (thread-local, valid until the next
 * call from the same thread).  Values of outputs are unspecified after an
 * error.
 */
#ifndef FEM_P1_H
#define FEM_P1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fem_status {
    FEM_OK = 0,
    FEM_EINVAL = -1,       /* bad argument (NULL pointer, negative size, lambda + mu <= 0, ...) */
    FEM_ERANGE = -2,       /* a vertex index of me outside [0, nq) */
    FEM_EDEGEN = -3,       /* a triangle repeats a vertex */
    FEM_ENOSPC = -4,       /* an output or workspace capacity is too small */
    FEM_EOVERFLOW = -5,    /* a count does not fit the int32 index type */
    FEM_EHIP = -6,         /* the HIP runtime reported an error */
    FEM_EUNSUPPORTED = -8  /* a row longer than 65535 entries */
} fem_status;

/* flags of the numeric calls */
enum {
    FEM_DETERMINISTIC = 0, /* row-owner gather: every value summed by one lane in a fixed
                              order; bitwise reproducible from run to run (default) */
    FEM_ATOMIC = 1,        /* one lane per triangle, FP64 atomic adds through the slot map
                              (needs me and slot); order of additions unspecified */
    FEM_ACCUMULATE = 2,    /* add into values instead of overwriting them */
    FEM_PACKED_QW = 4,     /* fem_adjoint_stiff_wmass, and fem_assemble with FEM_OP_WMASS
                              in the row-owner scheme: the first 32 nq bytes of the
                              workspace already hold the (x, y, w, 0) record of every vertex
                              for these q and w, as fem_assemble leaves them in its own
                              workspace when it assembles Mw (pass the same buffer again);
                              the packing pass is skipped.  fem_assemble returns FEM_EINVAL
                              for it without FEM_OP_WMASS or with FEM_ATOMIC, FEM_ENOSPC
                              without a workspace of 32 nq bytes */
    FEM_CHECK_AREA = 8     /* fem_assemble only: also test every triangle for zero area
                              (det = (q2-q3) x (q3-q1) == 0, where the element formulas
                              divide by zero) and return FEM_EDEGEN if one has it; uses the
                              workspace of fem_assemble_workspace and waits for the stream */
};

/* Tunable launch shape of the row-owner kernels. */
typedef struct fem_tune {
    int32_t lds_entries;   /* CSR entries staged in LDS per 64-row wave tile (rounded to a
                              compiled size in 256..1024, capped by 64 KiB of LDS; 0: 512) */
    int32_t grid_blocks;   /* persistent grid: number of one-wave workgroups that loop over
                              the tiles (0: one workgroup per tile) */
    int32_t variant;       /* 0: row accumulators in registers for rows of <= 8 entries,
                              longer rows per lane in register chunks of 8 (default);
                              1: row accumulators in LDS */
} fem_tune;

/* Message of the last failing call on this thread ("" if none). */
const char *fem_last_error(void);

/* Library ABI version (major * 100 + minor). */
int fem_version(void);

/* ------------------------------------------------------------------------ */
/* Symbolic phase                                                            */
/* ------------------------------------------------------------------------ */

/* HOST ONLY.  Bytes of device workspace fem_pattern needs for a mesh with nq
 * vertices and nme triangles. */
int fem_pattern_workspace(int32_t nq, int32_t nme, size_t *bytes /* HOST */);

/* Upper bound of the number of nonzeros, nq + 6 nme (each triangle adds at
 * most six off-diagonal entries); a safe col_cap. */
int64_t fem_nnz_bound(int32_t nq, int32_t nme);

/* Builds the CSR pattern of the scalar matrices (replaces the index arrays
 * Ig = me([1 2 3 1 2 3 1 2 3], :), Jg = me([1 1 1 2 2 2 3 3 3], :) and the
 * sort/compress inside sparse(Ig, Jg, Kg, nq, nq) of Section 6), plus the
 * data the numeric calls read:
 *
 *   row_ptr [nq+1]       CSR row offsets
 *   col_idx [col_cap]    CSR column indices; nnz of them are written
 *   inc_ptr [nq+1]       offsets of the triangle lists of each vertex
 *   inc     [3 nme]      for vertex v, the values 3k + a with me[k][a] == v, in
 *                        ascending k (the triangles around v)
 *   inc_pos [3 nme]      for the same entries, the positions inside row v
 *                        (relative to row_ptr[v]) of me[k][(a+1)%3] (low 16
 *                        bits) and me[k][(a+2)%3] (high 16 bits)
 *   fan     [nq]         optional (NULL to skip): the fan code of every row,
 *                        as fem_fan_plan writes it (computed here from the
 *                        rows just built, without a pass of its own)
 *   slot    [9][nme]     optional (NULL to skip): slot[(3b+a) nme + k] is the
 *                        CSR position of entry (me[k][a], me[k][b]) -- local
 *                        entry r = 3b + a of the column-wise element matrix
 *   work    [work_bytes] device workspace, >= fem_pattern_workspace(nq, nme)
 *   nnz_out HOST         number of nonzeros
 *
 * Requires nq >= 1, nme >= 0, 3 nme and nq + 6 nme within int32.  Returns
 * FEM_ERANGE / FEM_EDEGEN for an invalid me, FEM_ENOSPC if col_cap < nnz,
 * FEM_EUNSUPPORTED if a row would exceed 65535 entries.  Synchronises
 * `stream` once (twice when a mesh falls back from the fine to the coarse
 * bucket path); what follows the synchronisation is enqueued asynchronously.
 * Integer results are identical on every run and on every path. */
int fem_pattern(int32_t nq, int32_t nme, const int32_t *me,
                int32_t *row_ptr, int32_t *col_idx, int64_t col_cap,
                int32_t *inc_ptr, int32_t *inc, uint32_t *inc_pos,
                uint64_t *fan, int32_t *slot,
                void *work, size_t work_bytes,
                int64_t *nnz_out /* HOST */, void *stream);

/* HOST ONLY.  Which algorithm fem_pattern uses to group the incidences by
 * vertex (all give identical outputs):
 *   FEM_PATTERN_AUTO    fine buckets of 512 vertices sorted and turned into
 *                       rows in one kernel; coarse buckets of 4096 vertices
 *                       when a fine bucket does not fit (a vertex with more
 *                       than 64 triangles, or more than 4096 incidences in a
 *                       bucket); atomic counting beyond 151M vertices
 *   FEM_PATTERN_COARSE  coarse buckets, then per-vertex row kernels
 *   FEM_PATTERN_ATOMIC  per-vertex atomic counters, then per-vertex row kernels
 * A process-wide setting, meant for tests and tuning; returns FEM_EINVAL for
 * an unknown value and FEM_EUNSUPPORTED for FEM_PATTERN_COARSE on a mesh the
 * coarse histogram cannot hold (checked by fem_pattern). */
enum {
    FEM_PATTERN_AUTO = 0,
    FEM_PATTERN_COARSE = 1,
    FEM_PATTERN_ATOMIC = 2
};
int fem_pattern_set_path(int path);

/* Transpose map: tpos[p] is the position of entry (j, i) for the entry
 * p = (i, j), or -1 if the pattern has no entry (j, i) (every P1 mesh
 * pattern is structurally symmetric, so -1 never occurs there). */
int fem_transpose_map(int32_t nq, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      int32_t *tpos, void *stream);

/* Fan codes: for every row i, the order in which turning around vertex i
 * meets its triangles (one uint64 per row, fan [nq]).  Step j of the walk is
 * the triangle (i, s_j, s_{j+1}) in its own vertex order, so an off-diagonal
 * entry receives exactly the two terms of consecutive steps and the numeric
 * kernels need no search of the row per triangle.  Built from the arrays
 * fem_pattern wrote (row_ptr, inc_ptr, inc_pos; no other input), once per
 * mesh (fem_pattern writes the same codes when given its fan argument).  A
 * row gets code 0 -- and is then summed in ascending triangle order -- unless its triangles form a single consistently oriented fan
 * (closed around an inner vertex, open at a boundary vertex) of at most 13
 * neighbours; so on a mesh whose triangles are all counter-clockwise (or all
 * clockwise) every manifold row with up to 13 neighbours has one.  Layout:
 *   bits 0..3 n (slots on the walk, 0: none), bit 4 closed, bits 5..8 the
 *   diagonal's slot, bits 9 + 4j.. slot s_j (positions relative to
 *   row_ptr[i]). */
int fem_fan_plan(int32_t nq, int32_t nme, const int32_t *row_ptr, const int32_t *inc_ptr,
                 const uint32_t *inc_pos, uint64_t *fan, void *stream);

/* Elasticity pattern over the 2 nq degrees of freedom psi_{2i} = (phi_i, 0),
 * psi_{2i+1} = (0, phi_i) (the paper's interleaved basis, 0-based): row
 * 2i + alpha holds columns 2j, 2j + 1 for every column j of scalar row i.
 *   row_ptr_e [2nq+1]: row_ptr_e[2i] = 4 row_ptr[i],
 *                      row_ptr_e[2i+1] = 4 row_ptr[i] + 2 len_i
 *   col_idx_e [4 nnz], 8-byte aligned (FEM_EINVAL otherwise)
 * Entry (2i+alpha, 2j+beta), j the p-th column of row i, sits at
 * 4 row_ptr[i] + 2 alpha len_i + 2 (p - row_ptr[i]) + beta. */
int fem_elas_pattern(int32_t nq, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     int32_t *row_ptr_e, int32_t *col_idx_e, void *stream);

/* ------------------------------------------------------------------------ */
/* Numeric phase                                                             */
/* ------------------------------------------------------------------------ */
/* Common arguments: nq, nme, nnz and the arrays written by fem_pattern.
 * FEM_DETERMINISTIC reads q (w), row_ptr, col_idx, inc_ptr, inc_pos and, if
 * not NULL, the fan codes of fem_fan_plan for the same pattern; me and slot
 * may be NULL.  The order of additions is fixed by these arrays: with fan
 * codes, the diagonal of a row that has one sums its triangles in walk
 * order (every off-diagonal value is a sum of two terms, whose order does
 * not matter), otherwise in ascending triangle order; either way the values
 * do not depend on the launch shape or on which operators share the call.  FEM_ATOMIC reads q (w), me, slot (and row_ptr for the
 * elasticity layout); it clears values first unless FEM_ACCUMULATE.  values
 * has nnz entries (4 nnz for elasticity, in the layout of fem_elas_pattern).
 * Element formulas: Section 2 (MassElem, MassWElem, StiffMatElem) and the
 * elasticity section (K^e = |T| B^T C B); |T| = |det| / 2. */

int fem_assemble_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                      const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                      const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                      double *values, int flags, void *stream);

int fem_assemble_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                       const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                       const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                       const double *w, double *values, int flags, void *stream);

int fem_assemble_stiff(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                       const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                       const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                       double *values, int flags, void *stream);

/* Operator bits of fem_assemble. */
enum { FEM_OP_MASS = 1, FEM_OP_WMASS = 2, FEM_OP_STIFF = 4, FEM_OP_ELAS = 8 };

/* HOST ONLY.  Workspace bytes of fem_assemble for the operator set `ops`:
 * 32 nq (rounded up to 256) when FEM_OP_WMASS is requested (packed (x, y, w)
 * records, one random access per column instead of two), plus 256 bytes for
 * the flag of FEM_CHECK_AREA.  The workspace is optional without that flag. */
int fem_assemble_workspace(int32_t nq, int ops, size_t *bytes /* HOST */);

/* Any nonzero subset `ops` of {M, Mw, S, K} in ONE pass over the mesh: the
 * gathers of q (and w) by column -- every one a random access on a
 * relabelled mesh -- are shared by all requested operators.  Outputs of
 * operators not in `ops` may be NULL; vals_K [4 nnz] uses the layout of
 * fem_elas_pattern; lambda, mu are read only for FEM_OP_ELAS (then
 * lambda + mu > 0 is required).  work / work_bytes: optional device
 * workspace (fem_assemble_workspace), NULL allowed.  tune: optional launch
 * shape of the row-owner kernel (NULL: defaults).  Other arguments and flags
 * as in the single-operator calls below, which are this call with one bit. */
int fem_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q, const double *w,
                 const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                 const int32_t *inc_ptr, const uint32_t *inc_pos, const uint64_t *fan,
                 const int32_t *slot, double lambda, double mu, double *vals_M, double *vals_Mw,
                 double *vals_S,
                 double *vals_K, void *work, size_t work_bytes, const struct fem_tune *tune,
                 int flags, void *stream);

/* Measurement aid (not part of the assembly): the random accesses of the
 * row-owner kernels without their arithmetic.  Reads col_idx[e] and the
 * 16-byte vertex record q[col_idx[e]] for every e < nnz (mode 0), or q[e mod
 * nq] in stream order (mode 1); writes one partial sum per thread to sink
 * [fem_gather_probe_threads()].  The time of mode 0 is the floor that
 * random gathers set on a relabelled mesh. */
int fem_gather_probe_threads(void);
int fem_gather_probe(int64_t nnz, int32_t nq, const int32_t *col_idx, const double *q, int mode,
                     double *sink, void *stream);

/* fem_assemble for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * allocation): the same arguments and results without the workspace.  The
 * packed (x, y, w) records of the weighted mass and the FEM_CHECK_AREA flag
 * live in a fixed device array of the library (32 FEM_NOALLOC_MAX_NQ + 256
 * bytes, 32 MiB + 256; each GPU the library runs on holds its own copy until
 * the process ends); the call allocates nothing.  With FEM_OP_WMASS (row-owner
 * scheme) or FEM_CHECK_AREA, nq above FEM_NOALLOC_MAX_NQ returns FEM_ENOSPC;
 * FEM_PACKED_QW returns FEM_EINVAL.  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (several streams or host threads)
 * race: serialise them. */
#define FEM_NOALLOC_MAX_NQ 1048576
int fem_assemble_noalloc(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                         const double *w, const int32_t *me, const int32_t *row_ptr,
                         const int32_t *col_idx, const int32_t *inc_ptr, const uint32_t *inc_pos,
                         const uint64_t *fan, const int32_t *slot, double lambda, double mu,
                         double *vals_M, double *vals_Mw, double *vals_S, double *vals_K,
                         const struct fem_tune *tune, int flags, void *stream);

/* S and M in one pass over the mesh (shared gathers of q). */
int fem_assemble_stiff_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                            const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                            const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                            double *vals_S, double *vals_M, int flags, void *stream);

/* S and Mw in one pass (the forward of the differentiable assembly). */
int fem_assemble_stiff_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                             const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                             const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                             const double *w, double *vals_S, double *vals_Mw, int flags,
                             void *stream);

/* Elasticity stiffness (requires lambda + mu > 0); values_e [4 nnz] in the
 * layout of fem_elas_pattern. */
int fem_assemble_elas(int32_t nq, int32_t nme, int64_t nnz, const double *q, const int32_t *me,
                      const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                      const uint32_t *inc_pos, const uint64_t *fan, const int32_t *slot,
                      double lambda, double mu, double *values_e, int flags, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched assembly                                                          */
/* ------------------------------------------------------------------------ */

/* Globalises the connectivity of nb meshes stored back to back: triangles
 * elem_off[b] .. elem_off[b+1]-1 index vertices local to mesh b, whose
 * vertices are vtx_off[b] .. vtx_off[b+1]-1 of the concatenated q, so
 * me_global[k][a] = me_local[k][a] + vtx_off[b].  vtx_off, elem_off: DEVICE
 * [nb+1] int64, non-decreasing, elem_off[0] = 0, elem_off[nb] = nme (not
 * checked).  fem_pattern on the result gives the block-diagonal CSR of the
 * batch (block b = rows vtx_off[b] .. vtx_off[b+1]-1); its range check then
 * covers the whole batch. */
int fem_batch_globalize(int32_t nb, int32_t nme, const int64_t *vtx_off, const int64_t *elem_off,
                        const int32_t *me_local, int32_t *me_global, void *stream);

/* S and M of a batched (block-diagonal) pattern in ONE persistent launch;
 * nq, nnz and the pattern arrays are those of the whole batch.  tune may be
 * NULL (defaults).  Same semantics as fem_assemble_stiff_mass with
 * FEM_DETERMINISTIC. */
int fem_assemble_stiff_mass_batched(int32_t nb, int32_t nq, int64_t nnz, const double *q,
                                    const int32_t *row_ptr, const int32_t *col_idx,
                                    const int32_t *inc_ptr, const uint32_t *inc_pos,
                                    const uint64_t *fan, double *vals_S, double *vals_M,
                                    const fem_tune *tune /* HOST, nullable */, int flags,
                                    void *stream);

/* ------------------------------------------------------------------------ */
/* HIP graphs                                                                */
/* ------------------------------------------------------------------------ */

/* Begins capturing `stream` (must not be the NULL stream).  Every numeric
 * call enqueued on it until fem_graph_end is recorded instead of run
 * (fem_pattern must not be captured: it synchronises). */
int fem_graph_begin(void *stream);

/* Ends the capture and instantiates it; *graph_out (HOST) receives an opaque
 * handle for fem_graph_launch / fem_graph_destroy. */
int fem_graph_end(void *stream, void **graph_out /* HOST */);

/* Replays an instantiated graph on `stream`. */
int fem_graph_launch(void *graph, void *stream);

int fem_graph_destroy(void *graph);

/* ------------------------------------------------------------------------ */
/* General sparse(I, J, V, m, n)                                             */
/* ------------------------------------------------------------------------ */

/* HOST ONLY.  Bytes of device workspace fem_sparse needs for nt triplets. */
int fem_sparse_workspace(int32_t m, int32_t n, int64_t nt, size_t *bytes /* HOST */);

/* Matlab's A = sparse(I, J, V, m, n) (the compression that ends every OptV2
 * assembly, Section 6; storage as in Section 4), 0-based and in CSR:
 *   I, J [nt] int32   row and column of each triplet, in [0, m) and [0, n)
 *   V    [nt] f64     values (may be NULL when vals is NULL)
 *   row_ptr [m+1], col_idx [col_cap]   rows ascending, columns ascending, one
 *                     entry per distinct (i, j); entries whose values sum to
 *                     zero are kept (structural)
 *   vals [col_cap] or NULL: vals[p] = sum of V[t] over the triplets of entry p,
 *                     added in ascending t (a left-to-right sum: bitwise
 *                     reproducible, equal to a sequential loop over t)
 *   contrib_ptr [col_cap+1], contrib [nt], both or neither: the triplets of
 *                     entry p are contrib[contrib_ptr[p] .. contrib_ptr[p+1]),
 *                     ascending (fem_sparse_values re-sums new values)
 *   work [work_bytes] >= fem_sparse_workspace(m, n, nt); nnz_out HOST
 * Requires m, n >= 1 and 0 <= nt <= 2^31 - 1.  Returns
 * FEM_ERANGE for an index outside its range, FEM_ENOSPC if col_cap < nnz.
 * Synchronises `stream` once (to return nnz).  Rows whose triplets do not fit
 * the on-chip sort (more than 2688 in a bucket of rows) take a slower path
 * through global memory; results are identical. */
int fem_sparse(int32_t m, int32_t n, int64_t nt, const int32_t *I, const int32_t *J,
               const double *V, int32_t *row_ptr, int32_t *col_idx, double *vals,
               int64_t col_cap, int32_t *contrib_ptr, int32_t *contrib, void *work,
               size_t work_bytes, int64_t *nnz_out /* HOST */, void *stream);

/* vals[p] = sum of V[contrib[k]], k from contrib_ptr[p] to contrib_ptr[p+1] - 1,
 * in that order (the numeric phase of fem_sparse for new values on the same
 * I, J; bitwise equal to what fem_sparse returns for them).  flags: 0 or
 * FEM_ACCUMULATE. */
int fem_sparse_values(int64_t nnz, const int32_t *contrib_ptr, const int32_t *contrib,
                      const double *V, double *vals, int flags, void *stream);

/* ------------------------------------------------------------------------ */
/* P1 tetrahedra in 3D                                                       */
/* ------------------------------------------------------------------------ */

/* HOST ONLY.  Bytes of device workspace fem_tet_pattern needs. */
int fem_tet_pattern_workspace(int32_t nq, int32_t nme, size_t *bytes /* HOST */);

/* HOST ONLY.  nq + 12 nme: an upper bound of the tetrahedron pattern's nnz
 * (a vertex in d tetrahedra has at most 3 d neighbours); a safe col_cap. */
int64_t fem_tet_nnz_bound(int32_t nq, int32_t nme);

/* Pattern of the P1 tetrahedron matrices (the 3D extension named in the
 * Conclusion): the CSR pattern of sparse(Ig, Jg, .) over the 16 local entries
 * of every element (Section 6; entry (a, b) of element k lies at row
 * me[k][a], column me[k][b]), and per vertex its tetrahedra with the row
 * slots of their other vertices, which is what fem_tet_assemble reads.
 *   me [nme][4] int32, 16-byte aligned, 0-based vertex ids
 *   row_ptr [nq+1], col_idx [col_cap]: rows ascending, columns ascending; a
 *                vertex in no tetrahedron has an empty row
 *   inc_ptr [nq+1], inc [4 nme]: the tetrahedra of vertex v as 4 k + a
 *                (me[k][a] == v), ascending, at inc[inc_ptr[v] ..
 *                inc_ptr[v+1])
 *   inc_pos [4 nme]: for inc[i] = 4 k + a in row v, the row slots (offsets
 *                from row_ptr[v]) of me[k][(a+1)%4], me[k][(a+2)%4] and
 *                me[k][(a+3)%4] in bits 0-9, 10-19 and 20-29
 *   work [work_bytes] >= fem_tet_pattern_workspace(nq, nme); nnz_out HOST
 * All outputs are device memory owned by the caller.  Requires 16 nme <=
 * 2^31 - 1 and rows of at most 1024 entries (FEM_EUNSUPPORTED otherwise).
 * FEM_ERANGE / FEM_EDEGEN for an invalid me, FEM_ENOSPC if col_cap < nnz
 * (fem_tet_nnz_bound is always enough).  Synchronises `stream`. */
int fem_tet_pattern(int32_t nq, int32_t nme, const int32_t *me, int32_t *row_ptr,
                    int32_t *col_idx, int64_t col_cap, int32_t *inc_ptr, int32_t *inc,
                    uint32_t *inc_pos, void *work, size_t work_bytes, int64_t *nnz_out /* HOST */,
                    void *stream);

/* HOST ONLY.  Grouping of fem_tet_pattern: FEM_PATTERN_AUTO (buckets of 128
 * vertices in LDS, the general path for meshes beyond their limits) or
 * FEM_PATTERN_COARSE (always the general path: fem_sparse over the 16 nme
 * triplets).  Both give the same arrays bit for bit; for tests. */
int fem_tet_pattern_set_path(int path);

/* P1 tetrahedron mass (FEM_OP_MASS: |K| (1 + delta_ab) / 20) and / or
 * stiffness (FEM_OP_STIFF: |K| grad lambda_a . grad lambda_b), the 3D
 * counterparts of the element matrices of Section 3, summed over the
 * elements as sparse() does (Section 6), on the pattern of fem_tet_pattern.
 * One lane per row; every entry is the sum of its element terms in ascending
 * tetrahedron order (bitwise reproducible).
 *   q [nq][3] f64; row_ptr, col_idx, inc_ptr, inc_pos from fem_tet_pattern
 *   vals_M / vals_S [nnz] device, caller-owned
 * flags: 0 or FEM_ACCUMULATE.  A degenerate (flat) tetrahedron gives
 * non-finite stiffness values, as the element formula does. */
int fem_tet_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                     const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                     const uint32_t *inc_pos, double *vals_M, double *vals_S, int flags,
                     void *stream);

/* ------------------------------------------------------------------------ */
/* P2 (quadratic Lagrange) triangles                                         */
/* ------------------------------------------------------------------------ */

/* HOST ONLY.  Bytes of device workspace fem_p2_dofs needs. */
int fem_p2_dofs_workspace(int32_t nq, int32_t nme, size_t *bytes /* HOST */);

/* Degrees of freedom of the P2 triangle (the P_k extension named in the
 * Conclusion): the nq vertices, then the ne edges, edge e being DOF nq + e,
 * with edges numbered in ascending lexicographic order of (lower vertex,
 * higher vertex).
 *   me [nme][3] int32
 *   dofs [nme][6] int32 (8-byte aligned): v0, v1, v2, then nq + the edge
 *        opposite local vertex 0, 1, 2
 *   edges [edge_cap][2] int32 (8-byte aligned) or NULL: (lower, higher)
 *        vertex of each edge; ne <= 3 nme, and ne = nq + nme - 1 on a
 *        simply connected mesh
 *   work [work_bytes] >= fem_p2_dofs_workspace(nq, nme); ne_out HOST
 * Requires 36 nme <= 2^31 - 1 and nq + ne <= 2^31 - 1 (FEM_EOVERFLOW).
 * FEM_ERANGE / FEM_EDEGEN for an invalid me, FEM_ENOSPC if edges is given and
 * edge_cap < ne.  Synchronises `stream`. */
int fem_p2_dofs(int32_t nq, int32_t nme, const int32_t *me, int32_t *dofs, int32_t *edges,
                int64_t edge_cap, void *work, size_t work_bytes, int64_t *ne_out /* HOST */,
                void *stream);

/* HOST ONLY.  Bytes of device workspace fem_p2_pattern needs. */
int fem_p2_pattern_workspace(int32_t ndof, int32_t nme, size_t *bytes /* HOST */);

/* Pattern of the P2 matrices over ndof = nq + ne DOFs: the CSR pattern of
 * sparse(Ig, Jg, .) over the 36 local entries of every element (Section 6;
 * entry (a, b) of element k at row dofs[k][a], column dofs[k][b]), and per
 * DOF its triangles with the row slots of their six DOFs, which is what
 * fem_p2_assemble reads.
 *   dofs [nme][6] int32 from fem_p2_dofs (8-byte aligned)
 *   row_ptr [ndof+1], col_idx [col_cap]; nnz <= ndof + 30 nme
 *   inc_ptr [ndof+1], inc [6 nme]: the triangles of DOF i as 6 k + a
 *                (dofs[k][a] == i), ascending, at inc[inc_ptr[i] ..
 *                inc_ptr[i+1])
 *   inc_pos [6 nme] uint64 (8-byte aligned): for inc[j] = 6 k + a in row i,
 *                the row slot (offset from row_ptr[i]) of dofs[k][b] in bits
 *                10 b .. 10 b + 9 (b = 0..5), and a in bits 60-62
 *   work [work_bytes] >= fem_p2_pattern_workspace(ndof, nme); nnz_out HOST
 * All outputs are device memory owned by the caller.  FEM_ERANGE for a DOF
 * outside [0, ndof), FEM_ENOSPC if col_cap < nnz, FEM_EUNSUPPORTED for a row
 * over 1024 entries.  Synchronises `stream`. */
int fem_p2_pattern(int32_t ndof, int32_t nme, const int32_t *dofs, int32_t *row_ptr,
                   int32_t *col_idx, int64_t col_cap, int32_t *inc_ptr, int32_t *inc,
                   uint64_t *inc_pos, void *work, size_t work_bytes, int64_t *nnz_out /* HOST */,
                   void *stream);

/* HOST ONLY.  Bytes of device workspace fem_p2_assemble needs (32 nme). */
int fem_p2_assemble_workspace(int32_t nme, size_t *bytes /* HOST */);

/* P2 mass (FEM_OP_MASS: int phi_a phi_b) and / or stiffness (FEM_OP_STIFF:
 * int grad phi_a . grad phi_b) on the pattern of fem_p2_pattern, with the
 * basis phi_a = lambda_a (2 lambda_a - 1), phi_{3+a} = 4 lambda_b lambda_c
 * (the edge opposite vertex a), summed over the elements as sparse() does
 * (Section 6).  Four numbers per triangle (|T| / 180 and the three P1
 * off-diagonal stiffness entries / 3), then one lane per DOF row adds its
 * triangles' entries, each an integer combination of those numbers, in
 * ascending triangle order (bitwise reproducible).
 *   q [nq][2] f64 (16-byte aligned); me [nme][3] int32 as validated by
 *   fem_p2_dofs; row_ptr, inc_ptr, inc, inc_pos from fem_p2_pattern over
 *   ndof DOFs; vals_M / vals_S [nnz] device, caller-owned
 *   work [work_bytes] >= fem_p2_assemble_workspace(nme), 32-byte aligned
 * flags: 0 or FEM_ACCUMULATE. */
int fem_p2_assemble(int ops, int32_t nq, int32_t nme, int32_t ndof, int64_t nnz, const double *q,
                    const int32_t *me, const int32_t *row_ptr, const int32_t *inc_ptr,
                    const int32_t *inc, const uint64_t *inc_pos, double *vals_M, double *vals_S,
                    void *work, size_t work_bytes, int flags, void *stream);

/* ------------------------------------------------------------------------ */
/* Adjoint                                                                   */
/* ------------------------------------------------------------------------ */

/* HOST ONLY.  Bytes of device workspace for fem_adjoint_stiff_wmass:
 * packed (x, y, w) vertex records (32 nq) and the per-entry partial
 * derivatives (32 nnz). */
int fem_adjoint_workspace(int32_t nq, int64_t nnz, size_t *bytes /* HOST */);

/* Gradient of L = sum_ij GS_ij S_ij(q) + sum_ij GM_ij Mw_ij(q, w) with
 * respect to q and w (GS, GM [nnz] on the scalar pattern; either may be NULL
 * to drop its term; w may be NULL only if GM is).  dq [nq][2] and dw [nq]
 * are overwritten (FEM_ACCUMULATE adds into them).  tpos: the map that
 * fem_transpose_map wrote for this pattern (the partial derivatives are then
 * stored at the transposed places, which it must name), or NULL (then
 * found by search).  Patterns of fem_pattern are symmetric, so their map
 * has no -1; an entry whose map is -1 (no transposed entry) has no place
 * and its partial derivative is dropped, never stored out of bounds.  fan:
 * the codes of fem_fan_plan for this pattern, or NULL (the order of
 * additions follows them as in the forward calls).  flags: FEM_ACCUMULATE,
 * FEM_PACKED_QW.  Deterministic: two passes over the rows, no atomics; the
 * result does not depend on tpos, FEM_PACKED_QW or the launch shape. */
int fem_adjoint_stiff_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                            const double *w, const int32_t *row_ptr, const int32_t *col_idx,
                            const int32_t *inc_ptr, const uint32_t *inc_pos, const uint64_t *fan,
                            const int32_t *tpos, const double *GS, const double *GM, double *dq,
                            double *dw, void *work, size_t work_bytes, int flags, void *stream);

/* HOST ONLY.  Bytes of device workspace for fem_adjoint_elas: per-row
 * partial sums (at most 16 nq) and per-entry partial derivatives (16 nnz). */
int fem_adjoint_elas_workspace(int32_t nq, int64_t nnz, size_t *bytes /* HOST */);

/* Gradient of L = sum_e G_e K_e(q; lambda, mu) with respect to q and the
 * Lame parameters (K the elasticity matrix of fem_assemble_elas, G [4 nnz]
 * in its interleaved 2x2-block layout).
 *   dq [nq][2] (overwritten, or added to with FEM_ACCUMULATE)
 *   dlm [2] device or NULL: (dL/dlambda, dL/dmu), likewise
 * Pattern arrays (and fan codes, or NULL) as for fem_assemble
 * (FEM_DETERMINISTIC); tpos: the map that fem_transpose_map wrote for this
 * pattern, or NULL (search), as for fem_adjoint_stiff_wmass.  Two passes over
 * the rows plus a fixed-order reduction; no atomics, bitwise reproducible. */
int fem_adjoint_elas(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                     const int32_t *row_ptr, const int32_t *col_idx, const int32_t *inc_ptr,
                     const uint32_t *inc_pos, const uint64_t *fan, const int32_t *tpos,
                     double lambda, double mu, const double *G, double *dq, double *dlm, void *work,
                     size_t work_bytes, int flags, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FEM_P1_H */
