/*
 * fem_oracle.c -- plain CPU oracle for P1 finite element assembly on 2D
 * triangle meshes (Cuvelier, Japhet, Scarella, "An efficient way to perform
 * the assembly of finite element matrices in Matlab and Octave", 2013).
 *
 * TEST INFRASTRUCTURE.  This file is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or table with the
 * HIP library and must never be called from the product path.
 *
 * What it computes, in the paper's terms:
 *   - element matrices: eqs. (MassElem), (MassWElem), (StiffMatElem) of the
 *     Notations section, and K^e = |T| B^T C B of the linear elasticity
 *     section (Hooke's law with Lame parameters lambda, mu);
 *   - assembly: the "optimized version 1" shape of Section 5 -- one loop over
 *     the triangles in ascending order emitting triplets (I, J, K) with the
 *     element matrix stored column-wise (local index r = 3 b + a for row a and
 *     column b; r = 6 jl + il for elasticity), followed by the semantics of
 *     Matlab's sparse(I, J, K, m, n): entries with equal (I, J) are summed.
 *     Structural zeros are KEPT (reading: the pattern depends on the topology
 *     only and is shared by all operators), unlike Matlab which drops them.
 *   - the compressed format is CSR (the paper's Section 4 describes CSC; the
 *     four matrices are symmetric, so CSR of A is CSC of A^T = A).
 *
 * Extensions named in the Conclusion, in the same OptV2 shape (triplets
 * t = r nme + k, then sparse()): P1 tetrahedra (mass, stiffness) and P2
 * triangles (mass, stiffness; edge degrees of freedom numbered in
 * lexicographic order of their vertex pairs, element matrices integrated
 * exactly in barycentric coordinates).  Also the adjoints (gradients with
 * respect to the vertex coordinates, the weight and the Lame parameters) of
 * the stiffness, weighted-mass and elasticity assemblies.
 *
 * Conventions: 0-based indices; q is [nq][2] (x0, y0, x1, y1, ...), me is
 * [nme][3]; triangle areas are computed here as |det| / 2 (the paper takes
 * them as an input).  Values of each entry are summed in ascending (k, r)
 * order, in double precision.  Build with -ffp-contract=off.
 *
 * Deliberately slow and simple: no blocking, fusion or reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-2)
#define ORACLE_EDEGEN (-3)
#define ORACLE_ENOSPC (-4)
#define ORACLE_ENOMEM (-7)

enum { OP_MASS = 0, OP_WMASS = 1, OP_STIFF = 2, OP_ELAS = 3 };

/* ------------------------------------------------------------------ */
/* Geometry                                                           */
/* ------------------------------------------------------------------ */

/* Signed determinant of the triangle (q1, q2, q3): (q2-q1) x (q3-q1). */
double oracle_det(const double *q1, const double *q2, const double *q3)
{
    return (q2[0] - q1[0]) * (q3[1] - q1[1]) - (q3[0] - q1[0]) * (q2[1] - q1[1]);
}

/* |T| = |det| / 2. */
double oracle_area(const double *q1, const double *q2, const double *q3)
{
    return fabs(oracle_det(q1, q2, q3)) / 2.0;
}

/* ------------------------------------------------------------------ */
/* Element matrices (stored column-wise: E[3*b + a] = E_{a,b})        */
/* ------------------------------------------------------------------ */

/* eq. (MassElem): |T|/12 [2 1 1; 1 2 1; 1 1 2]. */
void oracle_elem_mass(double area, double E[9])
{
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a)
            E[3 * b + a] = (area / 12.0) * (a == b ? 2.0 : 1.0);
}

/* eq. (MassWElem): |T|/30 times
 *   [3w1+w2+w3      w1+w2+w3/2     w1+w2/2+w3
 *    w1+w2+w3/2     w1+3w2+w3      w1/2+w2+w3
 *    w1+w2/2+w3     w1/2+w2+w3     w1+w2+3w3 ]                        */
void oracle_elem_wmass(double area, const double w[3], double E[9])
{
    const double w1 = w[0], w2 = w[1], w3 = w[2];
    double m[3][3];
    m[0][0] = 3.0 * w1 + w2 + w3;
    m[0][1] = w1 + w2 + w3 / 2.0;
    m[0][2] = w1 + w2 / 2.0 + w3;
    m[1][0] = w1 + w2 + w3 / 2.0;
    m[1][1] = w1 + 3.0 * w2 + w3;
    m[1][2] = w1 / 2.0 + w2 + w3;
    m[2][0] = w1 + w2 / 2.0 + w3;
    m[2][1] = w1 / 2.0 + w2 + w3;
    m[2][2] = w1 + w2 + 3.0 * w3;
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a)
            E[3 * b + a] = (area / 30.0) * m[a][b];
}

/* eq. (StiffMatElem): with u = q2-q3, v = q3-q1, w = q1-q2 (the edge vectors
 * opposite each vertex), E_{a,b} = <r_a, r_b> / (4 |T|), r = (u, v, w). */
void oracle_elem_stiff(const double *q1, const double *q2, const double *q3, double E[9])
{
    const double area = oracle_area(q1, q2, q3);
    double r[3][2];
    r[0][0] = q2[0] - q3[0]; r[0][1] = q2[1] - q3[1];   /* u */
    r[1][0] = q3[0] - q1[0]; r[1][1] = q3[1] - q1[1];   /* v */
    r[2][0] = q1[0] - q2[0]; r[2][1] = q1[1] - q2[1];   /* w */
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a)
            E[3 * b + a] = (r[a][0] * r[b][0] + r[a][1] * r[b][1]) / (4.0 * area);
}

/* Linear elasticity section: K^e = |T| B^T C B, with
 *   C = [lambda+2mu, lambda, 0; lambda, lambda+2mu, 0; 0, 0, mu]
 *   B = 1/(2|T|) [ u2   0  v2   0  w2   0
 *                   0 -u1   0 -v1   0 -w1
 *                 -u1  u2 -v1  v2 -w1  w2 ]
 * (columns: strains of the local basis psi_1..psi_6, interleaved x/y per
 * vertex).  Output column-wise: E[6*jl + il] = K^e_{il,jl}.
 * B carries the counter-clockwise gradient formula (eq. GradFoncBas); for a
 * clockwise triangle every column of B flips sign and K^e is unchanged.   */
void oracle_elem_elas(const double *q1, const double *q2, const double *q3,
                      double lam, double mu, double E[36])
{
    const double area = oracle_area(q1, q2, q3);
    const double u[2] = {q2[0] - q3[0], q2[1] - q3[1]};
    const double v[2] = {q3[0] - q1[0], q3[1] - q1[1]};
    const double w[2] = {q1[0] - q2[0], q1[1] - q2[1]};
    double B[3][6] = {
        {u[1], 0.0, v[1], 0.0, w[1], 0.0},
        {0.0, -u[0], 0.0, -v[0], 0.0, -w[0]},
        {-u[0], u[1], -v[0], v[1], -w[0], w[1]},
    };
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j)
            B[i][j] = B[i][j] / (2.0 * area);
    const double C[3][3] = {
        {lam + 2.0 * mu, lam, 0.0},
        {lam, lam + 2.0 * mu, 0.0},
        {0.0, 0.0, mu},
    };
    double CB[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l)
                s += C[i][l] * B[l][j];
            CB[i][j] = s;
        }
    for (int jl = 0; jl < 6; ++jl)
        for (int il = 0; il < 6; ++il) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l)
                s += B[l][il] * CB[l][jl];
            E[6 * jl + il] = area * s;
        }
}

/* ------------------------------------------------------------------ */
/* sparse(I, J, K): triplets -> CSR, duplicates summed                */
/* ------------------------------------------------------------------ */

/* Builds the CSR pattern of ntrip triplets (I[t], J[t]) over nrows rows:
 * a stable sort of the triplets by (row, col) (counting sort on the row,
 * then insertion sort on the column inside each row), unique -> col_idx,
 * counts -> row_ptr.  trip_pos[t] receives the CSR position of triplet t.
 * col_idx must hold ntrip entries.  Returns nnz, or a negative status.   */
int64_t oracle_csr_pattern(int32_t nrows, int32_t ncols, int64_t ntrip,
                           const int32_t *I, const int32_t *J,
                           int32_t *row_ptr, int32_t *col_idx, int64_t *trip_pos)
{
    if (nrows < 0 || ncols < 0 || ntrip < 0)
        return ORACLE_EINVAL;
    for (int64_t t = 0; t < ntrip; ++t)
        if (I[t] < 0 || I[t] >= nrows || J[t] < 0 || J[t] >= ncols)
            return ORACLE_ERANGE;
    int64_t *start = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    if (!start || !order) {
        free(start);
        free(order);
        return ORACLE_ENOMEM;
    }
    /* counting sort on the row, stable (ascending t within a row) */
    for (int64_t t = 0; t < ntrip; ++t)
        start[I[t] + 1] += 1;
    for (int32_t i = 0; i < nrows; ++i)
        start[i + 1] += start[i];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nrows + 1));
        if (!fill) {
            free(start);
            free(order);
            return ORACLE_ENOMEM;
        }
        memcpy(fill, start, sizeof(int64_t) * ((size_t)nrows + 1));
        for (int64_t t = 0; t < ntrip; ++t)
            order[fill[I[t]]++] = t;
        free(fill);
    }
    /* inside each row: stable insertion sort on the column */
    for (int32_t i = 0; i < nrows; ++i) {
        for (int64_t s = start[i] + 1; s < start[i + 1]; ++s) {
            int64_t t = order[s];
            int64_t p = s;
            while (p > start[i] && J[order[p - 1]] > J[t]) {
                order[p] = order[p - 1];
                --p;
            }
            order[p] = t;
        }
    }
    /* unique */
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int32_t i = 0; i < nrows; ++i) {
        for (int64_t s = start[i]; s < start[i + 1]; ++s) {
            int64_t t = order[s];
            if (s == start[i] || J[t] != J[order[s - 1]])
                col_idx[nnz++] = J[t];
            trip_pos[t] = nnz - 1;
        }
        if (nnz > INT32_MAX) {
            free(start);
            free(order);
            return ORACLE_ENOSPC;
        }
        row_ptr[i + 1] = (int32_t)nnz;
    }
    free(start);
    free(order);
    return nnz;
}

/* Matlab's A = sparse(I, J, V, nrows, ncols) (Section 5, "OptV1"), keeping
 * structural zeros: CSR pattern plus values summed in ascending t.        */
int64_t oracle_sparse(int32_t nrows, int32_t ncols, int64_t ntrip, const int32_t *I,
                      const int32_t *J, const double *V, int32_t *row_ptr,
                      int32_t *col_idx, double *values)
{
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    if (!pos)
        return ORACLE_ENOMEM;
    int64_t nnz = oracle_csr_pattern(nrows, ncols, ntrip, I, J, row_ptr, col_idx, pos);
    if (nnz >= 0) {
        for (int64_t p = 0; p < nnz; ++p)
            values[p] = 0.0;
        for (int64_t t = 0; t < ntrip; ++t)
            values[pos[t]] += V[t];
    }
    free(pos);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Mesh validation                                                    */
/* ------------------------------------------------------------------ */

/* Every vertex index in [0, nq) and the three vertices of each triangle
 * distinct.  Returns 0, ORACLE_ERANGE or ORACLE_EDEGEN.                   */
int oracle_validate(int32_t nq, int32_t nme, const int32_t *me)
{
    if (nq <= 0 || nme < 0)
        return ORACLE_EINVAL;
    int status = ORACLE_OK;
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 3 * k;
        for (int a = 0; a < 3; ++a)
            if (t[a] < 0 || t[a] >= nq)
                return ORACLE_ERANGE;
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2])
            status = ORACLE_EDEGEN;
    }
    return status;
}

/* ------------------------------------------------------------------ */
/* Symbolic assembly of a P1 mesh                                     */
/* ------------------------------------------------------------------ */

/* Global index arrays of Section 6 (Ig = me([1 2 3 1 2 3 1 2 3], :),
 * Jg = me([1 1 1 2 2 2 3 3 3], :)), compressed:
 *   row_ptr [nq+1], col_idx [cap >= 9 nme]: the CSR pattern;
 *   slot [9][nme]: slot[r*nme + k] = CSR position of local entry r = 3b + a
 *                  of triangle k (row me[k][a], column me[k][b]);
 *   inc_ptr [nq+1], inc [3 nme]: for each vertex v, the pairs 3k + a with
 *                  me[k][a] == v, in ascending k (the triangles around v).
 * Any of slot, inc_ptr/inc may be NULL.  Returns nnz or a negative status. */
int64_t oracle_pattern(int32_t nq, int32_t nme, const int32_t *me, int32_t *row_ptr,
                       int32_t *col_idx, int32_t *slot, int32_t *inc_ptr, int32_t *inc)
{
    int st = oracle_validate(nq, nme, me);
    if (st != ORACLE_OK)
        return st;
    const int64_t ntrip = 9 * (int64_t)nme;
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    int32_t *J = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    if (!I || !J || !pos) {
        free(I); free(J); free(pos);
        return ORACLE_ENOMEM;
    }
    for (int64_t k = 0; k < nme; ++k)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                I[9 * k + 3 * b + a] = me[3 * k + a];
                J[9 * k + 3 * b + a] = me[3 * k + b];
            }
    int64_t nnz = oracle_csr_pattern(nq, nq, ntrip, I, J, row_ptr, col_idx, pos);
    if (nnz >= 0 && slot)
        for (int64_t k = 0; k < nme; ++k)
            for (int r = 0; r < 9; ++r)
                slot[(int64_t)r * nme + k] = (int32_t)pos[9 * k + r];
    if (nnz >= 0 && inc_ptr && inc) {
        for (int32_t v = 0; v <= nq; ++v)
            inc_ptr[v] = 0;
        for (int64_t k = 0; k < nme; ++k)
            for (int a = 0; a < 3; ++a)
                inc_ptr[me[3 * k + a] + 1] += 1;
        for (int32_t v = 0; v < nq; ++v)
            inc_ptr[v + 1] += inc_ptr[v];
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
        if (!fill) {
            free(I); free(J); free(pos);
            return ORACLE_ENOMEM;
        }
        memcpy(fill, inc_ptr, sizeof(int32_t) * (size_t)nq);
        for (int64_t k = 0; k < nme; ++k)
            for (int a = 0; a < 3; ++a)
                inc[fill[me[3 * k + a]]++] = (int32_t)(3 * k + a);
        free(fill);
    }
    free(I); free(J); free(pos);
    return nnz;
}

/* Elasticity pattern over the 2 nq degrees of freedom psi_{2i} = (phi_i, 0),
 * psi_{2i+1} = (0, phi_i) (0-based form of the paper's interleaved basis):
 * the triplets of each triangle are (I_k(il), I_k(jl)) with
 * I_k = [2me1, 2me1+1, 2me2, 2me2+1, 2me3, 2me3+1], stored column-wise
 * (r = 6 jl + il), compressed exactly like the scalar case.
 * slot_e [36][nme] may be NULL.  Returns nnz or a negative status.        */
int64_t oracle_pattern_elas(int32_t nq, int32_t nme, const int32_t *me, int32_t *row_ptr,
                            int32_t *col_idx, int32_t *slot_e)
{
    int st = oracle_validate(nq, nme, me);
    if (st != ORACLE_OK)
        return st;
    if ((int64_t)nq * 2 > INT32_MAX)
        return ORACLE_EINVAL;
    const int64_t ntrip = 36 * (int64_t)nme;
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    int32_t *J = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    if (!I || !J || !pos) {
        free(I); free(J); free(pos);
        return ORACLE_ENOMEM;
    }
    for (int64_t k = 0; k < nme; ++k) {
        int32_t dof[6];
        for (int g = 0; g < 3; ++g) {
            dof[2 * g] = 2 * me[3 * k + g];
            dof[2 * g + 1] = 2 * me[3 * k + g] + 1;
        }
        for (int jl = 0; jl < 6; ++jl)
            for (int il = 0; il < 6; ++il) {
                I[36 * k + 6 * jl + il] = dof[il];
                J[36 * k + 6 * jl + il] = dof[jl];
            }
    }
    int64_t nnz = oracle_csr_pattern(2 * nq, 2 * nq, ntrip, I, J, row_ptr, col_idx, pos);
    if (nnz >= 0 && slot_e)
        for (int64_t k = 0; k < nme; ++k)
            for (int r = 0; r < 36; ++r)
                slot_e[(int64_t)r * nme + k] = (int32_t)pos[36 * k + r];
    free(I); free(J); free(pos);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Numeric assembly                                                   */
/* ------------------------------------------------------------------ */

/* Element matrix of operator `op` for triangle k; returns the number of
 * local entries (9 or 36).                                                */
static int element(int op, const double *q, const int32_t *me, const double *w,
                   double lam, double mu, int64_t k, double *E)
{
    const int32_t *t = me + 3 * k;
    const double *q1 = q + 2 * (int64_t)t[0];
    const double *q2 = q + 2 * (int64_t)t[1];
    const double *q3 = q + 2 * (int64_t)t[2];
    switch (op) {
    case OP_MASS:
        oracle_elem_mass(oracle_area(q1, q2, q3), E);
        return 9;
    case OP_WMASS: {
        const double wl[3] = {w[t[0]], w[t[1]], w[t[2]]};
        oracle_elem_wmass(oracle_area(q1, q2, q3), wl, E);
        return 9;
    }
    case OP_STIFF:
        oracle_elem_stiff(q1, q2, q3, E);
        return 9;
    case OP_ELAS:
        oracle_elem_elas(q1, q2, q3, lam, mu, E);
        return 36;
    }
    return 0;
}

/* Values of operator op (mass, weighted mass, stiffness: slot [9][nme] from
 * oracle_pattern; elasticity: slot [36][nme] from oracle_pattern_elas):
 * loop over the triangles in ascending k and over the local entries in
 * ascending r, adding each into its CSR position.  w is the vertex weight
 * Tw (weighted mass only); lam, mu the Lame parameters (elasticity only). */
int oracle_assemble(int op, int32_t nq, int32_t nme, const double *q, const int32_t *me,
                    const double *w, double lam, double mu, const int32_t *slot,
                    int64_t nnz, double *values)
{
    if (op < OP_MASS || op > OP_ELAS || nq <= 0 || nme < 0 || !q || !me || !slot || !values)
        return ORACLE_EINVAL;
    if (op == OP_WMASS && !w)
        return ORACLE_EINVAL;
    if (op == OP_ELAS && !(lam + mu > 0.0))
        return ORACLE_EINVAL;
    for (int64_t p = 0; p < nnz; ++p)
        values[p] = 0.0;
    double E[36];
    for (int64_t k = 0; k < nme; ++k) {
        int nloc = element(op, q, me, w, lam, mu, k, E);
        for (int r = 0; r < nloc; ++r)
            values[slot[(int64_t)r * nme + k]] += E[r];
    }
    return ORACLE_OK;
}

/* Selected rows of operator op computed one by one, without the global
 * pattern: for each requested row, every triangle touching it contributes in
 * ascending k, so each value is summed in exactly the order of
 * oracle_assemble.  Rows are vertex indices (scalar operators) or degree-of-
 * freedom indices 2v + alpha (elasticity).  Output: out_ptr [nrows+1],
 * out_cols / out_vals [cap], each row sorted by column.  Returns the total
 * number of entries, or a negative status.                                */
int64_t oracle_rows(int op, int32_t nq, int32_t nme, const double *q, const int32_t *me,
                    const double *w, double lam, double mu, int32_t nrows,
                    const int32_t *rows, int32_t *out_ptr, int32_t *out_cols,
                    double *out_vals, int64_t cap)
{
    if (op < OP_MASS || op > OP_ELAS || nq <= 0 || nme < 0 || nrows < 0)
        return ORACLE_EINVAL;
    const int dofs = (op == OP_ELAS) ? 2 : 1;
    const int nl = 3 * dofs;
    const int64_t ndof = (int64_t)dofs * nq;
    int st = oracle_validate(nq, nme, me);
    if (st != ORACLE_OK)
        return st;
    int32_t *which = (int32_t *)malloc(sizeof(int32_t) * (size_t)ndof);
    int32_t *len = (int32_t *)calloc((size_t)nrows + 1, sizeof(int32_t));
    int64_t *roff = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    int32_t *deg = (int32_t *)calloc((size_t)nq, sizeof(int32_t));
    if (!which || !len || !roff || !deg) {
        free(which); free(len); free(roff); free(deg);
        return ORACLE_ENOMEM;
    }
    /* a row of vertex v holds at most dofs * (1 + 2 deg(v)) entries */
    for (int64_t k = 0; k < 3 * (int64_t)nme; ++k)
        deg[me[k]] += 1;
    for (int64_t i = 0; i < ndof; ++i)
        which[i] = -1;
    for (int32_t s = 0; s < nrows; ++s) {
        if (rows[s] < 0 || rows[s] >= ndof) {
            free(which); free(len); free(roff); free(deg);
            return ORACLE_ERANGE;
        }
        which[rows[s]] = s;   /* a repeated row keeps its last sample slot */
        roff[s + 1] = roff[s] + (int64_t)dofs * (1 + 2 * (int64_t)deg[rows[s] / dofs]);
    }
    free(deg);
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(roff[nrows] > 0 ? roff[nrows] : 1));
    double *vals = (double *)malloc(sizeof(double) * (size_t)(roff[nrows] > 0 ? roff[nrows] : 1));
    if (!cols || !vals) {
        free(which); free(len); free(roff); free(cols); free(vals);
        return ORACLE_ENOMEM;
    }
    int64_t status = 0;
    double E[36];
    for (int64_t k = 0; k < nme && status == 0; ++k) {
        int32_t dof[6];
        for (int g = 0; g < 3; ++g)
            for (int al = 0; al < dofs; ++al)
                dof[dofs * g + al] = dofs * me[3 * k + g] + al;
        int touched = 0;
        for (int il = 0; il < nl; ++il)
            if (which[dof[il]] >= 0)
                touched = 1;
        if (!touched)
            continue;
        element(op, q, me, w, lam, mu, k, E);
        for (int il = 0; il < nl && status == 0; ++il) {
            int32_t s = which[dof[il]];
            if (s < 0)
                continue;
            for (int jl = 0; jl < nl; ++jl) {
                int32_t c = dof[jl];
                int32_t *rc = cols + roff[s];
                double *rv = vals + roff[s];
                int32_t p = 0;
                while (p < len[s] && rc[p] != c)
                    ++p;
                if (p == len[s]) {
                    if (roff[s] + len[s] == roff[s + 1]) {
                        status = ORACLE_ENOSPC;
                        break;
                    }
                    rc[p] = c;
                    rv[p] = 0.0;
                    len[s] += 1;
                }
                rv[p] += E[nl * jl + il];
            }
        }
    }
    int64_t total = 0;
    if (status == 0) {
        out_ptr[0] = 0;
        for (int32_t s = 0; s < nrows; ++s) {
            int32_t src = which[rows[s]];     /* sample slot holding this row */
            int32_t *rc = cols + roff[src];
            double *rv = vals + roff[src];
            /* insertion sort of the row by column */
            for (int32_t a = 1; a < len[src]; ++a) {
                int32_t c = rc[a];
                double v = rv[a];
                int32_t b = a;
                while (b > 0 && rc[b - 1] > c) {
                    rc[b] = rc[b - 1];
                    rv[b] = rv[b - 1];
                    --b;
                }
                rc[b] = c;
                rv[b] = v;
            }
            if (total + len[src] > cap) {
                status = ORACLE_ENOSPC;
                break;
            }
            for (int32_t a = 0; a < len[src]; ++a) {
                out_cols[total + a] = rc[a];
                out_vals[total + a] = rv[a];
            }
            total += len[src];
            out_ptr[s + 1] = (int32_t)total;
        }
    }
    free(which); free(len); free(roff); free(cols); free(vals);
    return status != 0 ? status : total;
}

/* ------------------------------------------------------------------ */
/* Adjoint of L = <GS, S(q)> + <GM, Mw(q, w)>                         */
/* ------------------------------------------------------------------ */

/* Gradient of the scalar L = sum_ij GS_ij S_ij + sum_ij GM_ij Mw_ij with
 * respect to the vertex coordinates q and the vertex weights w, where S and
 * Mw are the assembled stiffness and weighted mass matrices on the pattern
 * described by slot [9][nme].  Derived by hand from the element formulas:
 *
 *   with D = (q2-q1) x (q3-q1), |T| = |D|/2, r = (q2-q3, q3-q1, q1-q2):
 *     d|D| / dq_c = sign(D) (r_c,y, -r_c,x)
 *   stiffness:  L_S = N / (2|D|),  N = sum_ab GS_ab <r_a, r_b>
 *     dN/dr_a = sum_b (GS_ab + GS_ba) r_b,
 *     dN/dq_1 = dN/dr_3 - dN/dr_2, dN/dq_2 = dN/dr_1 - dN/dr_3,
 *     dN/dq_3 = dN/dr_2 - dN/dr_1,
 *     dL_S/dq_c = dN/dq_c / (2|D|) - N / (2|D|^2) d|D|/dq_c
 *   weighted mass: L_M = |T|/30 sum_ab GM_ab P_ab(w), P from eq. (MassWElem)
 *     dL_M/dq_c = (sum_ab GM_ab P_ab) / 60 * d|D|/dq_c
 *     dL_M/dw_d = |T|/30 sum_ab GM_ab dP_ab/dw_d, with dP_aa/dw_d = 1 + 2[a=d]
 *     and, for a != b with third vertex c, dP_ab/dw_d = 1 - [d=c]/2.
 *
 * Contributions are added per vertex in ascending k.  dq is [nq][2], dw [nq];
 * both are overwritten.  GS or GM may be NULL (term omitted).              */
int oracle_adjoint_stiff_wmass(int32_t nq, int32_t nme, const double *q, const int32_t *me,
                               const double *w, const int32_t *slot, const double *GS,
                               const double *GM, double *dq, double *dw)
{
    if (nq <= 0 || nme < 0 || !q || !me || !slot || !dq || !dw || (GM && !w))
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < 2 * (int64_t)nq; ++i)
        dq[i] = 0.0;
    for (int64_t i = 0; i < nq; ++i)
        dw[i] = 0.0;
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 3 * k;
        const double *x[3] = {q + 2 * (int64_t)t[0], q + 2 * (int64_t)t[1],
                              q + 2 * (int64_t)t[2]};
        const double D = oracle_det(x[0], x[1], x[2]);
        const double absD = fabs(D);
        const double sgn = D > 0.0 ? 1.0 : (D < 0.0 ? -1.0 : 0.0);
        double r[3][2];
        for (int c = 0; c < 2; ++c) {
            r[0][c] = x[1][c] - x[2][c];
            r[1][c] = x[2][c] - x[0][c];
            r[2][c] = x[0][c] - x[1][c];
        }
        double dD[3][2];   /* d|D| / dq_c */
        for (int c = 0; c < 3; ++c) {
            dD[c][0] = sgn * r[c][1];
            dD[c][1] = -sgn * r[c][0];
        }
        double g[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        if (GS) {
            double G[3][3];
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a)
                    G[a][b] = GS[slot[(int64_t)(3 * b + a) * nme + k]];
            double N = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    N += G[a][b] * (r[a][0] * r[b][0] + r[a][1] * r[b][1]);
            double dNr[3][2];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 2; ++c) {
                    double s = 0.0;
                    for (int b = 0; b < 3; ++b)
                        s += (G[a][b] + G[b][a]) * r[b][c];
                    dNr[a][c] = s;
                }
            double dNq[3][2];
            for (int c = 0; c < 2; ++c) {
                dNq[0][c] = dNr[2][c] - dNr[1][c];
                dNq[1][c] = dNr[0][c] - dNr[2][c];
                dNq[2][c] = dNr[1][c] - dNr[0][c];
            }
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 2; ++c)
                    g[a][c] += dNq[a][c] / (2.0 * absD) - N / (2.0 * absD * absD) * dD[a][c];
        }
        if (GM) {
            const double wl[3] = {w[t[0]], w[t[1]], w[t[2]]};
            double P[9];
            oracle_elem_wmass(30.0, wl, P);   /* P_ab = E_ab with |T| = 30 */
            double GP = 0.0;
            double G[3][3];
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    G[a][b] = GM[slot[(int64_t)(3 * b + a) * nme + k]];
                    GP += G[a][b] * P[3 * b + a];
                }
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 2; ++c)
                    g[a][c] += GP / 60.0 * dD[a][c];
            const double area = absD / 2.0;
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double dP;
                        if (a == b)
                            dP = 1.0 + (a == d ? 2.0 : 0.0);
                        else
                            dP = (d == 3 - a - b) ? 0.5 : 1.0;
                        s += G[a][b] * dP;
                    }
                dw[t[d]] += area / 30.0 * s;
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 2; ++c)
                dq[2 * (int64_t)t[a] + c] += g[a][c];
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* P1 tetrahedra in 3D (the extension named in the Conclusion)        */
/* ------------------------------------------------------------------ */
/* q is [nq][3], me is [nme][4].  For the tetrahedron K = (x0, x1, x2, x3)
 * with J = [x1 - x0 | x2 - x0 | x3 - x0] (columns), |K| = |det J| / 6, the
 * barycentric coordinates are lambda_{1..3} = rows of J^{-1} applied to
 * (x - x0) and lambda_0 = 1 - their sum, so grad lambda_i is row i of J^{-1}
 * (i = 1..3) and grad lambda_0 = -(sum of those rows).                    */

/* det J = (x1 - x0) . ((x2 - x0) x (x3 - x0)) */
double oracle_tet_det(const double *x0, const double *x1, const double *x2, const double *x3)
{
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = x1[i] - x0[i];
        b[i] = x2[i] - x0[i];
        c[i] = x3[i] - x0[i];
    }
    const double bxc0 = b[1] * c[2] - b[2] * c[1];
    const double bxc1 = b[2] * c[0] - b[0] * c[2];
    const double bxc2 = b[0] * c[1] - b[1] * c[0];
    return a[0] * bxc0 + a[1] * bxc1 + a[2] * bxc2;
}

/* Mass: integral of lambda_a lambda_b = |K| (1 + delta_ab) / 20 (the 3D
 * counterpart of eq. MassElem).  E column-major, E[4 b + a]. */
void oracle_elem_tet_mass(double vol, double E[16])
{
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a)
            E[4 * b + a] = vol * (a == b ? 2.0 : 1.0) / 20.0;
}

/* Stiffness: |K| grad lambda_a . grad lambda_b, with J^{-1} = adj(J) / det J. */
void oracle_elem_tet_stiff(const double *x0, const double *x1, const double *x2,
                           const double *x3, double E[16])
{
    double J[3][3];   /* J[r][c]: component r of column c */
    for (int r = 0; r < 3; ++r) {
        J[r][0] = x1[r] - x0[r];
        J[r][1] = x2[r] - x0[r];
        J[r][2] = x3[r] - x0[r];
    }
    const double det = oracle_tet_det(x0, x1, x2, x3);
    /* inverse by the adjugate (cofactor transpose) */
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double g[4][3];
    for (int c = 0; c < 3; ++c) {
        g[1][c] = Ji[0][c];
        g[2][c] = Ji[1][c];
        g[3][c] = Ji[2][c];
        g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
    const double vol = fabs(det) / 6.0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a)
            E[4 * b + a] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
}

/* Global P1 tetrahedron matrices the OptV2 way: Ig, Jg, Kg of all 16 local
 * entries, triplet t = r nme + k for local entry r = 4 b + a of element k
 * (row me[k][a], column me[k][b]), then sparse() (values summed in ascending
 * t).  op: 0 mass, 1 stiffness.  col_idx / values hold 16 nme entries. */
int64_t oracle_assemble_tet(int op, int32_t nq, int32_t nme, const double *q, const int32_t *me,
                            int32_t *row_ptr, int32_t *col_idx, double *values)
{
    if (nq <= 0 || nme < 0 || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 4 * k;
        for (int a = 0; a < 4; ++a) {
            if (t[a] < 0 || t[a] >= nq)
                return ORACLE_ERANGE;
            for (int b = 0; b < a; ++b)
                if (t[a] == t[b])
                    return ORACLE_EDEGEN;
        }
    }
    const int64_t nt = 16 * (int64_t)nme;
    const size_t n = (size_t)(nt > 0 ? nt : 1);
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *Jv = (int32_t *)malloc(sizeof(int32_t) * n);
    double *V = (double *)malloc(sizeof(double) * n);
    if (!I || !Jv || !V) {
        free(I);
        free(Jv);
        free(V);
        return ORACLE_ENOMEM;
    }
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 4 * k;
        const double *x0 = q + 3 * (int64_t)t[0], *x1 = q + 3 * (int64_t)t[1];
        const double *x2 = q + 3 * (int64_t)t[2], *x3 = q + 3 * (int64_t)t[3];
        double E[16];
        if (op == 0)
            oracle_elem_tet_mass(fabs(oracle_tet_det(x0, x1, x2, x3)) / 6.0, E);
        else
            oracle_elem_tet_stiff(x0, x1, x2, x3, E);
        for (int r = 0; r < 16; ++r) {
            const int64_t s = (int64_t)r * nme + k;
            I[s] = t[r % 4];
            Jv[s] = t[r / 4];
            V[s] = E[r];
        }
    }
    const int64_t nnz = oracle_sparse(nq, nq, nt, I, Jv, V, row_ptr, col_idx, values);
    free(I);
    free(Jv);
    free(V);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Adjoint of the elasticity assembly                                 */
/* ------------------------------------------------------------------ */
/* Gradient of L = sum_ij G_ij K_ij(q; lambda, mu) over the elasticity
 * pattern (slot_e [36][nme] from oracle_pattern_elas).  dL/dq is obtained by
 * forward-mode differentiation (dual numbers over the six coordinates of a
 * triangle) of the very steps of oracle_elem_elas, so it needs no formula of
 * its own; K is linear in (lambda, mu), so dL/dlambda = <G, K(1, 0)> and
 * dL/dmu = <G, K(0, 1)>.  Contributions are added in ascending k.  dq is
 * [nq][2] and dlm [2] (dL/dlambda, dL/dmu); both are overwritten.          */

typedef struct {
    double v;
    double d[6];
} oracle_dual;

static oracle_dual dl_const(double v)
{
    oracle_dual r;
    r.v = v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = 0.0;
    return r;
}

static oracle_dual dl_add(oracle_dual a, oracle_dual b)
{
    oracle_dual r;
    r.v = a.v + b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] + b.d[i];
    return r;
}

static oracle_dual dl_sub(oracle_dual a, oracle_dual b)
{
    oracle_dual r;
    r.v = a.v - b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] - b.d[i];
    return r;
}

static oracle_dual dl_mul(oracle_dual a, oracle_dual b)
{
    oracle_dual r;
    r.v = a.v * b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}

static oracle_dual dl_div(oracle_dual a, oracle_dual b)
{
    oracle_dual r;
    r.v = a.v / b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}

static oracle_dual dl_abs(oracle_dual a)
{
    const double s = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
    oracle_dual r;
    r.v = fabs(a.v);
    for (int i = 0; i < 6; ++i)
        r.d[i] = s * a.d[i];
    return r;
}

/* the steps of oracle_elem_elas, on dual numbers */
static void dual_elem_elas(oracle_dual x[3][2], double lam, double mu, oracle_dual E[36])
{
    const oracle_dual D = dl_sub(dl_mul(dl_sub(x[1][0], x[0][0]), dl_sub(x[2][1], x[0][1])),
                                 dl_mul(dl_sub(x[2][0], x[0][0]), dl_sub(x[1][1], x[0][1])));
    const oracle_dual area = dl_div(dl_abs(D), dl_const(2.0));
    const oracle_dual zero = dl_const(0.0);
    oracle_dual u[2], v[2], w[2];
    for (int c = 0; c < 2; ++c) {
        u[c] = dl_sub(x[1][c], x[2][c]);
        v[c] = dl_sub(x[2][c], x[0][c]);
        w[c] = dl_sub(x[0][c], x[1][c]);
    }
    oracle_dual nu0 = dl_sub(zero, u[0]), nv0 = dl_sub(zero, v[0]), nw0 = dl_sub(zero, w[0]);
    oracle_dual B[3][6] = {
        {u[1], zero, v[1], zero, w[1], zero},
        {zero, nu0, zero, nv0, zero, nw0},
        {nu0, u[1], nv0, v[1], nw0, w[1]},
    };
    const oracle_dual two_area = dl_mul(dl_const(2.0), area);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j)
            B[i][j] = dl_div(B[i][j], two_area);
    const double C[3][3] = {
        {lam + 2.0 * mu, lam, 0.0},
        {lam, lam + 2.0 * mu, 0.0},
        {0.0, 0.0, mu},
    };
    oracle_dual CB[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j) {
            oracle_dual s = dl_const(0.0);
            for (int l = 0; l < 3; ++l)
                s = dl_add(s, dl_mul(dl_const(C[i][l]), B[l][j]));
            CB[i][j] = s;
        }
    for (int jl = 0; jl < 6; ++jl)
        for (int il = 0; il < 6; ++il) {
            oracle_dual s = dl_const(0.0);
            for (int l = 0; l < 3; ++l)
                s = dl_add(s, dl_mul(B[l][il], CB[l][jl]));
            E[6 * jl + il] = dl_mul(area, s);
        }
}

int oracle_adjoint_elas(int32_t nq, int32_t nme, const double *q, const int32_t *me,
                        const int32_t *slot_e, const double *G, double lam, double mu,
                        double *dq, double *dlm)
{
    if (nq <= 0 || nme < 0 || !q || !me || !slot_e || !G || !dq || !dlm)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < 2 * (int64_t)nq; ++i)
        dq[i] = 0.0;
    dlm[0] = dlm[1] = 0.0;
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 3 * k;
        oracle_dual x[3][2];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 2; ++c) {
                x[a][c] = dl_const(q[2 * (int64_t)t[a] + c]);
                x[a][c].d[2 * a + c] = 1.0;
            }
        oracle_dual E[36];
        dual_elem_elas(x, lam, mu, E);
        double El[36], Em[36];
        const double *x0 = q + 2 * (int64_t)t[0], *x1 = q + 2 * (int64_t)t[1];
        const double *x2 = q + 2 * (int64_t)t[2];
        oracle_elem_elas(x0, x1, x2, 1.0, 0.0, El);
        oracle_elem_elas(x0, x1, x2, 0.0, 1.0, Em);
        double dL[6] = {0, 0, 0, 0, 0, 0};
        for (int r = 0; r < 36; ++r) {
            const double g = G[slot_e[(int64_t)r * nme + k]];
            for (int i = 0; i < 6; ++i)
                dL[i] += g * E[r].d[i];
            dlm[0] += g * El[r];
            dlm[1] += g * Em[r];
        }
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 2; ++c)
                dq[2 * (int64_t)t[a] + c] += dL[2 * a + c];
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* P2 (quadratic) triangles (the P_k extension named in the Conclusion) */
/* ------------------------------------------------------------------ */
/* Degrees of freedom: the nq vertices, then the ne edges, edge e being
 * DOF nq + e; edges are numbered in ascending lexicographic order of
 * (lower vertex, higher vertex).  On the triangle (x0, x1, x2) the local
 * DOFs are the vertices 0, 1, 2 and then 3 + a = the edge opposite vertex a
 * (between the other two).  The basis, in barycentric coordinates, is
 *   phi_a = lambda_a (2 lambda_a - 1),  phi_{3+a} = 4 lambda_b lambda_c,
 * the Lagrange basis of the vertices and the edge midpoints.  Element
 * matrices are integrated exactly: each integrand is a polynomial in
 * (lambda_0, lambda_1, lambda_2) and
 *   int_T lambda_0^i lambda_1^j lambda_2^l = 2 |T| i! j! l! / (i + j + l + 2)!. */

#define BP_DEG 5   /* exponents 0..4 per coordinate */
typedef struct {
    double c[BP_DEG][BP_DEG][BP_DEG];   /* c[i][j][l]: coefficient of l0^i l1^j l2^l */
} bary_poly;

static void bp_basis_p2(int n, bary_poly *p)
{
    memset(p, 0, sizeof *p);
    if (n < 3) {
        int e2[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
        e2[n] = 2;
        e1[n] = 1;
        p->c[e2[0]][e2[1]][e2[2]] += 2.0;
        p->c[e1[0]][e1[1]][e1[2]] -= 1.0;
    } else {
        int e[3] = {1, 1, 1};
        e[n - 3] = 0;
        p->c[e[0]][e[1]][e[2]] += 4.0;
    }
}

static void bp_mul(const bary_poly *a, const bary_poly *b, bary_poly *o)
{
    memset(o, 0, sizeof *o);
    for (int i1 = 0; i1 < BP_DEG; ++i1)
        for (int j1 = 0; j1 < BP_DEG; ++j1)
            for (int l1 = 0; l1 < BP_DEG; ++l1) {
                const double ca = a->c[i1][j1][l1];
                if (ca == 0.0)
                    continue;
                for (int i2 = 0; i1 + i2 < BP_DEG; ++i2)
                    for (int j2 = 0; j1 + j2 < BP_DEG; ++j2)
                        for (int l2 = 0; l1 + l2 < BP_DEG; ++l2)
                            o->c[i1 + i2][j1 + j2][l1 + l2] += ca * b->c[i2][j2][l2];
            }
}

/* partial derivative with respect to lambda_m */
static void bp_diff(const bary_poly *a, int m, bary_poly *o)
{
    memset(o, 0, sizeof *o);
    for (int i = 0; i < BP_DEG; ++i)
        for (int j = 0; j < BP_DEG; ++j)
            for (int l = 0; l < BP_DEG; ++l) {
                const int e[3] = {i, j, l};
                if (e[m] == 0)
                    continue;
                int d[3] = {i, j, l};
                d[m] -= 1;
                o->c[d[0]][d[1]][d[2]] += e[m] * a->c[i][j][l];
            }
}

static double bp_integrate(const bary_poly *p, double area)
{
    static const double fact[13] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320, 362880,
                                    3628800, 39916800, 479001600};
    double s = 0.0;
    for (int i = 0; i < BP_DEG; ++i)
        for (int j = 0; j < BP_DEG; ++j)
            for (int l = 0; l < BP_DEG; ++l)
                if (p->c[i][j][l] != 0.0)
                    s += p->c[i][j][l] * fact[i] * fact[j] * fact[l] / fact[i + j + l + 2];
    return 2.0 * area * s;
}

/* Mass: E[6 b + a] = int_T phi_a phi_b. */
void oracle_elem_p2_mass(double area, double E[36])
{
    bary_poly pa, pb, prod;
    for (int b = 0; b < 6; ++b)
        for (int a = 0; a < 6; ++a) {
            bp_basis_p2(a, &pa);
            bp_basis_p2(b, &pb);
            bp_mul(&pa, &pb, &prod);
            E[6 * b + a] = bp_integrate(&prod, area);
        }
}

/* Stiffness: E[6 b + a] = int_T grad phi_a . grad phi_b, with
 * grad phi = sum_m (d phi / d lambda_m) grad lambda_m and grad lambda_1,
 * grad lambda_2 the rows of B^{-1}, B = [x1 - x0 | x2 - x0],
 * grad lambda_0 = -(grad lambda_1 + grad lambda_2). */
void oracle_elem_p2_stiff(const double *x0, const double *x1, const double *x2, double E[36])
{
    const double b00 = x1[0] - x0[0], b01 = x2[0] - x0[0];
    const double b10 = x1[1] - x0[1], b11 = x2[1] - x0[1];
    const double det = b00 * b11 - b01 * b10;
    double g[3][2];
    g[1][0] = b11 / det;
    g[1][1] = -b01 / det;
    g[2][0] = -b10 / det;
    g[2][1] = b00 / det;
    g[0][0] = -(g[1][0] + g[2][0]);
    g[0][1] = -(g[1][1] + g[2][1]);
    const double area = fabs(det) / 2.0;
    bary_poly pa, pb, da, db, prod;
    for (int b = 0; b < 6; ++b)
        for (int a = 0; a < 6; ++a) {
            bp_basis_p2(a, &pa);
            bp_basis_p2(b, &pb);
            double s = 0.0;
            for (int m = 0; m < 3; ++m)
                for (int n = 0; n < 3; ++n) {
                    bp_diff(&pa, m, &da);
                    bp_diff(&pb, n, &db);
                    bp_mul(&da, &db, &prod);
                    s += (g[m][0] * g[n][0] + g[m][1] * g[n][1]) * bp_integrate(&prod, area);
                }
            E[6 * b + a] = s;
        }
}

/* The P2 degrees of freedom of a triangle mesh: dofs [nme][6] (vertices,
 * then nq + the edge opposite local vertex 0, 1, 2) and edges [ne][2]
 * (lower, higher vertex; edges must hold 3 nme pairs).  The edge number is
 * the rank of its vertex pair among all distinct pairs in lexicographic
 * order.  Returns ne, or a negative status. */
int64_t oracle_p2_dofs(int32_t nq, int32_t nme, const int32_t *me, int32_t *dofs,
                       int32_t *edges)
{
    const int st = oracle_validate(nq, nme, me);
    if (st != ORACLE_OK)
        return st;
    const int64_t nt = 3 * (int64_t)nme;
    const size_t n = (size_t)(nt > 0 ? nt : 1);
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *Jv = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nq + 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t ne = ORACLE_ENOMEM;
    if (I && Jv && cols && rp && pos) {
        for (int64_t k = 0; k < nme; ++k)
            for (int a = 0; a < 3; ++a) {
                const int32_t u = me[3 * k + (a + 1) % 3], v = me[3 * k + (a + 2) % 3];
                I[a * nme + k] = u < v ? u : v;
                Jv[a * nme + k] = u < v ? v : u;
            }
        ne = oracle_csr_pattern(nq, nq, nt, I, Jv, rp, cols, pos);
        if (ne >= 0) {
            for (int64_t k = 0; k < nme; ++k)
                for (int a = 0; a < 3; ++a) {
                    dofs[6 * k + a] = me[3 * k + a];
                    dofs[6 * k + 3 + a] = (int32_t)(nq + pos[a * nme + k]);
                }
            for (int32_t i = 0; i < nq; ++i)
                for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                    edges[2 * (int64_t)e] = i;
                    edges[2 * (int64_t)e + 1] = cols[e];
                }
        }
    }
    free(I);
    free(Jv);
    free(cols);
    free(rp);
    free(pos);
    return ne;
}

/* Global P2 matrices the OptV2 way: Ig, Jg, Kg of all 36 local entries,
 * triplet t = r nme + k for local entry r = 6 b + a of element k (row
 * dofs[k][a], column dofs[k][b]), then sparse() (values summed in ascending
 * t).  op: 0 mass, 1 stiffness.  row_ptr [ndof + 1]; col_idx and values
 * hold 36 nme entries.  Returns nnz, or a negative status. */
int64_t oracle_assemble_p2(int op, int32_t ndof, int32_t nme, const double *q, const int32_t *me,
                           const int32_t *dofs, int32_t *row_ptr, int32_t *col_idx, double *values)
{
    if (ndof <= 0 || nme < 0 || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    const int64_t nt = 36 * (int64_t)nme;
    const size_t n = (size_t)(nt > 0 ? nt : 1);
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *Jv = (int32_t *)malloc(sizeof(int32_t) * n);
    double *V = (double *)malloc(sizeof(double) * n);
    if (!I || !Jv || !V) {
        free(I);
        free(Jv);
        free(V);
        return ORACLE_ENOMEM;
    }
    for (int64_t k = 0; k < nme; ++k) {
        const int32_t *t = me + 3 * k;
        const double *x0 = q + 2 * (int64_t)t[0], *x1 = q + 2 * (int64_t)t[1];
        const double *x2 = q + 2 * (int64_t)t[2];
        double E[36];
        if (op == 0)
            oracle_elem_p2_mass(oracle_area(x0, x1, x2), E);
        else
            oracle_elem_p2_stiff(x0, x1, x2, E);
        for (int r = 0; r < 36; ++r) {
            const int64_t s = (int64_t)r * nme + k;
            I[s] = dofs[6 * k + r % 6];
            Jv[s] = dofs[6 * k + r / 6];
            V[s] = E[r];
        }
    }
    const int64_t nnz = oracle_sparse(ndof, ndof, nt, I, Jv, V, row_ptr, col_idx, values);
    free(I);
    free(Jv);
    free(V);
    return nnz;
}
