/* cpu_rows_omp.c -- CPU BASELINE ONLY (the all-cores leg of the benchmark's
 * CPU baseline); test infrastructure like the rest of oracle/, and not the
 * oracle itself.
 *
 * The numeric phase of the P1 stiffness and mass matrices on every host
 * core, given the CSR pattern and the triangle lists that the oracle built
 * (oracle_csr_pattern): an OpenMP loop over the rows; each row visits its
 * triangles in ascending order and adds the row of each element matrix at
 * the columns' places in the row, so no two threads write the same value.
 * Element terms from the paper's closed forms: with the triangle's vertices
 * taken in its own cyclic order starting at the row's vertex (x0, x1, x2),
 * r_a = x_{a+1} - x_{a+2}, |T| = |det(x1 - x0, x2 - x0)| / 2,
 *   S_0b = <r_0, r_b> / (4 |T|)                    (eq. StiffMatElem)
 *   M_00 = |T| / 6,  M_0b = |T| / 12 (b != 0)       (eq. MassElem)
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int cpu_rows_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void cpu_rows_stiff_mass(int32_t nq, const double *q, const int32_t *me, const int32_t *row_ptr,
                         const int32_t *col_idx, const int32_t *inc_ptr, const int32_t *inc,
                         double *S, double *M) {
#pragma omp parallel for schedule(static, 1024)
    for (int32_t i = 0; i < nq; ++i) {
        const int32_t rs = row_ptr[i], re = row_ptr[i + 1];
        for (int32_t p = rs; p < re; ++p) S[p] = M[p] = 0.0;
        for (int32_t t = inc_ptr[i]; t < inc_ptr[i + 1]; ++t) {
            const int32_t k = inc[t] / 3, a = inc[t] % 3;
            int32_t v[3];
            double x[3], y[3];
            for (int b = 0; b < 3; ++b) {
                v[b] = me[3 * (int64_t)k + (a + b) % 3];
                x[b] = q[2 * (int64_t)v[b]];
                y[b] = q[2 * (int64_t)v[b] + 1];
            }
            double rx[3], ry[3];
            for (int b = 0; b < 3; ++b) {
                rx[b] = x[(b + 1) % 3] - x[(b + 2) % 3];
                ry[b] = y[(b + 1) % 3] - y[(b + 2) % 3];
            }
            const double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
            const double area = fabs(det) / 2.0;
            for (int b = 0; b < 3; ++b) {
                int32_t p = rs;
                while (p < re - 1 && col_idx[p] != v[b]) ++p;
                S[p] += (rx[0] * rx[b] + ry[0] * ry[b]) / (4.0 * area);
                M[p] += b == 0 ? area / 6.0 : area / 12.0;
            }
        }
    }
}
