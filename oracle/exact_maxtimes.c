/*
 * Oracle (test infrastructure only): the exact (max, x) matrix product of
 * Alg. 2 (Sec. 2.2 of Serang, arXiv 1511.05690) in FP64,
 *     R[i][j] = max_k A[i][k] * B[k][j],   R starting at 0.
 *
 * Plain loops, parallel over rows with OpenMP.  For each (i, j) the products
 * are visited in ascending k as in Alg. 2; the j loop is placed innermost only
 * so that B is read along its rows.  max is exact, so the result is the same
 * number Alg. 2 produces in any visiting order.
 *
 * A: m x k row-major, B: k x n row-major, R: m x n row-major (FP64).
 * `rows` (nullable) selects which rows of A to use: R row t is row rows[t].
 */
#include <stdint.h>

void oracle_exact_maxtimes_f64(const double* A, const double* B, double* R,
                               int64_t m, int64_t k, int64_t n,
                               const int64_t* rows) {
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < m; ++t) {
        const int64_t i = rows ? rows[t] : t;
        double* Ri = R + t * n;
        for (int64_t j = 0; j < n; ++j) Ri[j] = 0.0;
        for (int64_t kk = 0; kk < k; ++kk) {
            const double a = A[i * k + kk];
            const double* Bk = B + kk * n;
            for (int64_t j = 0; j < n; ++j) {
                const double v = a * Bk[j];
                Ri[j] = v > Ri[j] ? v : Ri[j];
            }
        }
    }
}

/* Same definition with FP32 storage of A and B (each product is formed in
 * FP64 from the exactly converted operands). */
void oracle_exact_maxtimes_f32in(const float* A, const float* B, double* R,
                                 int64_t m, int64_t k, int64_t n,
                                 const int64_t* rows) {
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < m; ++t) {
        const int64_t i = rows ? rows[t] : t;
        double* Ri = R + t * n;
        for (int64_t j = 0; j < n; ++j) Ri[j] = 0.0;
        for (int64_t kk = 0; kk < k; ++kk) {
            const double a = (double)A[i * k + kk];
            const float* Bk = B + kk * n;
            for (int64_t j = 0; j < n; ++j) {
                const double v = a * (double)Bk[j];
                Ri[j] = v > Ri[j] ? v : Ri[j];
            }
        }
    }
}
