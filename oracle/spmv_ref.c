/*
 * Plain float64 CSR sparse matrix-vector product, w = A v (section 1 of
 * Bienz, Gropp, Olson, "Node aware sparse matrix-vector multiplication").
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this library.
 *
 * Each row is summed sequentially in stored order, one multiply and one add
 * per stored entry (built with -ffp-contract=off, so no fused multiply-add),
 * which is the definition of the product written out.  Rows are independent,
 * so OpenMP splits them statically over threads without changing any result.
 */
#include <stdint.h>
#include <omp.h>

void spmv_ref_f64(int64_t n, const int64_t *rowptr, const int32_t *col,
                  const double *val, const double *v, double *w, int threads)
{
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            double prod = val[k] * v[col[k]];
            s = s + prod;
        }
        w[i] = s;
    }
}

/* Number of threads an OpenMP parallel region actually uses. */
int spmv_ref_threads(int threads)
{
    int used = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    return used;
}
