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

/*
 * The same product as algorithm standard_spmv of section 2.1 computes it on
 * every process r: local_spmv(A_on_process, v) into w, then
 * local_spmv(A_off_process, b_recv) accumulated into w.  Row i of block r
 * (rows [starts[r], starts[r+1])) adds, sequentially from 0, first the
 * products of its stored entries whose column lies in the same block, in
 * stored order, then the products of the other entries, in stored order.
 * b_recv holds copies of v, so the received value of column j is v[j].
 */
void spmv_split_ref_f64(int64_t n, const int64_t *rowptr, const int32_t *col,
                        const double *val, const double *v, double *w,
                        int64_t n_p, const int64_t *starts, int threads)
{
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_p; ++r) {
        const int64_t lo = starts[r], hi = starts[r + 1];
        for (int64_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                if (col[k] < lo || col[k] >= hi) continue;
                double prod = val[k] * v[col[k]];
                s = s + prod;
            }
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                if (col[k] >= lo && col[k] < hi) continue;
                double prod = val[k] * v[col[k]];
                s = s + prod;
            }
            w[i] = s;
        }
    }
}

/*
 * The same product as algorithm NAPSpMV of section 4.3 forms it on every
 * process r of node n = r / ppn: local_spmv(A_on_process, v) into w, then
 * local_spmv(A_on_node, b_{l->l}) accumulated into w, then
 * local_spmv(A_off_node, b) accumulated into w.  Row i of block r adds,
 * sequentially from 0: the products of its stored entries whose column lies
 * in block r, in stored order; then those whose column lies in another
 * block of node n (rows [starts[n ppn], starts[(n+1) ppn])), in stored
 * order; then the rest, in stored order.  Every buffer holds copies of v.
 */
void spmv_split3_ref_f64(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const double *val, const double *v, double *w,
                         int64_t n_p, const int64_t *starts, int64_t ppn, int threads)
{
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_p; ++r) {
        const int64_t lo = starts[r], hi = starts[r + 1];
        const int64_t node = r / ppn;
        const int64_t nlo = starts[node * ppn], nhi = starts[(node + 1) * ppn];
        for (int64_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int part = 0; part < 3; ++part) {
                for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                    const int32_t j = col[k];
                    const int own = j >= lo && j < hi;
                    const int on_node = !own && j >= nlo && j < nhi;
                    const int which = own ? 0 : (on_node ? 1 : 2);
                    if (which != part) continue;
                    double prod = val[k] * v[j];
                    s = s + prod;
                }
            }
            w[i] = s;
        }
    }
}

/*
 * The split-order products above for any partition, given as the owner of
 * every index (owner[i] = the process holding row i and v_i): row i of
 * process t = owner[i] adds, sequentially from 0, its entries with
 * owner[col] == t, then (parts == 3 only) those with owner[col] on t's node
 * (owner[col] / ppn == t / ppn), then the rest, each group in stored order.
 * parts == 2 is standard_spmv's order, parts == 3 NAPSpMV's.
 */
void spmv_split_owner_ref_f64(int64_t n, const int64_t *rowptr, const int32_t *col,
                              const double *val, const double *v, double *w,
                              const int32_t *owner, int64_t ppn, int parts, int threads)
{
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t t = owner[i];
        double s = 0.0;
        for (int part = 0; part < 3; ++part) {
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int32_t r = owner[col[k]];
                int which = 2;
                if (r == t) which = 0;
                else if (parts == 3 && r / ppn == t / ppn) which = 1;
                if (which != part) continue;
                double prod = val[k] * v[col[k]];
                s = s + prod;
            }
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
