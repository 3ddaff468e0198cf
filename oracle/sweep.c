/*
 * Oracle (test infrastructure only): Gauss-Seidel directional sweeping for
 * x = q + W x on a structured grid, Section 3.6 (repeated directional sweeping
 * as a stationary matrix splitting).  W is given explicitly in CSR form with
 * natural node order (row i lists w_ij for the dependencies j -> i); the
 * transpose problem passes the explicitly formed W^T.
 *
 * One cycle visits the 2^dim axis orderings: ordering o runs axis d backwards
 * when bit d of o is set, with loops k outer, j, i inner.  Each visit sets
 * x_p <- q_p + sum_j w_pj x_j using the newest values.  A solve stops when a
 * whole cycle changes no entry by more than tol_change * max|x| and the
 * residual ||q - (I - W) x||_2 / ||q||_2 <= tol_res, or after max_cycles.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double row_value(int64_t p, const int64_t *rowptr, const int32_t *col, const double *val,
                        const double *q, const double *x) {
    double acc = 0.0;
    for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) acc += val[e] * x[col[e]];
    return q[p] + acc;
}

static double residual_rel(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                           const double *q, const double *x) {
    double rr = 0.0, qq = 0.0;
    for (int64_t p = 0; p < N; p++) {
        double ax = x[p];
        for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) ax -= val[e] * x[col[e]];
        double r = q[p] - ax;
        rr += r * r;
        qq += q[p] * q[p];
    }
    if (qq == 0.0) return sqrt(rr);
    return sqrt(rr / qq);
}

/* returns cycles used (>0), or -cycles if max_cycles was reached unconverged */
static int gs_one(int dim, const int64_t n[3], const int64_t *rowptr, const int32_t *col,
                  const double *val, const double *q, double *x, int max_cycles, double tol_change,
                  double tol_res, double *xold) {
    int64_t N = n[0] * n[1] * n[2];
    int norders = 1 << dim;
    for (int64_t p = 0; p < N; p++) x[p] = 0.0;
    int cyc;
    for (cyc = 1; cyc <= max_cycles; cyc++) {
        memcpy(xold, x, sizeof(double) * (size_t)N);
        for (int o = 0; o < norders; o++) {
            int rev0 = o & 1, rev1 = (o >> 1) & 1, rev2 = (o >> 2) & 1;
            for (int64_t kk = 0; kk < n[2]; kk++) {
                int64_t k = rev2 ? n[2] - 1 - kk : kk;
                for (int64_t jj = 0; jj < n[1]; jj++) {
                    int64_t j = rev1 ? n[1] - 1 - jj : jj;
                    int64_t base = n[0] * (j + n[1] * k);
                    for (int64_t ii = 0; ii < n[0]; ii++) {
                        int64_t i = rev0 ? n[0] - 1 - ii : ii;
                        int64_t p = base + i;
                        x[p] = row_value(p, rowptr, col, val, q, x);
                    }
                }
            }
        }
        double xmax = 0.0, dmax = 0.0;
        for (int64_t p = 0; p < N; p++) {
            double a = fabs(x[p]);
            if (a > xmax) xmax = a;
            double d = fabs(x[p] - xold[p]);
            if (d > dmax) dmax = d;
        }
        if (dmax <= tol_change * xmax) {
            if (residual_rel(N, rowptr, col, val, q, x) <= tol_res) return cyc;
        }
    }
    return -max_cycles;
}

/*
 * Solve nrhs independent systems x_r = q_r + W x_r (q, x laid out [nrhs][N]).
 * dims: dim = 2 uses axes (n1, n3) with n2 = 1.  cycles[r] receives the cycle
 * count (negative when unconverged).  OpenMP runs one right-hand side per
 * thread.  Returns 0, or -1 on bad arguments, -2 on allocation failure.
 */
int oracle_gs_sweep(int dim, int64_t n1, int64_t n2, int64_t n3, const int64_t *rowptr,
                    const int32_t *col, const double *val, int32_t nrhs, const double *q, double *x,
                    int32_t max_cycles, double tol_change, double tol_res, int32_t nthreads,
                    int32_t *cycles) {
    if (dim != 2 && dim != 3) return -1;
    int64_t n[3];
    n[0] = n1;
    if (dim == 3) { n[1] = n2; n[2] = n3; }
    else { n[1] = n3; n[2] = 1; }
    int64_t N = n[0] * n[1] * n[2];
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(min : rc)
    {
        double *xold = (double *)malloc(sizeof(double) * (size_t)N);
        if (!xold) rc = -2;
#pragma omp for schedule(dynamic, 1)
        for (int32_t r = 0; r < nrhs; r++) {
            if (!xold) continue;
            cycles[r] = gs_one(dim, n, rowptr, col, val, q + (size_t)r * N, x + (size_t)r * N,
                               max_cycles, tol_change, tol_res, xold);
        }
        free(xold);
    }
    return rc;
}
