/*
 * First-arrival traveltime generator on a boundary-conforming logical grid.
 *
 * This is an input generator, not part of the transport method: it produces
 * the converged background traveltime T that the frozen tangent transport is
 * built from (the nonlinear state of Section 2.1, eq. (eikonal) written in
 * logical coordinates as eq. (metric-eikonal): grad_xi T^T G grad_xi T = s^2).
 * The paper computes this state with a cited factored solver; any first-arrival
 * solver serves to generate synthetic inputs, so this file uses a fast-marching
 * scheme with metric-aware simplex updates.
 *
 * Simplex update.  Around node p the accepted face neighbours give, per
 * logical axis d, a value t_d and a side sigma_d (+1: neighbour at p-e_d,
 * -1: neighbour at p+e_d), so that the one-sided derivative is
 * g_d = sigma_d (T - t_d).  For a subset S of axes the gradient components off
 * S are free; minimising grad^T G grad over them leaves the Schur complement
 * M_S = ((G^{-1})_{SS})^{-1}, where G^{-1} = J^T J is the covariant metric.
 * The update solves g_S^T M_S g_S = s^2 for T and accepts it when the
 * characteristic M_S g_S enters p from the neighbour side on every axis of S.
 * A one-axis update reduces to T = t_d + s * |edge|, so one is always valid.
 *
 * Point source: nodes within an index box of the source are initialised with
 * the straight-ray time (mean of the two end slownesses times the distance),
 * which is the usual treatment of the point-source singularity.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (see the workloads package).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double *key;
    int32_t *heap;
    int32_t *pos; /* position of a node in heap, -1 if absent */
    int32_t n;
} heap_t;

static void heap_swap(heap_t *h, int32_t a, int32_t b) {
    int32_t na = h->heap[a], nb = h->heap[b];
    h->heap[a] = nb; h->heap[b] = na;
    h->pos[nb] = a; h->pos[na] = b;
}

static void heap_up(heap_t *h, int32_t i) {
    while (i > 0) {
        int32_t p = (i - 1) >> 1;
        if (h->key[h->heap[p]] <= h->key[h->heap[i]]) break;
        heap_swap(h, i, p);
        i = p;
    }
}

static void heap_down(heap_t *h, int32_t i) {
    for (;;) {
        int32_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h->key[h->heap[l]] < h->key[h->heap[m]]) m = l;
        if (r < h->n && h->key[h->heap[r]] < h->key[h->heap[m]]) m = r;
        if (m == i) break;
        heap_swap(h, i, m);
        i = m;
    }
}

static void heap_push_or_decrease(heap_t *h, int32_t node) {
    if (h->pos[node] < 0) {
        h->heap[h->n] = node;
        h->pos[node] = h->n;
        h->n++;
        heap_up(h, h->n - 1);
    } else {
        heap_up(h, h->pos[node]);
    }
}

static int32_t heap_pop(heap_t *h) {
    int32_t top = h->heap[0];
    h->n--;
    if (h->n > 0) {
        h->heap[0] = h->heap[h->n];
        h->pos[h->heap[0]] = 0;
        heap_down(h, 0);
    }
    h->pos[top] = -1;
    return top;
}

/* full symmetric 3x3 (or 2x2 embedded) metric of node p, as m[3][3] */
static void load_metric(int dim, const double *G, int64_t p, double m[3][3]) {
    memset(m, 0, 9 * sizeof(double));
    if (dim == 3) {
        const double *g = G + 6 * p;
        m[0][0] = g[0]; m[1][1] = g[1]; m[2][2] = g[2];
        m[0][1] = m[1][0] = g[3];
        m[0][2] = m[2][0] = g[4];
        m[1][2] = m[2][1] = g[5];
    } else {
        const double *g = G + 3 * p;
        m[0][0] = g[0]; m[1][1] = g[1];
        m[0][1] = m[1][0] = g[2];
    }
}

/* inverse of a symmetric k x k matrix (k <= 3) stored in a[3][3] */
static int inv_small(int k, double a[3][3], double out[3][3]) {
    if (k == 1) {
        if (a[0][0] == 0.0) return -1;
        out[0][0] = 1.0 / a[0][0];
        return 0;
    }
    if (k == 2) {
        double det = a[0][0] * a[1][1] - a[0][1] * a[1][0];
        if (det == 0.0) return -1;
        out[0][0] = a[1][1] / det; out[1][1] = a[0][0] / det;
        out[0][1] = -a[0][1] / det; out[1][0] = -a[1][0] / det;
        return 0;
    }
    double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    double c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
    if (det == 0.0) return -1;
    out[0][0] = c00 / det;
    out[1][0] = c01 / det;
    out[2][0] = c02 / det;
    out[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
    out[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
    out[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
    out[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
    out[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
    out[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
    return 0;
}

typedef struct {
    int dim;
    int64_t n[3];       /* nodes per logical axis (axis 0 fastest) */
    int64_t stride[3];
    const double *G;
    const double *s;
} grid_t;

static void node_coords(const grid_t *g, int64_t p, int64_t c[3]) {
    c[0] = p % g->n[0];
    int64_t r = p / g->n[0];
    if (g->dim == 3) {
        c[1] = r % g->n[1];
        c[2] = r / g->n[1];
    } else {
        c[1] = r;
        c[2] = 0;
    }
}

/* tentative arrival at node p from its accepted face neighbours */
static double local_update(const grid_t *g, int64_t p, const double *T, const uint8_t *known) {
    int64_t c[3];
    node_coords(g, p, c);
    double t[3];
    double sg[3];
    int ax[3];
    int na = 0;
    for (int d = 0; d < g->dim; d++) {
        double best = INFINITY;
        double side = 0.0;
        if (c[d] > 0) {
            int64_t q = p - g->stride[d];
            if (known[q] && T[q] < best) { best = T[q]; side = 1.0; }
        }
        if (c[d] + 1 < g->n[d]) {
            int64_t q = p + g->stride[d];
            if (known[q] && T[q] < best) { best = T[q]; side = -1.0; }
        }
        if (side != 0.0) { t[na] = best; sg[na] = side; ax[na] = d; na++; }
    }
    if (na == 0) return INFINITY;
    double Gm[3][3], cov[3][3];
    load_metric(g->dim, g->G, p, Gm);
    if (inv_small(g->dim, Gm, cov) != 0) return INFINITY;
    double sp = g->s[p];
    double best = INFINITY;
    for (int mask = 1; mask < (1 << na); mask++) {
        int idx[3], k = 0;
        for (int a = 0; a < na; a++)
            if (mask & (1 << a)) idx[k++] = a;
        double sub[3][3], M[3][3];
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) sub[a][b] = cov[ax[idx[a]]][ax[idx[b]]];
        if (inv_small(k, sub, M) != 0) continue;
        /* quadratic qa T^2 - 2 qb T + qc = 0 with M'_{ab} = M_{ab} sigma_a sigma_b */
        double qa = 0.0, qb = 0.0, qc = -sp * sp;
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) {
                double mab = M[a][b] * sg[idx[a]] * sg[idx[b]];
                qa += mab;
                qb += mab * t[idx[b]];
                qc += mab * t[idx[a]] * t[idx[b]];
            }
        if (qa <= 0.0) continue;
        double disc = qb * qb - qa * qc;
        if (disc < 0.0) continue;
        double Tn = (qb + sqrt(disc)) / qa;
        int ok = 1;
        for (int a = 0; a < k && ok; a++)
            if (Tn < t[idx[a]]) ok = 0;
        if (!ok) continue;
        if (k > 1) {
            for (int a = 0; a < k && ok; a++) {
                double comp = 0.0;
                for (int b = 0; b < k; b++) comp += M[a][b] * sg[idx[b]] * (Tn - t[idx[b]]);
                if (sg[idx[a]] * comp < 0.0) ok = 0;
            }
            if (!ok) continue;
        }
        if (Tn < best) best = Tn;
    }
    return best;
}

/* Off-grid point source at logical coordinates xi (dim values): the seed
 * region is every node within max-norm distance rho of xi, initialised with
 * the straight-ray time (s_src + s_p)/2 |x_p - x_src|, where s_src and x_src
 * are multilinear interpolations over the corners of xi's cell; the rest is
 * the same fast marching as for an on-grid source. */
static int solve_one_pt(const grid_t *g, const double *X, const double *xi, double rho, double *T);

static int solve_one(const grid_t *g, const double *X, int64_t src, int init_radius, double *T) {
    int64_t N = g->n[0] * g->n[1] * g->n[2];
    uint8_t *known = (uint8_t *)calloc((size_t)N, 1);
    uint8_t *frozen = (uint8_t *)calloc((size_t)N, 1);
    heap_t h;
    h.key = T;
    h.heap = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    h.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    h.n = 0;
    if (!known || !frozen || !h.heap || !h.pos) {
        free(known); free(frozen); free(h.heap); free(h.pos);
        return -2;
    }
    for (int64_t p = 0; p < N; p++) { T[p] = INFINITY; h.pos[p] = -1; }

    int64_t cs[3];
    node_coords(g, src, cs);
    int dim = g->dim;
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        if (d < dim) {
            lo[d] = cs[d] - init_radius < 0 ? 0 : cs[d] - init_radius;
            hi[d] = cs[d] + init_radius > g->n[d] - 1 ? g->n[d] - 1 : cs[d] + init_radius;
        } else {
            lo[d] = hi[d] = 0;
        }
    }
    const double *xs = X + (size_t)dim * src;
    for (int64_t k = lo[2]; k <= hi[2]; k++)
        for (int64_t j = lo[1]; j <= hi[1]; j++)
            for (int64_t i = lo[0]; i <= hi[0]; i++) {
                int64_t p = (dim == 3) ? i + g->n[0] * (j + g->n[1] * k) : i + g->n[0] * j;
                const double *xp = X + (size_t)dim * p;
                double r2 = 0.0;
                for (int d = 0; d < dim; d++) r2 += (xp[d] - xs[d]) * (xp[d] - xs[d]);
                T[p] = (p == src) ? 0.0 : 0.5 * (g->s[src] + g->s[p]) * sqrt(r2);
                frozen[p] = 1;
                heap_push_or_decrease(&h, (int32_t)p);
            }

    while (h.n > 0) {
        int32_t p = heap_pop(&h);
        known[p] = 1;
        int64_t c[3];
        node_coords(g, p, c);
        for (int d = 0; d < dim; d++) {
            for (int side = -1; side <= 1; side += 2) {
                int64_t cc = c[d] + side;
                if (cc < 0 || cc >= g->n[d]) continue;
                int64_t q = p + side * g->stride[d];
                if (known[q] || frozen[q]) continue;
                double tn = local_update(g, q, T, known);
                if (tn < T[q]) {
                    T[q] = tn;
                    heap_push_or_decrease(&h, (int32_t)q);
                }
            }
        }
    }
    free(known); free(frozen); free(h.heap); free(h.pos);
    return 0;
}

/*
 * Solve for nsrc sources in parallel.  G is [N][6] (3D: Gxx,Gyy,Gzz,Gxy,Gxz,Gyz)
 * or [N][3] (2D: Gxx,Gzz,Gxz) in logical index units; X is [N][dim] physical
 * node coordinates; s is [N] slowness; T is [nsrc][N] output.
 * Returns 0, or a negative code for bad arguments or allocation failure.
 */
int fmgen_eikonal(int dim, int64_t n1, int64_t n2, int64_t n3, const double *G, const double *X,
                  const double *s, int32_t nsrc, const int64_t *src, int32_t init_radius,
                  int32_t nthreads, double *T) {
    if (dim != 2 && dim != 3) return -1;
    grid_t g;
    g.dim = dim;
    g.n[0] = n1;
    if (dim == 3) { g.n[1] = n2; g.n[2] = n3; }
    else { g.n[1] = n3; g.n[2] = 1; }
    g.stride[0] = 1;
    g.stride[1] = g.n[0];
    g.stride[2] = g.n[0] * g.n[1];
    g.G = G;
    g.s = s;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    if (N <= 0 || N >= ((int64_t)1 << 31)) return -1;
    for (int32_t a = 0; a < nsrc; a++)
        if (src[a] < 0 || src[a] >= N) return -1;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1) reduction(min : rc)
    for (int32_t a = 0; a < nsrc; a++) {
        int r = solve_one(&g, X, src[a], init_radius, T + (size_t)a * (size_t)N);
        if (r < rc) rc = r;
    }
    return rc;
}

static int solve_one_pt(const grid_t *g, const double *X, const double *xi, double rho, double *T) {
    int64_t N = g->n[0] * g->n[1] * g->n[2];
    int dim = g->dim;
    uint8_t *known = (uint8_t *)calloc((size_t)N, 1);
    uint8_t *frozen = (uint8_t *)calloc((size_t)N, 1);
    heap_t h;
    h.key = T;
    h.heap = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    h.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    h.n = 0;
    if (!known || !frozen || !h.heap || !h.pos) {
        free(known); free(frozen); free(h.heap); free(h.pos);
        return -2;
    }
    for (int64_t p = 0; p < N; p++) { T[p] = INFINITY; h.pos[p] = -1; }
    /* the source cell and its multilinear weights */
    int64_t base[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int d = 0; d < dim; d++) {
        double f = floor(xi[d]);
        int64_t b = (int64_t)f;
        if (b > g->n[d] - 2) b = g->n[d] - 2;
        if (b < 0) b = 0;
        base[d] = b;
        t[d] = xi[d] - (double)b;
    }
    double s_src = 0.0, x_src[3] = {0, 0, 0};
    for (int corner = 0; corner < (1 << dim); corner++) {
        double w = 1.0;
        int64_t p = 0;
        for (int d = 0; d < dim; d++) {
            int up = (corner >> d) & 1;
            int64_t c = base[d] + (g->n[d] > 1 ? up : 0);
            w *= up ? t[d] : 1.0 - t[d];
            p += c * g->stride[d];
        }
        s_src += w * g->s[p];
        for (int d = 0; d < dim; d++) x_src[d] += w * X[(size_t)dim * p + d];
    }
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; d++) {
        lo[d] = (int64_t)ceil(xi[d] - rho);
        hi[d] = (int64_t)floor(xi[d] + rho);
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > g->n[d] - 1) hi[d] = g->n[d] - 1;
    }
    int nseed = 0;
    for (int64_t k = lo[2]; k <= hi[2]; k++)
        for (int64_t j = lo[1]; j <= hi[1]; j++)
            for (int64_t i = lo[0]; i <= hi[0]; i++) {
                int64_t p = i + g->stride[1] * j + g->stride[2] * k;
                const double *xp = X + (size_t)dim * p;
                double r2 = 0.0;
                for (int d = 0; d < dim; d++) r2 += (xp[d] - x_src[d]) * (xp[d] - x_src[d]);
                T[p] = 0.5 * (s_src + g->s[p]) * sqrt(r2);
                frozen[p] = 1;
                heap_push_or_decrease(&h, (int32_t)p);
                nseed++;
            }
    if (nseed == 0) {
        free(known); free(frozen); free(h.heap); free(h.pos);
        return -3;
    }
    while (h.n > 0) {
        int32_t p = heap_pop(&h);
        known[p] = 1;
        int64_t c[3];
        node_coords(g, p, c);
        for (int d = 0; d < dim; d++) {
            for (int side = -1; side <= 1; side += 2) {
                int64_t cc = c[d] + side;
                if (cc < 0 || cc >= g->n[d]) continue;
                int64_t q = p + side * g->stride[d];
                if (known[q] || frozen[q]) continue;
                double tn = local_update(g, q, T, known);
                if (tn < T[q]) {
                    T[q] = tn;
                    heap_push_or_decrease(&h, (int32_t)q);
                }
            }
        }
    }
    free(known); free(frozen); free(h.heap); free(h.pos);
    return 0;
}

/*
 * Off-grid point sources: xi is [nsrc][dim] logical source coordinates, rho
 * the seed radius (max-norm, logical units); otherwise as fmgen_eikonal.
 */
int fmgen_eikonal_pt(int dim, int64_t n1, int64_t n2, int64_t n3, const double *G, const double *X,
                     const double *s, int32_t nsrc, const double *xi, double rho, int32_t nthreads, double *T) {
    if (dim != 2 && dim != 3) return -1;
    grid_t g;
    g.dim = dim;
    g.n[0] = n1;
    if (dim == 3) { g.n[1] = n2; g.n[2] = n3; }
    else { g.n[1] = n3; g.n[2] = 1; }
    g.stride[0] = 1;
    g.stride[1] = g.n[0];
    g.stride[2] = g.n[0] * g.n[1];
    g.G = G;
    g.s = s;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    if (N <= 0 || N >= ((int64_t)1 << 31) || !(rho >= 0.0)) return -1;
    for (int32_t a = 0; a < nsrc; a++)
        for (int d = 0; d < dim; d++)
            if (!(xi[(size_t)a * dim + d] >= 0.0) || !(xi[(size_t)a * dim + d] <= (double)(g.n[d] - 1))) return -1;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1) reduction(min : rc)
    for (int32_t a = 0; a < nsrc; a++) {
        int r = solve_one_pt(&g, X, xi + (size_t)a * dim, rho, T + (size_t)a * (size_t)N);
        if (r < rc) rc = r;
    }
    return rc;
}
