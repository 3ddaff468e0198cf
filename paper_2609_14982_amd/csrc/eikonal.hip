// First-arrival traveltimes on the GPU: the state of Section 2.1, T the
// viscosity solution of |grad_x T| = s with T = 0 at the source, computed for
// S sources at once before the tangent setup (Algorithm 1, Phase I).
//
// Discretisation (the paper only cites its factored solver): a monotone
// semi-Lagrangian update on the boundary-conforming grid.  Node i's stencil
// is its face neighbours (one logical step along each axis); its simplices
// are the neighbours, the segments joining neighbours on two different axes
// and, in 3-D, the triangles with one neighbour per axis.  The update is
//   T_i = min over simplices S, min over y in S, of T_S(y) + s_i |x_i - y|,
// T_S linear over S, x the physical node positions.  The inner minimum is
// convex in the barycentric coordinates: it is the least of the vertex
// values, the stationary points inside the segments, and the stationary
// points inside the triangles, all in closed form.  The update is monotone
// in the neighbour values, so from T = +inf off the seeds every iteration
// order decreases T to the same (largest) fixed point; here it is Jacobi
// iteration, T^{n+1} = min(T^n, F(T^n)), double-buffered, until an
// iteration changes nothing.
//
// Seeds: the nodes within max-norm logical distance rho of the source's
// logical coordinates xi keep the straight-ray time
// (s_src + s_p)/2 |x_p - x_src|, s_src and x_src multilinear over xi's cell
// (a source on a node is the case of integer xi).
//
// Work per iteration: a node is recomputed only when a neighbour changed in
// the previous iteration (one state byte per node and source: changed, seed);
// the others keep their value, which the buffer being written already holds
// unless the node changed in the previous iteration.  The per-iteration
// "anything changed" flags are read by the host once per chunk of iterations.  Built with
// -ffp-contract=off: every product and sum is rounded as written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fmbtf.h"
#include "internal.h"
#include "batch.h"

struct fm_eikonal {
    int dim = 3;
    int64_t n[3] = {1, 1, 1};
    int64_t N = 0;
    int32_t S = 0;                  // capacity in sources
    double* X = nullptr;            // device [N][dim]
    double* Tb = nullptr;           // device [S][N] second buffer
    uint8_t* st[2] = {nullptr, nullptr};   // device [S][N] node states
    double* xi = nullptr;           // device [S][3]
    unsigned* flags = nullptr;      // device [kChunk]
    unsigned* flags_h = nullptr;    // pinned host [kChunk]
    hipStream_t stream = nullptr;
    int device = -1;
};

namespace fm {

namespace {

constexpr int kChunk = 16;          // iterations between convergence checks
constexpr uint8_t kChanged = 1, kSeed = 2;

struct EikDims {
    int dim;
    int64_t n0, n1, n2, N;
};

__device__ __forceinline__ void logical(const EikDims& d, int64_t p, int64_t c[3]) {
    c[0] = p % d.n0;
    const int64_t r = p / d.n0;
    c[1] = r % d.n1;
    c[2] = r / d.n1;
}

__device__ __forceinline__ double dist(const double* a, const double* b, int dim) {
    double acc = 0.0;
    for (int k = 0; k < dim; ++k) {
        const double t = a[k] - b[k];
        acc = acc + t * t;
    }
    return sqrt(acc);
}

__device__ __forceinline__ double dot(const double* a, const double* b, int dim) {
    double acc = 0.0;
    for (int k = 0; k < dim; ++k) acc = acc + a[k] * b[k];
    return acc;
}

// Stationary point inside the segment [x1, x2] of t(y) + si |xi - y| (t
// linear, t1 at x1, t2 at x2), or +inf when there is none inside.  With
// e = x2 - x1, d0 = xi - x1, a = |e|^2, b = d0.e, delta = t2 - t1: the
// distance from xi to the segment's line is rperp, and at the stationary
// point |xi - y| = rperp / sqrt(1 - delta^2 / (a si^2)) and
// lambda = b/a - (|xi - y| / si) delta / a.
__device__ __forceinline__ double seg_inner(const double* xi, double si, const double* x1, double t1,
                                           const double* x2, double t2, int dim) {
    if (!(t1 < INFINITY) || !(t2 < INFINITY)) return INFINITY;
    double e[3], d0[3];
    for (int k = 0; k < dim; ++k) { e[k] = x2[k] - x1[k]; d0[k] = xi[k] - x1[k]; }
    const double a = dot(e, e, dim), b = dot(d0, e, dim), c = dot(d0, d0, dim);
    const double delta = t2 - t1;
    if (!(a * si * si > delta * delta)) return INFINITY;
    const double rperp2 = fmax(c - b * b / a, 0.0);
    const double rn = sqrt(rperp2) / sqrt(1.0 - delta * delta / (a * si * si));
    const double lam = b / a - (rn / si) * delta / a;
    if (!(lam > 0.0 && lam < 1.0)) return INFINITY;
    return t1 + lam * delta + si * rn;
}

// Stationary point inside the triangle (x1, x2, x3), or +inf.  With
// E = [x2 - x1, x3 - x1], Gm = E^T E, mu = Gm^{-1} E^T (xi - x1) (the
// projection of xi), delta = (t2 - t1, t3 - t1), q = delta^T Gm^{-1} delta:
// |xi - y| = rperp / sqrt(1 - q / si^2), lambda = mu - (|xi - y| / si) Gm^{-1} delta.
__device__ __forceinline__ double tri_inner(const double* xi, double si, const double* x1, double t1,
                                           const double* x2, double t2, const double* x3, double t3) {
    if (!(t1 < INFINITY) || !(t2 < INFINITY) || !(t3 < INFINITY)) return INFINITY;
    double e2[3], e3[3], d0[3];
    for (int k = 0; k < 3; ++k) { e2[k] = x2[k] - x1[k]; e3[k] = x3[k] - x1[k]; d0[k] = xi[k] - x1[k]; }
    const double g22 = dot(e2, e2, 3), g23 = dot(e2, e3, 3), g33 = dot(e3, e3, 3);
    const double h2 = dot(e2, d0, 3), h3 = dot(e3, d0, 3);
    const double det = g22 * g33 - g23 * g23;
    if (!(det > 0.0)) return INFINITY;
    const double mu2 = (g33 * h2 - g23 * h3) / det;
    const double mu3 = (g22 * h3 - g23 * h2) / det;
    const double rperp2 = fmax(dot(d0, d0, 3) - (mu2 * h2 + mu3 * h3), 0.0);
    const double d2 = t2 - t1, d3 = t3 - t1;
    const double i2 = (g33 * d2 - g23 * d3) / det;
    const double i3 = (g22 * d3 - g23 * d2) / det;
    const double q = d2 * i2 + d3 * i3;
    if (!(si * si > q)) return INFINITY;
    const double rn = sqrt(rperp2) / sqrt(1.0 - q / (si * si));
    const double l2 = mu2 - (rn / si) * i2;
    const double l3 = mu3 - (rn / si) * i3;
    if (!(l2 > 0.0 && l3 > 0.0 && l2 + l3 < 1.0)) return INFINITY;
    return t1 + l2 * d2 + l3 * d3 + si * rn;
}

// Seeds and +inf in both buffers (an iteration leaves a node's value in the
// buffer it writes untouched when that buffer already holds it): one thread
// per (source, node).
__global__ void k_eik_init(EikDims d, int32_t S, const double* __restrict__ X, const double* __restrict__ s,
                           const double* __restrict__ xi, double rho, double* __restrict__ T,
                           double* __restrict__ T2, uint8_t* __restrict__ st) {
    const int64_t total = (int64_t)S * d.N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t alpha = t / d.N, p = t - alpha * d.N;
        const double* xs = xi + alpha * 3;
        int64_t c[3];
        logical(d, p, c);
        bool seed = true;
        for (int k = 0; k < d.dim; ++k) seed = seed && fabs((double)c[k] - xs[k]) <= rho;
        if (!seed) {
            T[t] = INFINITY;
            T2[t] = INFINITY;
            st[t] = 0;
            continue;
        }
        // the source's cell: corners and multilinear weights
        const int64_t nn[3] = {d.n0, d.n1, d.n2};
        int64_t base[3] = {0, 0, 0};
        double fr[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < d.dim; ++k) {
            int64_t b = (int64_t)floor(xs[k]);
            b = b < 0 ? 0 : b;
            b = b > nn[k] - 2 ? (nn[k] - 2 < 0 ? 0 : nn[k] - 2) : b;
            base[k] = b;
            fr[k] = xs[k] - (double)b;
        }
        double s_src = 0.0, x_src[3] = {0.0, 0.0, 0.0};
        for (int corner = 0; corner < (1 << d.dim); ++corner) {
            double w = 1.0;
            int64_t q = 0, stride = 1;
            for (int k = 0; k < d.dim; ++k) {
                const int up = (corner >> k) & 1;
                w = w * (up ? fr[k] : 1.0 - fr[k]);
                q += (base[k] + (nn[k] > 1 ? up : 0)) * stride;
                stride *= nn[k];
            }
            s_src = s_src + w * s[q];
            for (int k = 0; k < d.dim; ++k) x_src[k] = x_src[k] + w * X[q * d.dim + k];
        }
        const double v = 0.5 * (s_src + s[p]) * dist(X + p * d.dim, x_src, d.dim);
        T[t] = v;
        T2[t] = v;
        st[t] = kSeed | kChanged;
    }
}

__global__ void k_clear_flags(unsigned* f) {
    if (threadIdx.x < kChunk) f[threadIdx.x] = 0u;
}

// One Jacobi iteration for every (source, node).
template <int DIM>
__global__ void k_eik_step(EikDims d, int32_t S, const double* __restrict__ X, const double* __restrict__ s,
                           const double* __restrict__ Told, double* __restrict__ Tnew,
                           const uint8_t* __restrict__ sold, uint8_t* __restrict__ snew, unsigned* flag) {
    const int64_t total = (int64_t)S * d.N;
    const int64_t stride[3] = {1, d.n0, d.n0 * d.n1};
    const int64_t nn[3] = {d.n0, d.n1, d.n2};
    int any = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t alpha = t / d.N, p = t - alpha * d.N;
        const int64_t row = alpha * d.N;
        const uint8_t me = sold[t];
        if (me & kSeed) {
            snew[t] = kSeed;
            continue;
        }
        int64_t c[3];
        logical(d, p, c);
        int64_t nb[DIM][2];
        bool act = false;
        for (int k = 0; k < DIM; ++k) {
            nb[k][0] = c[k] > 0 ? p - stride[k] : -1;
            nb[k][1] = c[k] < nn[k] - 1 ? p + stride[k] : -1;
            for (int side = 0; side < 2; ++side)
                if (nb[k][side] >= 0) act = act || (sold[row + nb[k][side]] & kChanged);
        }
        if (!act) {
            // T^{n+1} = T^n; the buffer written now holds T^{n-1}, which is
            // the same value unless the node changed in the last iteration
            if (me & kChanged) Tnew[t] = Told[t];
            snew[t] = 0;
            continue;
        }
        const double told = Told[t];
        double v = told;
        {
            const double si = s[p];
            double xi[3], xk[DIM][2][3], tk[DIM][2];
            for (int k = 0; k < DIM; ++k) xi[k] = X[p * DIM + k];
            double best = INFINITY;
            for (int k = 0; k < DIM; ++k)
                for (int side = 0; side < 2; ++side) {
                    const int64_t q = nb[k][side];
                    tk[k][side] = q >= 0 ? Told[row + q] : INFINITY;
                    for (int m = 0; m < DIM; ++m) xk[k][side][m] = q >= 0 ? X[q * DIM + m] : 0.0;
                    if (q >= 0) best = fmin(best, tk[k][side] + si * dist(xi, xk[k][side], DIM));
                }
            // a simplex whose vertex values are all >= best cannot lower it:
            // its interior values exceed its least vertex value
            for (int a = 0; a < DIM; ++a)
                for (int b = a + 1; b < DIM; ++b)
                    for (int sa = 0; sa < 2; ++sa)
                        for (int sb = 0; sb < 2; ++sb)
                            if (nb[a][sa] >= 0 && nb[b][sb] >= 0 && fmin(tk[a][sa], tk[b][sb]) < best)
                                best = fmin(best, seg_inner(xi, si, xk[a][sa], tk[a][sa], xk[b][sb], tk[b][sb], DIM));
            if constexpr (DIM == 3) {
                for (int s0 = 0; s0 < 2; ++s0)
                    for (int s1 = 0; s1 < 2; ++s1)
                        for (int s2 = 0; s2 < 2; ++s2)
                            if (nb[0][s0] >= 0 && nb[1][s1] >= 0 && nb[2][s2] >= 0 &&
                                fmin(fmin(tk[0][s0], tk[1][s1]), tk[2][s2]) < best)
                                best = fmin(best, tri_inner(xi, si, xk[0][s0], tk[0][s0], xk[1][s1], tk[1][s1],
                                                            xk[2][s2], tk[2][s2]));
            }
            v = fmin(told, best);
        }
        Tnew[t] = v;
        const bool ch = v != told;
        snew[t] = ch ? kChanged : 0;
        any |= ch ? 1 : 0;
    }
    if (__syncthreads_or(any) && threadIdx.x == 0) atomicOr(flag, 1u);
}

}  // namespace

}  // namespace fm

extern "C" {

int fm_eikonal_create(int32_t dim, int64_t n1, int64_t n2, int64_t n3, const double* X, int32_t max_sources,
                      void* hip_stream, fm_eikonal** out) {
    using namespace fm;
    clear_error();
    if (!out) { set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { set_error("dim must be 2 or 3, got %d", dim); return FM_EINVAL; }
    if (dim == 2 && n2 != 1) { set_error("2-D grids need n2 == 1"); return FM_EINVAL; }
    if (n1 < 1 || n2 < 1 || n3 < 1) { set_error("grid sizes must be >= 1"); return FM_EINVAL; }
    if (!X) { set_error("null node coordinates"); return FM_EINVAL; }
    if (max_sources < 1) { set_error("max_sources must be >= 1"); return FM_EINVAL; }
    const int64_t N = n1 * n2 * n3;
    if (N >= ((int64_t)1 << 31)) { set_error("grid too large: %lld nodes", (long long)N); return FM_EINVAL; }
    for (int64_t i = 0; i < N * dim; i++)
        if (!std::isfinite(X[i])) { set_error("node coordinate %lld is not finite", (long long)i); return FM_EINVAL; }
    fm_eikonal* e = new (std::nothrow) fm_eikonal();
    if (!e) { set_error("out of host memory"); return FM_ENOMEM; }
    e->dim = dim;
    e->n[0] = n1;
    e->n[1] = dim == 3 ? n2 : n3;
    e->n[2] = dim == 3 ? n3 : 1;
    e->N = N;
    e->S = max_sources;
    e->stream = (hipStream_t)hip_stream;
    hipError_t h = hipGetDevice(&e->device);
    const size_t nsn = (size_t)max_sources * (size_t)N;
    if (h == hipSuccess) h = hipMalloc(&e->X, sizeof(double) * (size_t)N * dim);
    if (h == hipSuccess) h = hipMalloc(&e->Tb, sizeof(double) * nsn);
    if (h == hipSuccess) h = hipMalloc(&e->st[0], nsn);
    if (h == hipSuccess) h = hipMalloc(&e->st[1], nsn);
    if (h == hipSuccess) h = hipMalloc(&e->xi, sizeof(double) * 3 * (size_t)max_sources);
    if (h == hipSuccess) h = hipMalloc(&e->flags, sizeof(unsigned) * kChunk);
    if (h == hipSuccess) h = hipHostMalloc((void**)&e->flags_h, sizeof(unsigned) * kChunk, hipHostMallocDefault);
    if (h == hipSuccess) h = hipMemcpy(e->X, X, sizeof(double) * (size_t)N * dim, hipMemcpyHostToDevice);
    if (h != hipSuccess) {
        set_error("first-arrival solver allocation failed: %s", hipGetErrorString(h));
        fm_eikonal_free(e);
        return h == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    *out = e;
    return FM_OK;
}

int fm_eikonal_set_stream(fm_eikonal* e, void* hip_stream) {
    fm::clear_error();
    if (!e) { fm::set_error("null solver"); return FM_EINVAL; }
    e->stream = (hipStream_t)hip_stream;
    return FM_OK;
}

int fm_eikonal_solve(fm_eikonal* e, const double* s, int32_t S, const double* xi_src, double seed_radius,
                     int32_t max_iter, double* T, int32_t* iterations) {
    using namespace fm;
    clear_error();
    if (iterations) *iterations = 0;
    if (!e || !s || !xi_src || !T) { set_error("null argument"); return FM_EINVAL; }
    if (S < 1 || S > e->S) { set_error("S = %d outside 1..%d (the solver's capacity)", S, e->S); return FM_EINVAL; }
    if (!(seed_radius >= 0.0) || !std::isfinite(seed_radius)) { set_error("seed radius must be finite and >= 0"); return FM_EINVAL; }
    if (max_iter < 1) { set_error("max_iter must be >= 1"); return FM_EINVAL; }
    if (((uintptr_t)s & 7u) || ((uintptr_t)T & 7u)) { set_error("device buffers must be 8-byte aligned"); return FM_EINVAL; }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != e->device) { set_error("solver lives on device %d (current device %d)", e->device, dev); return FM_ESTATE; }
    std::vector<double> xi((size_t)3 * S, 0.0);
    for (int32_t a = 0; a < S; a++) {
        for (int k = 0; k < e->dim; k++) {
            const double v = xi_src[(size_t)a * e->dim + k];
            if (!(v >= 0.0) || !(v <= (double)(e->n[k] - 1))) {
                set_error("source %d: coordinate %d (%g) outside [0, %lld]", a, k, v, (long long)(e->n[k] - 1));
                return FM_EINVAL;
            }
            // the seed region must hold a node along every axis
            const double lo = std::max(0.0, std::ceil(v - seed_radius));
            const double hi = std::min((double)(e->n[k] - 1), std::floor(v + seed_radius));
            if (lo > hi) {
                set_error("source %d: the seed region (radius %g) holds no node", a, seed_radius);
                return FM_EINVAL;
            }
            xi[(size_t)a * 3 + k] = v;
        }
    }
    hipStream_t st = e->stream;
    HIP_TRY(hipMemcpyAsync(e->xi, xi.data(), sizeof(double) * xi.size(), hipMemcpyHostToDevice, st));
    EikDims d{e->dim, e->n[0], e->n[1], e->n[2], e->N};
    const int64_t total = (int64_t)S * e->N;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
    double* buf[2] = {T, e->Tb};
    hipLaunchKernelGGL(k_eik_init, dim3(grid), dim3(256), 0, st, d, S, e->X, s, e->xi, seed_radius, buf[0], buf[1],
                       e->st[0]);
    HIP_TRY(hipGetLastError());
    int cur = 0;
    int32_t done = 0;
    while (done < max_iter) {
        const int n = std::min<int32_t>(kChunk, max_iter - done);
        hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, st, e->flags);
        for (int j = 0; j < n; j++) {
            if (e->dim == 3)
                hipLaunchKernelGGL(k_eik_step<3>, dim3(grid), dim3(256), 0, st, d, S, e->X, s, buf[cur], buf[cur ^ 1],
                                   e->st[cur], e->st[cur ^ 1], e->flags + j);
            else
                hipLaunchKernelGGL(k_eik_step<2>, dim3(grid), dim3(256), 0, st, d, S, e->X, s, buf[cur], buf[cur ^ 1],
                                   e->st[cur], e->st[cur ^ 1], e->flags + j);
            cur ^= 1;
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(e->flags_h, e->flags, sizeof(unsigned) * n, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int j = 0; j < n; j++) {
            if (!e->flags_h[j]) {
                // iteration done + j + 1 changed nothing; the later ones of the
                // chunk left the same values in the buffer now current
                if (iterations) *iterations = done + j + 1;
                if (cur != 0)
                    HIP_TRY(hipMemcpyAsync(T, e->Tb, sizeof(double) * (size_t)total, hipMemcpyDeviceToDevice, st));
                HIP_TRY(hipStreamSynchronize(st));
                return FM_OK;
            }
        }
        done += n;
    }
    if (iterations) *iterations = done;
    if (cur != 0) HIP_TRY(hipMemcpyAsync(T, e->Tb, sizeof(double) * (size_t)total, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    set_error("no fixed point within %d iterations (T holds the last iterate)", max_iter);
    return FM_ESTATE;
}

void fm_eikonal_free(fm_eikonal* e) {
    if (!e) return;
    if (e->X) (void)hipFree(e->X);
    if (e->Tb) (void)hipFree(e->Tb);
    if (e->st[0]) (void)hipFree(e->st[0]);
    if (e->st[1]) (void)hipFree(e->st[1]);
    if (e->xi) (void)hipFree(e->xi);
    if (e->flags) (void)hipFree(e->flags);
    if (e->flags_h) (void)hipHostFree(e->flags_h);
    delete e;
}

}  // extern "C"
