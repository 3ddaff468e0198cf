// LSQR inner loop over the paired actions (the Krylov least-squares solve of
// Algorithm 1, which calls J and J^T once per iteration at the same
// frozen state, Section 4.5).  The harness solves min ||J x - d|| column by
// column for the B right-hand sides of a batch: model-space vectors are
// [N][B] (one model block shared by all sources, FM_DS_BROADCAST), data-space
// vectors are [S][R][B] (receiver data of every source), so J maps model
// blocks to stacked receiver data and J^T sums over the sources (Section 4.4).
//
// Every per-column scalar lives on the device and every step is a kernel on
// the batch stream: no allocation, no synchronisation and no memset after
// creation, so a whole run of iterations can be captured once as a HIP graph
// and replayed.  Column norms are two-stage reductions with a fixed
// block-to-row assignment and a fixed summation order (deterministic).
//
// The recurrences are the standard LSQR ones (Paige and Saunders):
//   beta_1 u_1 = d, alpha_1 v_1 = J^T u_1, w_1 = v_1, x_0 = 0,
//   phibar_1 = beta_1, rhobar_1 = alpha_1; then per iteration
//   beta u = J v - alpha u;  alpha v = J^T u - beta v;
//   rho = sqrt(rhobar^2 + beta^2), c = rhobar/rho, s = beta/rho,
//   theta = s alpha, rhobar = -c alpha, phi = c phibar, phibar = s phibar,
//   x += (phi/rho) w,  w = v - (theta/rho) w.
//
// CGLS (Hestenes and Stiefel's conjugate gradients on the normal equations,
// in the least-squares form that never forms J^T J) is the inner solver of the
// Gauss-Newton step through the autograd wrapper; per column b:
//   x_0 = 0, r_0 = d, s_0 = J^T r_0, p_0 = s_0, gamma_0 = ||s_0||^2; then
//   q = J p, alpha = gamma / ||q||^2, x += alpha p, r -= alpha q,
//   s = J^T r, gamma' = ||s||^2, beta = gamma' / gamma, p = s + beta p.
// Same device-resident scalars, same capture rules as LSQR.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "batch.h"

namespace fm {

constexpr int kRedBlocks = 512;     // partial sums per column norm
constexpr int kRedThreads = 256;

// per-column scalars, [kScalars][B] doubles on the device
enum : int { sAlpha = 0, sBeta, sRhobar, sPhibar, sRho, sPhi, sTheta, sInvNorm, kScalars };
// CGLS per-column scalars, [kCgScalars][B]
enum : int { cGamma = 0, cQQ, cAlpha, cGnew, cBeta, cRR, kCgScalars };

// partial[blk][b] = sum over this block's rows of x[row][b]^2
template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_colsq_partial(const V* __restrict__ x, int64_t rows, int B,
                                                                double* __restrict__ partial) {
    __shared__ double red[kRedThreads];
    const int per = kRedThreads / B;           // rows per step (B <= 256)
    const int col = threadIdx.x % B;
    const int lr = threadIdx.x / B;
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = blockIdx.x * chunk;
    const int64_t r1 = min(rows, r0 + chunk);
    double acc = 0.0;
    if (lr < per)
        for (int64_t r = r0 + lr; r < r1; r += per) {
            const double v = (double)x[r * B + col];
            acc += v * v;
        }
    red[threadIdx.x] = (lr < per) ? acc : 0.0;
    __syncthreads();
    if (threadIdx.x < B) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += red[q * B + threadIdx.x];
        partial[(int64_t)blockIdx.x * B + threadIdx.x] = s;
    }
}

// norm[b] = sqrt(sum_blk partial[blk][b]) into scalars[slot]; inverse kept too
__global__ void k_colnorm_finalize(const double* __restrict__ partial, int nblk, int B, double* scal, int slot) {
    const int b = threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int q = 0; q < nblk; ++q) s += partial[(int64_t)q * B + b];
    const double n = sqrt(s);
    scal[slot * B + b] = n;
    scal[sInvNorm * B + b] = n > 0.0 ? 1.0 / n : 0.0;
}

// x[:, b] *= scal[sInvNorm][b]
template <typename V>
__global__ void k_scale_inv(V* __restrict__ x, int64_t rows, int B, const double* __restrict__ scal) {
    const int64_t n = rows * B;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = (V)((double)x[t] * scal[sInvNorm * B + (int)(t % B)]);
}

// y[:, b] = t[:, b] - scal[slot][b] * y[:, b]
template <typename V>
__global__ void k_sub_scaled(V* __restrict__ y, const V* __restrict__ t, int64_t rows, int B,
                             const double* __restrict__ scal, int slot) {
    const int64_t n = rows * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (V)((double)t[i] - scal[slot * B + (int)(i % B)] * (double)y[i]);
}

// start: phibar = beta, rhobar = alpha
__global__ void k_lsqr_start_scalars(double* scal, int B) {
    const int b = threadIdx.x;
    if (b >= B) return;
    scal[sPhibar * B + b] = scal[sBeta * B + b];
    scal[sRhobar * B + b] = scal[sAlpha * B + b];
}

// the plane rotation of one iteration, per column
__global__ void k_lsqr_rotation(double* scal, int B) {
    const int b = threadIdx.x;
    if (b >= B) return;
    const double alpha = scal[sAlpha * B + b], beta = scal[sBeta * B + b];
    const double rhobar = scal[sRhobar * B + b], phibar = scal[sPhibar * B + b];
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rho > 0.0 ? rhobar / rho : 0.0;
    const double s = rho > 0.0 ? beta / rho : 0.0;
    scal[sRho * B + b] = rho;
    scal[sTheta * B + b] = s * alpha;
    scal[sRhobar * B + b] = -c * alpha;
    scal[sPhi * B + b] = c * phibar;
    scal[sPhibar * B + b] = s * phibar;
}

// v = v / alpha; x += (phi/rho) w; w = v - (theta/rho) w
template <typename V>
__global__ void k_lsqr_xw(V* __restrict__ v, V* __restrict__ x, V* __restrict__ w, int64_t rows, int B,
                          const double* __restrict__ scal) {
    const int64_t n = rows * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i % B);
        const double rho = scal[sRho * B + b];
        const double fphi = rho > 0.0 ? scal[sPhi * B + b] / rho : 0.0;
        const double fth = rho > 0.0 ? scal[sTheta * B + b] / rho : 0.0;
        const double vn = (double)v[i] * scal[sInvNorm * B + b];
        const double wi = (double)w[i];
        v[i] = (V)vn;
        x[i] = (V)((double)x[i] + fphi * wi);
        w[i] = (V)(vn - fth * wi);
    }
}

// y = c (a fill without memset, safe inside captured graphs)
template <typename V>
__global__ void k_fill(V* __restrict__ y, int64_t n, V c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = c;
}

template <typename V>
__global__ void k_copy(V* __restrict__ y, const V* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = x[i];
}

// scal[slot][b] = sum_blk partial[blk][b] (a squared column norm)
__global__ void k_colsum_finalize(const double* __restrict__ partial, int nblk, int B, double* scal, int slot) {
    const int b = threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int q = 0; q < nblk; ++q) s += partial[(int64_t)q * B + b];
    scal[slot * B + b] = s;
}

// CGLS step length and direction scalars, per column; a zero denominator
// (converged column) gives a zero step, so the column stays where it is
__global__ void k_cgls_alpha(double* scal, int B) {
    const int b = threadIdx.x;
    if (b >= B) return;
    const double qq = scal[cQQ * B + b];
    scal[cAlpha * B + b] = qq > 0.0 ? scal[cGamma * B + b] / qq : 0.0;
}

__global__ void k_cgls_beta(double* scal, int B) {
    const int b = threadIdx.x;
    if (b >= B) return;
    const double g = scal[cGamma * B + b], gn = scal[cGnew * B + b];
    scal[cBeta * B + b] = g > 0.0 ? gn / g : 0.0;
    scal[cGamma * B + b] = gn;
}

// x += alpha p (model rows) and r -= alpha q (data rows), one launch each
template <typename V>
__global__ void k_axpy_col(V* __restrict__ y, const V* __restrict__ x, int64_t rows, int B,
                           const double* __restrict__ scal, int slot, double sign) {
    const int64_t n = rows * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (V)((double)y[i] + sign * scal[slot * B + (int)(i % B)] * (double)x[i]);
}

// hist[row][b] = scal[slot][b]
__global__ void k_copy_row(double* __restrict__ hist, int row, const double* __restrict__ scal, int slot, int B) {
    const int b = threadIdx.x;
    if (b < B) hist[(int64_t)row * B + b] = scal[slot * B + b];
}

// p = s + beta p
template <typename V>
__global__ void k_xpby_col(V* __restrict__ p, const V* __restrict__ s, int64_t rows, int B,
                           const double* __restrict__ scal, int slot) {
    const int64_t n = rows * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (V)((double)s[i] + scal[slot * B + (int)(i % B)] * (double)p[i]);
}

}  // namespace fm

struct fm_lsqr {
    fm_batch* b = nullptr;
    void* u = nullptr;       // [S][R][B]
    void* td = nullptr;      // [S][R][B] J v
    void* v = nullptr;       // [N][B]
    void* w = nullptr;       // [N][B]
    void* x = nullptr;       // [N][B]
    void* tv = nullptr;      // [N][B] J^T u
    double* scal = nullptr;  // [kScalars][B]
    double* partial = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_iters = 0;
};

struct fm_cgls {
    fm_batch* b = nullptr;
    void* x = nullptr;       // [N][B]
    void* p = nullptr;       // [N][B]
    void* s = nullptr;       // [N][B] J^T r
    void* r = nullptr;       // [S][R][B]
    void* q = nullptr;       // [S][R][B] J p
    double* scal = nullptr;  // [kCgScalars][B]
    double* partial = nullptr;
    double* hist = nullptr;  // [max_iter + 1][B] ||r||^2 after start and after each iteration
    int32_t max_iter = 0;
    int32_t it = 0;          // iterations enqueued since start (a graph records its own positions)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace fm {

static int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

template <typename V>
static int colnorm(fm_lsqr* L, const void* x, int64_t rows, int slot) {
    fm_batch* b = L->b;
    hipLaunchKernelGGL(k_colsq_partial<V>, dim3(kRedBlocks), dim3(kRedThreads), 0, b->stream, (const V*)x, rows,
                       b->B, L->partial);
    hipLaunchKernelGGL(k_colnorm_finalize, dim3(1), dim3(std::max(64, b->B)), 0, b->stream,
                       (const double*)L->partial, kRedBlocks, b->B, L->scal, slot);
    return hipGetLastError() == hipSuccess ? FM_OK : FM_EHIP;
}

template <typename V>
static int lsqr_start(fm_lsqr* L, const void* d) {
    fm_batch* b = L->b;
    const int64_t nd = (int64_t)b->S * b->R, nm = b->N;
    hipLaunchKernelGGL(k_copy<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)L->u, (const V*)d, nd * b->B);
    int rc = colnorm<V>(L, L->u, nd, sBeta);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scale_inv<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)L->u, nd, b->B,
                       (const double*)L->scal);
    rc = apply_JT(b, L->u, FM_W_RECEIVERS, L->v, FM_JT_SUMMED);
    if (rc) return rc;
    rc = colnorm<V>(L, L->v, nm, sAlpha);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scale_inv<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)L->v, nm, b->B,
                       (const double*)L->scal);
    hipLaunchKernelGGL(k_copy<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)L->w, (const V*)L->v, nm * b->B);
    hipLaunchKernelGGL(k_fill<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)L->x, nm * b->B, (V)0);
    hipLaunchKernelGGL(k_lsqr_start_scalars, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, L->scal, b->B);
    return hipGetLastError() == hipSuccess ? FM_OK : FM_EHIP;
}

template <typename V>
static int lsqr_iterate(fm_lsqr* L, int n) {
    fm_batch* b = L->b;
    const int64_t nd = (int64_t)b->S * b->R, nm = b->N;
    for (int it = 0; it < n; ++it) {
        int rc = apply_J(b, L->v, FM_DS_BROADCAST, L->td, FM_OUT_RECEIVERS);
        if (rc) return rc;
        hipLaunchKernelGGL(k_sub_scaled<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)L->u,
                           (const V*)L->td, nd, b->B, (const double*)L->scal, (int)sAlpha);
        rc = colnorm<V>(L, L->u, nd, sBeta);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scale_inv<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)L->u, nd, b->B,
                           (const double*)L->scal);
        rc = apply_JT(b, L->u, FM_W_RECEIVERS, L->tv, FM_JT_SUMMED);
        if (rc) return rc;
        hipLaunchKernelGGL(k_sub_scaled<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)L->v,
                           (const V*)L->tv, nm, b->B, (const double*)L->scal, (int)sBeta);
        rc = colnorm<V>(L, L->v, nm, sAlpha);
        if (rc) return rc;
        hipLaunchKernelGGL(k_lsqr_rotation, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, L->scal, b->B);
        hipLaunchKernelGGL(k_lsqr_xw<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)L->v, (V*)L->x,
                           (V*)L->w, nm, b->B, (const double*)L->scal);
        if (hipGetLastError() != hipSuccess) { set_error("LSQR kernel launch failed"); return FM_EHIP; }
    }
    return FM_OK;
}

static void lsqr_release(fm_lsqr* L) {
    if (!L) return;
    if (L->exec) (void)hipGraphExecDestroy(L->exec);
    if (L->graph) (void)hipGraphDestroy(L->graph);
    void* bufs[] = {L->u, L->td, L->v, L->w, L->x, L->tv, L->scal, L->partial};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete L;
}

int lsqr_create(fm_batch* b, fm_lsqr** out) {
    if (!b || !out) { set_error("null argument"); return FM_EINVAL; }
    *out = nullptr;
    if (b->R == 0) { set_error("the states have no receivers"); return FM_EINVAL; }
    if (b->B > 256) { set_error("LSQR supports at most 256 right-hand sides"); return FM_EINVAL; }
    fm_lsqr* L = new fm_lsqr();
    L->b = b;
    const size_t vb = b->prec == FM_FP64 ? 8 : 4;
    const size_t nd = (size_t)b->S * b->R * b->B * vb, nm = (size_t)b->N * b->B * vb;
    hipError_t e = hipSuccess;
    void** targets[] = {&L->u, &L->td, &L->v, &L->w, &L->x, &L->tv};
    size_t sizes[] = {nd, nd, nm, nm, nm, nm};
    for (int i = 0; i < 6 && e == hipSuccess; i++) e = hipMalloc(targets[i], sizes[i]);
    if (e == hipSuccess) e = hipMalloc((void**)&L->scal, sizeof(double) * kScalars * b->B);
    if (e == hipSuccess) e = hipMalloc((void**)&L->partial, sizeof(double) * kRedBlocks * b->B);
    if (e != hipSuccess) {
        lsqr_release(L);
        set_error("LSQR allocation failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    *out = L;
    return FM_OK;
}

int lsqr_start_any(fm_lsqr* L, const void* d) {
    if (!L || !d) { set_error("null argument"); return FM_EINVAL; }
    return L->b->prec == FM_FP64 ? lsqr_start<double>(L, d) : lsqr_start<float>(L, d);
}

int lsqr_iterate_any(fm_lsqr* L, int32_t n) {
    if (!L || n < 0) { set_error("bad arguments"); return FM_EINVAL; }
    return L->b->prec == FM_FP64 ? lsqr_iterate<double>(L, n) : lsqr_iterate<float>(L, n);
}

int lsqr_capture(fm_lsqr* L, int32_t n) {
    if (!L || n < 1) { set_error("bad arguments"); return FM_EINVAL; }
    if (L->exec) { (void)hipGraphExecDestroy(L->exec); L->exec = nullptr; }
    if (L->graph) { (void)hipGraphDestroy(L->graph); L->graph = nullptr; }
    hipStream_t s = L->b->stream;
    if (s == nullptr) { set_error("graph capture needs a non-null batch stream"); return FM_EINVAL; }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = lsqr_iterate_any(L, n);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    e = hipGraphInstantiate(&L->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return FM_EHIP;
    }
    L->graph = g;
    L->graph_iters = n;
    return FM_OK;
}

int lsqr_replay(fm_lsqr* L) {
    if (!L || !L->exec) { set_error("no captured graph"); return FM_ESTATE; }
    HIP_TRY(hipGraphLaunch(L->exec, L->b->stream));
    return FM_OK;
}

int lsqr_buffers(const fm_lsqr* L, void** x, void** u, void** v, double** scal) {
    if (!L) { set_error("null argument"); return FM_EINVAL; }
    if (x) *x = L->x;
    if (u) *u = L->u;
    if (v) *v = L->v;
    if (scal) *scal = L->scal;
    return FM_OK;
}

void lsqr_free(fm_lsqr* L) { lsqr_release(L); }

// ---------------------------------------------------------------------------
// CGLS
// ---------------------------------------------------------------------------
template <typename V>
static void colsq(fm_batch* b, double* partial, double* scal, const void* x, int64_t rows, int slot) {
    hipLaunchKernelGGL(k_colsq_partial<V>, dim3(kRedBlocks), dim3(kRedThreads), 0, b->stream, (const V*)x, rows,
                       b->B, partial);
    hipLaunchKernelGGL(k_colsum_finalize, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, (const double*)partial,
                       kRedBlocks, b->B, scal, slot);
}

template <typename V>
static int cgls_start(fm_cgls* C, const void* d) {
    fm_batch* b = C->b;
    const int64_t nd = (int64_t)b->S * b->R, nm = b->N;
    hipLaunchKernelGGL(k_copy<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)C->r, (const V*)d, nd * b->B);
    int rc = apply_JT(b, C->r, FM_W_RECEIVERS, C->s, FM_JT_SUMMED);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)C->p, (const V*)C->s, nm * b->B);
    hipLaunchKernelGGL(k_fill<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)C->x, nm * b->B, (V)0);
    colsq<V>(b, C->partial, C->scal, C->s, nm, cGamma);
    colsq<V>(b, C->partial, C->scal, C->r, nd, cRR);
    C->it = 0;
    hipLaunchKernelGGL(k_copy_row, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, C->hist, 0,
                       (const double*)C->scal, (int)cRR, b->B);
    if (hipGetLastError() != hipSuccess) { set_error("CGLS kernel launch failed"); return FM_EHIP; }
    return FM_OK;
}

template <typename V>
static int cgls_iterate(fm_cgls* C, int n) {
    fm_batch* b = C->b;
    const int64_t nd = (int64_t)b->S * b->R, nm = b->N;
    for (int it = 0; it < n; ++it) {
        int rc = apply_J(b, C->p, FM_DS_BROADCAST, C->q, FM_OUT_RECEIVERS);
        if (rc) return rc;
        colsq<V>(b, C->partial, C->scal, C->q, nd, cQQ);
        hipLaunchKernelGGL(k_cgls_alpha, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, C->scal, b->B);
        hipLaunchKernelGGL(k_axpy_col<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)C->x,
                           (const V*)C->p, nm, b->B, (const double*)C->scal, (int)cAlpha, 1.0);
        hipLaunchKernelGGL(k_axpy_col<V>, dim3(grid_for(nd * b->B)), dim3(256), 0, b->stream, (V*)C->r,
                           (const V*)C->q, nd, b->B, (const double*)C->scal, (int)cAlpha, -1.0);
        rc = apply_JT(b, C->r, FM_W_RECEIVERS, C->s, FM_JT_SUMMED);
        if (rc) return rc;
        colsq<V>(b, C->partial, C->scal, C->s, nm, cGnew);
        hipLaunchKernelGGL(k_cgls_beta, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, C->scal, b->B);
        hipLaunchKernelGGL(k_xpby_col<V>, dim3(grid_for(nm * b->B)), dim3(256), 0, b->stream, (V*)C->p,
                           (const V*)C->s, nm, b->B, (const double*)C->scal, (int)cBeta);
        colsq<V>(b, C->partial, C->scal, C->r, nd, cRR);
        if (++C->it <= C->max_iter)
            hipLaunchKernelGGL(k_copy_row, dim3(1), dim3(std::max(64, b->B)), 0, b->stream, C->hist, C->it,
                               (const double*)C->scal, (int)cRR, b->B);
        if (hipGetLastError() != hipSuccess) { set_error("CGLS kernel launch failed"); return FM_EHIP; }
    }
    return FM_OK;
}

static void cgls_release(fm_cgls* C) {
    if (!C) return;
    if (C->exec) (void)hipGraphExecDestroy(C->exec);
    if (C->graph) (void)hipGraphDestroy(C->graph);
    void* bufs[] = {C->x, C->p, C->s, C->r, C->q, C->scal, C->partial, C->hist};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete C;
}

int cgls_create(fm_batch* b, int32_t max_iter, fm_cgls** out) {
    if (!b || !out) { set_error("null argument"); return FM_EINVAL; }
    if (max_iter < 0) { set_error("max_iter must be >= 0"); return FM_EINVAL; }
    *out = nullptr;
    if (b->R == 0) { set_error("the states have no receivers"); return FM_EINVAL; }
    if (b->B > 256) { set_error("CGLS supports at most 256 right-hand sides"); return FM_EINVAL; }
    fm_cgls* C = new fm_cgls();
    C->b = b;
    C->max_iter = max_iter;
    const size_t vb = b->prec == FM_FP64 ? 8 : 4;
    const size_t nd = (size_t)b->S * b->R * b->B * vb, nm = (size_t)b->N * b->B * vb;
    hipError_t e = hipSuccess;
    void** targets[] = {&C->x, &C->p, &C->s, &C->r, &C->q};
    size_t sizes[] = {nm, nm, nm, nd, nd};
    for (int i = 0; i < 5 && e == hipSuccess; i++) e = hipMalloc(targets[i], sizes[i]);
    if (e == hipSuccess) e = hipMalloc((void**)&C->scal, sizeof(double) * kCgScalars * b->B);
    if (e == hipSuccess) e = hipMalloc((void**)&C->partial, sizeof(double) * kRedBlocks * b->B);
    if (e == hipSuccess) e = hipMalloc((void**)&C->hist, sizeof(double) * ((size_t)max_iter + 1) * b->B);
    if (e != hipSuccess) {
        cgls_release(C);
        set_error("CGLS allocation failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    *out = C;
    return FM_OK;
}

int cgls_start_any(fm_cgls* C, const void* d) {
    if (!C || !d) { set_error("null argument"); return FM_EINVAL; }
    return C->b->prec == FM_FP64 ? cgls_start<double>(C, d) : cgls_start<float>(C, d);
}

int cgls_iterate_any(fm_cgls* C, int32_t n) {
    if (!C || n < 0) { set_error("bad arguments"); return FM_EINVAL; }
    return C->b->prec == FM_FP64 ? cgls_iterate<double>(C, n) : cgls_iterate<float>(C, n);
}

int cgls_capture(fm_cgls* C, int32_t n) {
    if (!C || n < 1) { set_error("bad arguments"); return FM_EINVAL; }
    if (C->exec) { (void)hipGraphExecDestroy(C->exec); C->exec = nullptr; }
    if (C->graph) { (void)hipGraphDestroy(C->graph); C->graph = nullptr; }
    hipStream_t s = C->b->stream;
    if (s == nullptr) { set_error("graph capture needs a non-null batch stream"); return FM_EINVAL; }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = cgls_iterate_any(C, n);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    e = hipGraphInstantiate(&C->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return FM_EHIP;
    }
    C->graph = g;
    return FM_OK;
}

int cgls_replay(fm_cgls* C) {
    if (!C || !C->exec) { set_error("no captured graph"); return FM_ESTATE; }
    HIP_TRY(hipGraphLaunch(C->exec, C->b->stream));
    return FM_OK;
}

int cgls_buffers(const fm_cgls* C, void** x, void** r, double** scal, double** hist) {
    if (!C) { set_error("null argument"); return FM_EINVAL; }
    if (x) *x = C->x;
    if (r) *r = C->r;
    if (scal) *scal = C->scal;
    if (hist) *hist = C->hist;
    return FM_OK;
}

void cgls_free(fm_cgls* C) { cgls_release(C); }

}  // namespace fm
