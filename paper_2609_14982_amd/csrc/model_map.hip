// Cell-velocity model map M_alpha (Section 4.4, eq. (source-jacobian)): the
// inversion unknowns are cell velocities, the transport takes nodal slowness.
// A node's slowness is the reciprocal of the mean velocity of the cells that
// share it, s_p = 1 / vbar_p with vbar_p = (1/n_p) sum_{c around p} v_c, so
// the linearised map and its transpose are
//   (M dv)_p    = a_p sum_{c around p} dv_c,      a_p = -1 / (n_p vbar_p^2),
//   (M^T g)_c   = sum_{p corner of c} a_p g_p.
// Cells are the logical hexahedra (quadrilaterals in 2-D) between nodes,
// cell id c = ci + (n1-1) (cj + (n2-1) ck); a node has 1, 2, 4 or 8 cells.
// M is the same for every source, so one application serves a whole batch
// (J M = stacked J_alpha of the broadcast model block, M^T after the source
// sum).  Both products are gathers with a fixed summation order (ascending
// cell or node id): deterministic, no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fmbtf.h"
#include "internal.h"
#include "batch.h"

struct fm_model_map {
    int dim = 3;
    int64_t n[3] = {1, 1, 1};    // nodes per logical axis (axis 0 fastest; 2-D: n[1] = n3, n[2] = 1)
    int64_t c[3] = {1, 1, 1};    // cells per axis (1 for an axis of one node)
    int64_t N = 0, Nc = 0;
    std::vector<double> slow;    // host [N] background slowness 1 / vbar
    double* scale = nullptr;     // device [N] a_p
    hipStream_t stream = nullptr;
    int device = -1;
};

namespace fm {

struct MapDims {
    int64_t n0, n1, n2, c0, c1, c2;
};

__device__ __forceinline__ void cell_range(int64_t i, int64_t n, int64_t& lo, int64_t& hi) {
    if (n == 1) { lo = 0; hi = 0; return; }
    lo = i > 0 ? i - 1 : 0;
    hi = i < n - 1 ? i : n - 2;
}

template <typename V>
__global__ void k_model_map(MapDims d, const double* __restrict__ a, const V* __restrict__ dv, V* __restrict__ ds,
                            int B) {
    const int64_t total = d.n0 * d.n1 * d.n2 * B;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / B, b = t - p * B;
        const int64_t i = p % d.n0, r = p / d.n0, j = r % d.n1, k = r / d.n1;
        int64_t i0, i1, j0, j1, k0, k1;
        cell_range(i, d.n0, i0, i1);
        cell_range(j, d.n1, j0, j1);
        cell_range(k, d.n2, k0, k1);
        V acc = (V)0;
        for (int64_t ck = k0; ck <= k1; ++ck)
            for (int64_t cj = j0; cj <= j1; ++cj)
                for (int64_t ci = i0; ci <= i1; ++ci) acc += dv[(ci + d.c0 * (cj + d.c1 * ck)) * B + b];
        ds[t] = (V)a[p] * acc;
    }
}

template <typename V>
__global__ void k_model_map_t(MapDims d, const double* __restrict__ a, const V* __restrict__ g, V* __restrict__ out,
                              int B) {
    const int64_t total = d.c0 * d.c1 * d.c2 * B;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / B, b = t - c * B;
        const int64_t ci = c % d.c0, r = c / d.c0, cj = r % d.c1, ck = r / d.c1;
        const int64_t i1 = d.n0 > 1 ? ci + 1 : ci, j1 = d.n1 > 1 ? cj + 1 : cj, k1 = d.n2 > 1 ? ck + 1 : ck;
        V acc = (V)0;
        for (int64_t k = ck; k <= k1; ++k)
            for (int64_t j = cj; j <= j1; ++j)
                for (int64_t i = ci; i <= i1; ++i) {
                    const int64_t p = i + d.n0 * (j + d.n1 * k);
                    acc += (V)a[p] * g[p * B + b];
                }
        out[t] = acc;
    }
}

static MapDims dims_of(const fm_model_map* m) {
    return MapDims{m->n[0], m->n[1], m->n[2], m->c[0], m->c[1], m->c[2]};
}

static int check_map(const fm_model_map* m, int32_t B, int32_t precision, const void* x, const void* y) {
    if (!m) { set_error("null model map"); return FM_EINVAL; }
    if (B < 1) { set_error("B must be >= 1"); return FM_EINVAL; }
    if (precision != FM_FP64 && precision != FM_FP32) { set_error("precision must be FM_FP64 or FM_FP32"); return FM_EINVAL; }
    if (!x || !y) { set_error("null vector"); return FM_EINVAL; }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) { set_error("model map lives on device %d (current device %d)", m->device, dev); return FM_ESTATE; }
    return FM_OK;
}

static int grid_for(int64_t work) {
    return (int)std::min<int64_t>(std::max<int64_t>((work + 255) / 256, 1), 16384);
}

}  // namespace fm

extern "C" {

int fm_model_map_create(int32_t dim, int64_t n1, int64_t n2, int64_t n3, const double* v_cell, void* hip_stream,
                        fm_model_map** out) {
    using namespace fm;
    clear_error();
    if (!out) { set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { set_error("dim must be 2 or 3, got %d", dim); return FM_EINVAL; }
    if (dim == 2 && n2 != 1) { set_error("2-D grids need n2 == 1"); return FM_EINVAL; }
    if (n1 < 2 || n3 < 2 || (dim == 3 && n2 < 2)) { set_error("every axis of the grid needs at least 2 nodes"); return FM_EINVAL; }
    if (!v_cell) { set_error("null cell velocities"); return FM_EINVAL; }
    fm_model_map* m = new (std::nothrow) fm_model_map();
    if (!m) { set_error("out of host memory"); return FM_ENOMEM; }
    m->dim = dim;
    m->n[0] = n1;
    m->n[1] = dim == 3 ? n2 : n3;
    m->n[2] = dim == 3 ? n3 : 1;
    for (int d = 0; d < 3; d++) m->c[d] = m->n[d] > 1 ? m->n[d] - 1 : 1;
    m->N = m->n[0] * m->n[1] * m->n[2];
    m->Nc = m->c[0] * m->c[1] * m->c[2];
    for (int64_t c = 0; c < m->Nc; c++)
        if (!(v_cell[c] > 0.0) || !std::isfinite(v_cell[c])) {
            set_error("cell velocity %lld must be finite and > 0", (long long)c);
            delete m;
            return FM_EINVAL;
        }
    std::vector<double> a;
    try {
        m->slow.resize(m->N);
        a.resize(m->N);
    } catch (const std::bad_alloc&) {
        delete m;
        set_error("out of host memory");
        return FM_ENOMEM;
    }
    auto range = [&](int64_t i, int d, int64_t& lo, int64_t& hi) {
        if (m->n[d] == 1) { lo = hi = 0; return; }
        lo = i > 0 ? i - 1 : 0;
        hi = i < m->n[d] - 1 ? i : m->n[d] - 2;
    };
    for (int64_t p = 0; p < m->N; p++) {
        const int64_t i = p % m->n[0], r = p / m->n[0], j = r % m->n[1], k = r / m->n[1];
        int64_t i0, i1, j0, j1, k0, k1;
        range(i, 0, i0, i1);
        range(j, 1, j0, j1);
        range(k, 2, k0, k1);
        double sum = 0.0;
        int cnt = 0;
        for (int64_t ck = k0; ck <= k1; ++ck)
            for (int64_t cj = j0; cj <= j1; ++cj)
                for (int64_t ci = i0; ci <= i1; ++ci) {
                    sum += v_cell[ci + m->c[0] * (cj + m->c[1] * ck)];
                    cnt++;
                }
        const double vbar = sum / cnt;
        m->slow[p] = 1.0 / vbar;
        a[p] = -1.0 / ((double)cnt * vbar * vbar);
    }
    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) e = hipMalloc((void**)&m->scale, sizeof(double) * (size_t)m->N);
    if (e == hipSuccess) e = hipMemcpy(m->scale, a.data(), sizeof(double) * (size_t)m->N, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (m->scale) (void)hipFree(m->scale);
        set_error("model map upload failed: %s", hipGetErrorString(e));
        const bool oom = e == hipErrorOutOfMemory;
        delete m;
        return oom ? FM_ENOMEM : FM_EHIP;
    }
    m->stream = (hipStream_t)hip_stream;
    *out = m;
    return FM_OK;
}

int fm_model_map_sizes(const fm_model_map* m, int64_t* n_nodes, int64_t* n_cells) {
    fm::clear_error();
    if (!m) { fm::set_error("null model map"); return FM_EINVAL; }
    if (n_nodes) *n_nodes = m->N;
    if (n_cells) *n_cells = m->Nc;
    return FM_OK;
}

int fm_model_map_slowness(const fm_model_map* m, double* s_out) {
    fm::clear_error();
    if (!m || !s_out) { fm::set_error("null argument"); return FM_EINVAL; }
    std::copy(m->slow.begin(), m->slow.end(), s_out);
    return FM_OK;
}

int fm_model_map_set_stream(fm_model_map* m, void* hip_stream) {
    fm::clear_error();
    if (!m) { fm::set_error("null model map"); return FM_EINVAL; }
    m->stream = (hipStream_t)hip_stream;
    return FM_OK;
}

int fm_model_map_apply(fm_model_map* m, int32_t B, int32_t precision, const void* dv, void* ds) {
    using namespace fm;
    clear_error();
    int rc = check_map(m, B, precision, dv, ds);
    if (rc) return rc;
    const int grid = grid_for(m->N * B);
    if (precision == FM_FP64)
        hipLaunchKernelGGL(k_model_map<double>, dim3(grid), dim3(256), 0, m->stream, dims_of(m), m->scale,
                           (const double*)dv, (double*)ds, (int)B);
    else
        hipLaunchKernelGGL(k_model_map<float>, dim3(grid), dim3(256), 0, m->stream, dims_of(m), m->scale,
                           (const float*)dv, (float*)ds, (int)B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("model map launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    return FM_OK;
}

int fm_model_map_apply_T(fm_model_map* m, int32_t B, int32_t precision, const void* g, void* dv_out) {
    using namespace fm;
    clear_error();
    int rc = check_map(m, B, precision, g, dv_out);
    if (rc) return rc;
    const int grid = grid_for(m->Nc * B);
    if (precision == FM_FP64)
        hipLaunchKernelGGL(k_model_map_t<double>, dim3(grid), dim3(256), 0, m->stream, dims_of(m), m->scale,
                           (const double*)g, (double*)dv_out, (int)B);
    else
        hipLaunchKernelGGL(k_model_map_t<float>, dim3(grid), dim3(256), 0, m->stream, dims_of(m), m->scale,
                           (const float*)g, (float*)dv_out, (int)B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("model map transpose launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    return FM_OK;
}

void fm_model_map_free(fm_model_map* m) {
    if (!m) return;
    if (m->scale) (void)hipFree(m->scale);
    delete m;
}

}  // extern "C"
