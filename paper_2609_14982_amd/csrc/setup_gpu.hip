// The GPU setup pass (Algorithm 1, Phase I, lines 7-8): the couplings of
// every source's frozen operator computed on the device, for all sources of
// a batch at once, from traveltimes that are already there (the GPU
// first-arrival solver's output, or an upload).
//
// Per (source, node), as the host setup does it (Sections 3.1-3.2): the face
// coefficient a_f of each of the node's faces (G_f the mean of the two nodal
// metrics, the normal derivative the compact difference, each tangential
// derivative the mean of the two nodal central differences, one-sided at the
// ends of an axis), the upwind parts c = max(+-a_f, 0) towards the node, the
// weights w = c / sum c (an identity row at the source and where nothing
// flows in), the calibration c_i = (T_i - sum_j w_ij T_j) / s_i, and the
// count of violating edges (T_j > T_i for an edge j -> i).  Every product and
// sum is rounded as written and in the host's order (-ffp-contract=off), so
// the couplings equal the host's bit for bit; the host then finishes the
// state (SCCs, levels, block factors, packing) from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fmbtf.h"
#include "internal.h"
#include "batch.h"

namespace fm {

namespace {

struct SetupDims {
    int dim, ncomp_g;
    int64_t n[3], stride[3], N;
};

__device__ __forceinline__ int64_t coord_of(const SetupDims& g, int64_t p, int axis) {
    return (p / g.stride[axis]) % g.n[axis];
}

__device__ __forceinline__ double metric_of(const SetupDims& g, const double* __restrict__ G, int64_t p, int a, int b) {
    const double* m = G + (size_t)g.ncomp_g * (size_t)p;
    if (g.dim == 2) return a == b ? m[a] : m[2];
    if (a == b) return m[a];
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    if (lo == 0 && hi == 1) return m[3];
    if (lo == 0 && hi == 2) return m[4];
    return m[5];
}

__device__ __forceinline__ double nodal_diff(const SetupDims& g, const double* __restrict__ T, int64_t p, int axis) {
    const int64_t c = coord_of(g, p, axis), n = g.n[axis], st = g.stride[axis];
    if (n == 1) return 0.0;
    if (c == 0) return T[p + st] - T[p];
    if (c == n - 1) return T[p] - T[p - st];
    return 0.5 * (T[p + st] - T[p - st]);
}

// a_f of the face between lo and lo + e_d
__device__ __forceinline__ double face_coef(const SetupDims& g, const double* __restrict__ G,
                                            const double* __restrict__ T, int64_t lo, int d) {
    const int64_t hi = lo + g.stride[d];
    double a = 0.0;
    for (int dp = 0; dp < g.dim; dp++) {
        double gd;
        if (dp == d) gd = T[hi] - T[lo];
        else gd = 0.5 * (nodal_diff(g, T, lo, dp) + nodal_diff(g, T, hi, dp));
        const double Gf = 0.5 * (metric_of(g, G, lo, d, dp) + metric_of(g, G, hi, d, dp));
        const double term = Gf * gd;
        a = dp == 0 ? term : a + term;
    }
    return a;
}

__global__ void k_setup_couplings(SetupDims g, int32_t S, const double* __restrict__ G,
                                  const double* __restrict__ Tall, const double* __restrict__ s,
                                  const int64_t* __restrict__ src, double* __restrict__ w6,
                                  uint8_t* __restrict__ pmask, double* __restrict__ cal,
                                  unsigned long long* __restrict__ nvio, int* __restrict__ bad) {
    const int nslot = 2 * g.dim;
    const int64_t total = (int64_t)S * g.N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t alpha = t / g.N, p = t - alpha * g.N;
        const double* __restrict__ T = Tall + alpha * g.N;
        if (!isfinite(T[p])) atomicOr(bad + alpha, 1);
        if (p == src[alpha] && T[p] != 0.0) atomicOr(bad + alpha, 2);
        double c6[6] = {0, 0, 0, 0, 0, 0};
        for (int slot = 0; slot < nslot; slot++) {
            const int d = slot >> 1;
            const int64_t c = coord_of(g, p, d);
            if (slot & 1) {
                if (c + 1 >= g.n[d]) continue;
                const double a = face_coef(g, G, T, p, d);
                c6[slot] = -a > 0.0 ? -a : 0.0;
            } else {
                if (c == 0) continue;
                const double a = face_coef(g, G, T, p - g.stride[d], d);
                c6[slot] = a > 0.0 ? a : 0.0;
            }
        }
        double dsum = 0.0;
        for (int slot = 0; slot < nslot; slot++) dsum = dsum + c6[slot];
        double acc = 0.0;
        uint8_t mask = 0;
        double w[6] = {0, 0, 0, 0, 0, 0};
        unsigned nv = 0;
        if (p != src[alpha] && dsum > 0.0) {
            for (int slot = 0; slot < nslot; slot++) {
                if (c6[slot] > 0.0) {
                    const double wt = c6[slot] / dsum;
                    if (wt > 0.0) {
                        const int d = slot >> 1;
                        const int64_t q = (slot & 1) ? p + g.stride[d] : p - g.stride[d];
                        w[slot] = wt;
                        mask |= (uint8_t)(1u << slot);
                        acc = acc + wt * T[q];
                        nv += T[q] > T[p] ? 1u : 0u;
                    }
                }
            }
        }
        for (int slot = 0; slot < 6; slot++) w6[t * 6 + slot] = w[slot];
        pmask[t] = mask;
        const double ell = T[p] - acc;
        cal[t] = ell / s[p];
        if (nv) atomicAdd(nvio + alpha, (unsigned long long)nv);
    }
}

}  // namespace

}  // namespace fm

extern "C" int fm_build_frozen_states_gpu(const fm_grid* g, int32_t S, const double* T_dev, const double* s,
                                          const int64_t* src_nodes, const int64_t* rcv_nodes,
                                          const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv,
                                          int32_t nthreads, void* hip_stream, fm_state** out) {
    using namespace fm;
    clear_error();
    if (!g || !g->G || !T_dev || !s || !src_nodes || !out || S < 1) { set_error("bad arguments"); return FM_EINVAL; }
    if (g->dim != 2 && g->dim != 3) { set_error("dim must be 2 or 3, got %d", g->dim); return FM_EINVAL; }
    if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1) { set_error("grid sizes must be >= 1"); return FM_EINVAL; }
    if (g->dim == 2 && g->n2 != 1) { set_error("2-D grids need n2 == 1"); return FM_EINVAL; }
    if (k_per_rcv < 1) { set_error("entries per receiver must be >= 1"); return FM_EINVAL; }
    if (g->stencil != 0 && g->stencil != 6) {
        set_error("the GPU setup pass builds face-stencil states only (stencil %d)", g->stencil);
        return FM_EINVAL;
    }
    if ((uintptr_t)T_dev & 7u) { set_error("T must be 8-byte aligned"); return FM_EINVAL; }
    SetupDims d{};
    d.dim = g->dim;
    d.ncomp_g = g->dim == 3 ? 6 : 3;
    d.n[0] = g->n1;
    d.n[1] = g->dim == 3 ? g->n2 : g->n3;
    d.n[2] = g->dim == 3 ? g->n3 : 1;
    d.stride[0] = 1;
    d.stride[1] = d.n[0];
    d.stride[2] = d.n[0] * d.n[1];
    d.N = d.n[0] * d.n[1] * d.n[2];
    const int64_t N = d.N;
    if (N >= (int64_t)kNodeMask) { set_error("grid too large: %lld nodes", (long long)N); return FM_EINVAL; }
    for (int32_t a = 0; a < S; a++)
        if (src_nodes[a] < 0 || src_nodes[a] >= N) {
            set_error("source %d: node %lld out of range", a, (long long)src_nodes[a]);
            return FM_EINVAL;
        }
    hipStream_t st = (hipStream_t)hip_stream;
    const int nt = std::max(1, std::min<int32_t>(nthreads > 0 ? nthreads : 1, S));
    // sources go through the device in chunks of up to nt (about 2 GB of
    // couplings at most); host threads finish the states of one chunk while
    // the device computes the next
    const int32_t chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t)(2LL << 30) / (N * 57)));
    double *dG = nullptr, *ds = nullptr, *dw = nullptr, *dc = nullptr;
    uint8_t* dm = nullptr;
    int64_t* dsrc = nullptr;
    unsigned long long* dnv = nullptr;
    int* dbad = nullptr;
    auto release = [&]() {
        for (void* p : {(void*)dG, (void*)ds, (void*)dw, (void*)dc, (void*)dm, (void*)dsrc, (void*)dnv, (void*)dbad})
            if (p) (void)hipFree(p);
    };
    hipError_t e = hipMalloc(&dG, sizeof(double) * (size_t)N * d.ncomp_g);
    if (e == hipSuccess) e = hipMalloc(&ds, sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = hipMalloc(&dw, sizeof(double) * 6 * (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dc, sizeof(double) * (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dm, (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dsrc, sizeof(int64_t) * S);
    if (e == hipSuccess) e = hipMalloc(&dnv, sizeof(unsigned long long) * S);
    if (e == hipSuccess) e = hipMalloc(&dbad, sizeof(int) * S);
    if (e == hipSuccess) e = hipMemcpy(dG, g->G, sizeof(double) * (size_t)N * d.ncomp_g, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ds, s, sizeof(double) * (size_t)N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dsrc, src_nodes, sizeof(int64_t) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(dnv, 0, sizeof(unsigned long long) * S);
    if (e == hipSuccess) e = hipMemset(dbad, 0, sizeof(int) * S);
    if (e != hipSuccess) {
        release();
        set_error("GPU setup allocation failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    struct Couplings {
        std::vector<uint8_t> m;
        std::vector<double> w, c;
    };
    std::vector<Couplings> buf(S);
    std::vector<fm_state*> res(S, nullptr);
    std::vector<unsigned long long> nv(S);
    std::vector<int> bad(S);
    std::vector<int> rcs(S, FM_OK);
    std::vector<std::string> msgs(S);
    const size_t per_src = (size_t)(n_rcv > 0 ? n_rcv : 0) * (size_t)k_per_rcv;
    std::mutex mu;
    std::condition_variable cv;
    int32_t ready = 0;         // sources whose couplings are on the host
    bool stop = false;         // the device side failed: workers finish what they hold
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int32_t a;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&]() { return stop || next.load() < ready || next.load() >= S; });
                if (next.load() >= S || (stop && next.load() >= ready)) return;
                a = next.fetch_add(1);
            }
            Assembled pre{buf[a].m.data(), buf[a].w.data(), buf[a].c.data(), (int64_t)nv[a]};
            fm_state* stt = nullptr;
            const int r = build_state(g, nullptr, s, src_nodes[a],
                                      n_rcv > 0 ? rcv_nodes + (size_t)a * per_src : nullptr,
                                      n_rcv > 0 && rcv_weights ? rcv_weights + (size_t)a * per_src : nullptr,
                                      n_rcv, k_per_rcv, &stt, nullptr, &pre);
            rcs[a] = r;
            res[a] = stt;
            if (r != FM_OK) msgs[a] = fm_last_error();
            std::vector<uint8_t>().swap(buf[a].m);
            std::vector<double>().swap(buf[a].w);
            std::vector<double>().swap(buf[a].c);
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < nt; i++) th.emplace_back(worker);
    int rc = FM_OK;
    std::string msg;
    for (int32_t a0 = 0; a0 < S; a0 += chunk) {
        const int32_t n = std::min(chunk, S - a0);
        const int64_t total = (int64_t)n * N;
        const int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        hipLaunchKernelGGL(k_setup_couplings, dim3(grid), dim3(256), 0, st, d, n, dG, T_dev + (size_t)a0 * N, ds,
                           dsrc + a0, dw, dm, dc, dnv + a0, dbad + a0);
        e = hipGetLastError();
        for (int32_t k = 0; k < n && e == hipSuccess; k++) {
            Couplings& cp = buf[a0 + k];
            cp.m.resize((size_t)N);
            cp.w.resize((size_t)N * 6);
            cp.c.resize((size_t)N);
            e = hipMemcpyAsync(cp.m.data(), dm + (size_t)k * N, (size_t)N, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cp.w.data(), dw + (size_t)k * N * 6, sizeof(double) * 6 * (size_t)N,
                                   hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cp.c.data(), dc + (size_t)k * N, sizeof(double) * (size_t)N, hipMemcpyDeviceToHost, st);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(nv.data() + a0, dnv + a0, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(bad.data() + a0, dbad + a0, sizeof(int) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            rc = FM_EHIP;
            msg = std::string("GPU setup pass failed: ") + hipGetErrorString(e);
            break;
        }
        for (int32_t k = 0; k < n && rc == FM_OK; k++)
            if (bad[a0 + k]) {
                rc = FM_EINVAL;
                msg = "source " + std::to_string(a0 + k) +
                      (bad[a0 + k] & 1 ? ": T is not finite" : ": T at the source node must be 0");
            }
        if (rc != FM_OK) break;
        {
            std::lock_guard<std::mutex> lk(mu);
            ready = a0 + n;
        }
        cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        if (rc != FM_OK) stop = true;
    }
    cv.notify_all();
    for (auto& t : th) t.join();
    for (int32_t a = 0; a < S && rc == FM_OK; a++)
        if (res[a] == nullptr || rcs[a] != FM_OK) {
            rc = rcs[a] != FM_OK ? rcs[a] : FM_EHIP;
            msg = "source " + std::to_string(a) + ": " + msgs[a];
        }
    release();
    if (rc != FM_OK) {
        for (auto* p : res) fm_state_free(p);
        set_error("%s", msg.c_str());
        return rc;
    }
    std::copy(res.begin(), res.end(), out);
    return FM_OK;
}
