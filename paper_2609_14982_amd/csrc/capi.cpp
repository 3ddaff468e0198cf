// extern "C" boundary of fmbtf (declared in include/fmbtf.h).
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace fm {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// device.hip
int batch_create(fm_state* const* states, int32_t S, int32_t B, int32_t precision, const fm_tuning* tuning,
                 void* stream, fm_batch** out);
void batch_free(fm_batch* b);
int apply_J(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode);
int apply_JT(fm_batch* b, const void* w, int32_t w_mode, void* out, int32_t out_mode);
int batch_set_stream(fm_batch* b, void* stream);
int batch_tuning(const fm_batch* b, fm_tuning* out);
int batch_status(fm_batch* b);
int batch_split_info(fm_batch* b, int32_t* xcd_masks);
int autotune(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* stream, const void* ds,
             int32_t ds_mode, void* j_out, int32_t out_mode, const void* w, int32_t w_mode, void* jt_out,
             int32_t jt_mode, int32_t reps, const char* cache_path, fm_tuning* best, fm_tuning* cands, float* ms,
             int32_t max_out, int32_t* n_out);
int apply_J_static(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* stream, const void* ds,
                   int32_t ds_mode, void* out, int32_t out_mode);
int apply_J_sweep(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode, int32_t max_cycles,
                  int32_t* cycles_host);
int apply_JT_sweep(fm_batch* b, const void* w, void* out, int32_t out_mode, int32_t max_cycles, int32_t* cycles_host);
int lsqr_create(fm_batch* b, fm_lsqr** out);
int lsqr_start_any(fm_lsqr* L, const void* d);
int lsqr_iterate_any(fm_lsqr* L, int32_t n);
int lsqr_capture(fm_lsqr* L, int32_t n);
int lsqr_replay(fm_lsqr* L);
int lsqr_buffers(const fm_lsqr* L, void** x, void** u, void** v, double** scal);
void lsqr_free(fm_lsqr* L);
int cgls_create(fm_batch* b, int32_t max_iter, fm_cgls** out);
int cgls_start_any(fm_cgls* C, const void* d);
int cgls_iterate_any(fm_cgls* C, int32_t n);
int cgls_capture(fm_cgls* C, int32_t n);
int cgls_replay(fm_cgls* C);
int cgls_buffers(const fm_cgls* C, void** x, void** r, double** scal, double** hist);
void cgls_free(fm_cgls* C);

}  // namespace fm

using fm::HostState;

extern "C" {

int fm_build_frozen_state(const fm_grid* g, const double* T, const double* s, int64_t src_node,
                          const int64_t* rcv_nodes, int32_t n_rcv, fm_state** out) {
    return fm_build_frozen_state_w(g, T, s, src_node, rcv_nodes, nullptr, n_rcv, 1, out);
}

int fm_build_frozen_state_w(const fm_grid* g, const double* T, const double* s, int64_t src_node,
                            const int64_t* rcv_nodes, const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv,
                            fm_state** out) {
    fm::clear_error();
    if (!out) { fm::set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    return fm::build_state(g, T, s, src_node, rcv_nodes, rcv_weights, n_rcv, k_per_rcv, out);
}

int fm_build_frozen_states(const fm_grid* g, int32_t S, const double* T, const double* s,
                           const int64_t* src_nodes, const int64_t* rcv_nodes, int32_t n_rcv,
                           int32_t nthreads, fm_state** out) {
    return fm_build_frozen_states_w(g, S, T, s, src_nodes, rcv_nodes, nullptr, n_rcv, 1, nthreads, out);
}

int fm_build_frozen_states_w(const fm_grid* g, int32_t S, const double* T, const double* s,
                             const int64_t* src_nodes, const int64_t* rcv_nodes, const double* rcv_weights,
                             int32_t n_rcv, int32_t k_per_rcv, int32_t nthreads, fm_state** out) {
    fm::clear_error();
    if (!g || !T || !s || !src_nodes || !out || S < 1) { fm::set_error("bad arguments"); return FM_EINVAL; }
    if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1) { fm::set_error("grid sizes must be >= 1"); return FM_EINVAL; }
    if (k_per_rcv < 1) { fm::set_error("entries per receiver must be >= 1"); return FM_EINVAL; }
    const int64_t N = g->n1 * g->n2 * g->n3;
    const size_t per_src = (size_t)(n_rcv > 0 ? n_rcv : 0) * (size_t)k_per_rcv;
    std::vector<fm_state*> res(S, nullptr);
    std::vector<int> rcs(S, FM_OK);
    std::vector<std::string> msgs(S);
    std::atomic<int32_t> next{0};
    int nt = std::max(1, std::min<int32_t>(nthreads > 0 ? nthreads : 1, S));
    auto worker = [&]() {
        for (;;) {
            int32_t a = next.fetch_add(1);
            if (a >= S) break;
            fm_state* st = nullptr;
            int rc = fm_build_frozen_state_w(g, T + (size_t)a * N, s, src_nodes[a],
                                             n_rcv > 0 ? rcv_nodes + (size_t)a * per_src : nullptr,
                                             n_rcv > 0 && rcv_weights ? rcv_weights + (size_t)a * per_src : nullptr,
                                             n_rcv, k_per_rcv, &st);
            rcs[a] = rc;
            res[a] = st;
            if (rc != FM_OK) msgs[a] = fm_last_error();
        }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; i++) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
    for (int32_t a = 0; a < S; a++) {
        if (rcs[a] != FM_OK) {
            for (auto* p : res) fm_state_free(p);
            fm::set_error("source %d: %s", a, msgs[a].c_str());
            return rcs[a];
        }
    }
    std::copy(res.begin(), res.end(), out);
    return FM_OK;
}

int fm_build_frozen_state_pt(const fm_grid* g, const double* X, const double* T, const double* s,
                             const double* xi_src, double seed_radius, const int64_t* rcv_nodes,
                             const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv, fm_state** out) {
    fm::clear_error();
    if (!out) { fm::set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    if (!g || !xi_src) { fm::set_error("null argument"); return FM_EINVAL; }
    if (g->dim != 2 && g->dim != 3) { fm::set_error("dim must be 2 or 3, got %d", g->dim); return FM_EINVAL; }
    fm::PointSource ps{};
    ps.X = X;
    for (int d = 0; d < g->dim; d++) ps.xi[d] = xi_src[d];
    ps.rho = seed_radius;
    return fm::build_state(g, T, s, -1, rcv_nodes, rcv_weights, n_rcv, k_per_rcv, out, &ps);
}

int fm_build_frozen_states_pt(const fm_grid* g, const double* X, int32_t S, const double* T, const double* s,
                              const double* xi_src, double seed_radius, const int64_t* rcv_nodes,
                              const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv, int32_t nthreads,
                              fm_state** out) {
    fm::clear_error();
    if (!g || !T || !s || !xi_src || !out || S < 1) { fm::set_error("bad arguments"); return FM_EINVAL; }
    if (g->dim != 2 && g->dim != 3) { fm::set_error("dim must be 2 or 3, got %d", g->dim); return FM_EINVAL; }
    if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1) { fm::set_error("grid sizes must be >= 1"); return FM_EINVAL; }
    if (k_per_rcv < 1) { fm::set_error("entries per receiver must be >= 1"); return FM_EINVAL; }
    const int64_t N = g->n1 * g->n2 * g->n3;
    const size_t per_src = (size_t)(n_rcv > 0 ? n_rcv : 0) * (size_t)k_per_rcv;
    std::vector<fm_state*> res(S, nullptr);
    std::vector<int> rcs(S, FM_OK);
    std::vector<std::string> msgs(S);
    std::atomic<int32_t> next{0};
    int nt = std::max(1, std::min<int32_t>(nthreads > 0 ? nthreads : 1, S));
    auto worker = [&]() {
        for (;;) {
            int32_t a = next.fetch_add(1);
            if (a >= S) break;
            fm_state* st = nullptr;
            int rc = fm_build_frozen_state_pt(g, X, T + (size_t)a * N, s, xi_src + (size_t)a * g->dim, seed_radius,
                                              n_rcv > 0 ? rcv_nodes + (size_t)a * per_src : nullptr,
                                              n_rcv > 0 && rcv_weights ? rcv_weights + (size_t)a * per_src : nullptr,
                                              n_rcv, k_per_rcv, &st);
            rcs[a] = rc;
            res[a] = st;
            if (rc != FM_OK) msgs[a] = fm_last_error();
        }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; i++) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
    for (int32_t a = 0; a < S; a++) {
        if (rcs[a] != FM_OK) {
            for (auto* p : res) fm_state_free(p);
            fm::set_error("source %d: %s", a, msgs[a].c_str());
            return rcs[a];
        }
    }
    std::copy(res.begin(), res.end(), out);
    return FM_OK;
}

int fm_set_iterative_block_min(int32_t k_min) {
    fm::clear_error();
    if (k_min == 1) { fm::set_error("a block has at least 2 nodes: k_min must be >= 2, 0 or negative"); return FM_EINVAL; }
    fm::set_iterative_min(k_min);
    return FM_OK;
}

int fm_state_stats(const fm_state* st, fm_stats* out) {
    fm::clear_error();
    if (!st || !out) { fm::set_error("null argument"); return FM_EINVAL; }
    *out = st->stats;
    return FM_OK;
}

int fm_state_export_operator(const fm_state* st, int64_t* rowptr, int32_t* col, double* w, double* c) {
    fm::clear_error();
    if (!st) { fm::set_error("null state"); return FM_EINVAL; }
    const int nslot = st->nslot();
    int64_t e = 0;
    for (int64_t p = 0; p < st->N; p++) {
        if (rowptr) rowptr[p] = e;
        // neighbours in ascending node id: face slots -z, -y, -x, +x, +y, +z;
        // cube slots are already in that order
        static const int order3[6] = {4, 2, 0, 1, 3, 5};
        static const int order2[4] = {2, 0, 1, 3};
        const int* order = st->dim == 3 ? order3 : order2;
        for (int q = 0; q < nslot; q++) {
            int slot = st->stencil == 26 ? q : order[q];
            if (!(st->pmask[p] & (1u << slot))) continue;
            if (col) col[e] = (int32_t)st->neighbour(p, slot);
            if (w) w[e] = st->weight(p, slot);
            e++;
        }
    }
    if (rowptr) rowptr[st->N] = e;
    if (c) std::memcpy(c, st->cal.data(), sizeof(double) * st->N);
    return FM_OK;
}

int fm_state_export_graph(const fm_state* st, int32_t* comp, int32_t* level_fwd, int32_t* level_rev) {
    fm::clear_error();
    if (!st) { fm::set_error("null state"); return FM_EINVAL; }
    for (int64_t p = 0; p < st->N; p++) {
        int32_t c = st->comp[p];
        if (comp) comp[p] = c;
        if (level_fwd) level_fwd[p] = st->clev_f[c];
        if (level_rev) level_rev[p] = st->clev_r[c];
    }
    return FM_OK;
}

void fm_state_free(fm_state* st) {
    if (!st) return;
    fm::free_device_state(st);
    delete st;
}

int fm_batch_create(fm_state* const* states, int32_t S, int32_t B, int32_t precision, const fm_tuning* tuning,
                    void* hip_stream, fm_batch** out) {
    fm::clear_error();
    return fm::batch_create(states, S, B, precision, tuning, hip_stream, out);
}

int fm_batch_set_stream(fm_batch* b, void* hip_stream) {
    fm::clear_error();
    return fm::batch_set_stream(b, hip_stream);
}

int fm_batch_tuning(const fm_batch* b, fm_tuning* out) {
    fm::clear_error();
    return fm::batch_tuning(b, out);
}

int fm_batch_status(fm_batch* b) {
    fm::clear_error();
    return fm::batch_status(b);
}

int fm_autotune(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* hip_stream,
                const void* ds, int32_t ds_mode, void* j_out, int32_t out_mode, const void* w, int32_t w_mode,
                void* jt_out, int32_t jt_mode, int32_t reps, const char* cache_path, fm_tuning* best,
                fm_tuning* candidates, float* ms, int32_t max_out, int32_t* n_out) {
    fm::clear_error();
    return fm::autotune(states, S, B, precision, hip_stream, ds, ds_mode, j_out, out_mode, w, w_mode, jt_out, jt_mode,
                        reps, cache_path, best, candidates, ms, max_out, n_out);
}

int fm_batch_split_info(fm_batch* b, int32_t* xcd_masks) {
    fm::clear_error();
    return fm::batch_split_info(b, xcd_masks);
}

int fm_apply_J(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode) {
    fm::clear_error();
    return fm::apply_J(b, ds, ds_mode, out, out_mode);
}

int fm_apply_J_static(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* hip_stream,
                      const void* ds, int32_t ds_mode, void* out, int32_t out_mode) {
    fm::clear_error();
    return fm::apply_J_static(states, S, B, precision, hip_stream, ds, ds_mode, out, out_mode);
}

int fm_apply_JT(fm_batch* b, const void* w, int32_t w_mode, void* out, int32_t out_mode) {
    fm::clear_error();
    return fm::apply_JT(b, w, w_mode, out, out_mode);
}

int fm_apply_J_sweep(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode,
                     int32_t max_cycles, int32_t* cycles) {
    fm::clear_error();
    return fm::apply_J_sweep(b, ds, ds_mode, out, out_mode, max_cycles, cycles);
}

int fm_apply_JT_sweep(fm_batch* b, const void* w, void* out, int32_t out_mode, int32_t max_cycles,
                      int32_t* cycles) {
    fm::clear_error();
    return fm::apply_JT_sweep(b, w, out, out_mode, max_cycles, cycles);
}

int fm_lsqr_create(fm_batch* b, fm_lsqr** out) {
    fm::clear_error();
    return fm::lsqr_create(b, out);
}

int fm_lsqr_start(fm_lsqr* L, const void* d) {
    fm::clear_error();
    return fm::lsqr_start_any(L, d);
}

int fm_lsqr_iterate(fm_lsqr* L, int32_t n) {
    fm::clear_error();
    return fm::lsqr_iterate_any(L, n);
}

int fm_lsqr_capture(fm_lsqr* L, int32_t n) {
    fm::clear_error();
    return fm::lsqr_capture(L, n);
}

int fm_lsqr_replay(fm_lsqr* L) {
    fm::clear_error();
    return fm::lsqr_replay(L);
}

int fm_lsqr_buffers(const fm_lsqr* L, void** x, void** u, void** v, double** scalars) {
    fm::clear_error();
    return fm::lsqr_buffers(L, x, u, v, scalars);
}

int fm_cgls_create(fm_batch* b, int32_t max_iter, fm_cgls** out) {
    fm::clear_error();
    return fm::cgls_create(b, max_iter, out);
}

int fm_cgls_start(fm_cgls* C, const void* d) {
    fm::clear_error();
    return fm::cgls_start_any(C, d);
}

int fm_cgls_iterate(fm_cgls* C, int32_t n) {
    fm::clear_error();
    return fm::cgls_iterate_any(C, n);
}

int fm_cgls_capture(fm_cgls* C, int32_t n) {
    fm::clear_error();
    return fm::cgls_capture(C, n);
}

int fm_cgls_replay(fm_cgls* C) {
    fm::clear_error();
    return fm::cgls_replay(C);
}

int fm_cgls_buffers(const fm_cgls* C, void** x, void** r, double** scalars, double** history) {
    fm::clear_error();
    return fm::cgls_buffers(C, x, r, scalars, history);
}

void fm_cgls_free(fm_cgls* C) { fm::cgls_free(C); }

void fm_lsqr_free(fm_lsqr* L) { fm::lsqr_free(L); }

void fm_batch_free(fm_batch* b) { fm::batch_free(b); }

const char* fm_last_error(void) { return fm::g_err; }

}  // extern "C"
