// The GPU setup pass (Algorithm 1, Phase I: the frozen states): the couplings of
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
// the couplings equal the host's bit for bit.  Then the graph work: Kahn's
// elimination forward and backward trims every node that is not both on or
// downstream and on or upstream of a cycle (Section 3.5, Proposition 2), the
// host finds the SCCs among the rest only, and the longest-path levels of
// the condensation DAG in both directions come from Kahn's elimination over
// the components on the device (Section 4.1); the host finishes the state
// (block factors, packing) from them.
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

// Successor masks from the predecessor masks: slot b of v is set when the
// neighbour in slot b has v as a predecessor (its opposite slot set).
__global__ void k_setup_smask(SetupDims g, int32_t S, const uint8_t* __restrict__ pmask, uint8_t* __restrict__ smask) {
    const int nslot = 2 * g.dim;
    const int64_t total = (int64_t)S * g.N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t alpha = t / g.N, p = t - alpha * g.N;
        const uint8_t* pm = pmask + alpha * g.N;
        uint8_t m = 0;
        for (int slot = 0; slot < nslot; slot++) {
            const int d = slot >> 1;
            const int64_t c = coord_of(g, p, d);
            if ((slot & 1) ? c + 1 >= g.n[d] : c == 0) continue;
            const int64_t q = (slot & 1) ? p + g.stride[d] : p - g.stride[d];
            if (pm[q] & (1u << (slot ^ 1))) m |= (uint8_t)(1u << slot);
        }
        smask[t] = m;
    }
}

// Kahn's elimination on one source per workgroup (Sections 3.5, 4.1): a
// component whose external in-edges (predecessors for the forward order,
// successors for the reverse one) are all eliminated joins the next
// frontier; the round in which a component leaves the frontier is its
// longest-path level.  Component ids: a node that is its own component has
// its node id, the members of nontrivial component b share the id N + b
// (IDENT: every node is its own component; the elimination then stops at
// the cycles, and the nodes it never reaches keep level -1).  Frontiers are
// compacted per wave: a ballot of the lanes that push, one LDS atomic for
// the wave, and each lane's slot from the count of pushing lanes below it.
struct KahnArgs {
    SetupDims g;
    const uint8_t* pmask;        // predecessor masks [S][N]
    const uint8_t* smask;        // successor masks [S][N]
    const int32_t* cid;          // [N] component id of each node (not IDENT)
    const int32_t* bptr;         // [nblk + 1] members of the nontrivial components
    const int32_t* bmem;
    int32_t nblk;
    int32_t* cnt;                // scratch [S][N + nblk]
    int32_t* f0;
    int32_t* f1;
    int32_t* lev;                // [S][N + nblk] level of each component id (-2: not an id)
};

__device__ __forceinline__ void frontier_push(int32_t* __restrict__ F, int* s_n, bool want, int32_t val) {
    const uint64_t b = __ballot(want);
    if (b == 0) return;
    const int lane = (int)__lane_id();
    const int leader = __ffsll((unsigned long long)b) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(s_n, __popcll(b));
    base = __shfl(base, leader);
    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (want) F[base + below] = val;
}

template <bool REV, bool IDENT>
__device__ __forceinline__ void kahn_run(const KahnArgs& k, int64_t off, int64_t moff) {
    const SetupDims& g = k.g;
    const int64_t N = g.N;
    const int32_t nc = (int32_t)N + (IDENT ? 0 : k.nblk);
    const uint8_t* __restrict__ inm = (REV ? k.smask : k.pmask) + moff;
    const uint8_t* __restrict__ outm = (REV ? k.pmask : k.smask) + moff;
    int32_t* __restrict__ cnt = k.cnt + off;
    int32_t* F = k.f0 + off;
    int32_t* Fn = k.f1 + off;
    int32_t* __restrict__ lev = k.lev + off;
    __shared__ int s_n;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    auto cid_of = [&](int64_t v) -> int32_t { return IDENT ? (int32_t)v : k.cid[v]; };
    // component ids of the neighbours of m along the set bits of b (-1 elsewhere), loads in flight together
    auto nbr_ids = [&](int64_t m, uint32_t b, int32_t cu[6]) {
#pragma unroll
        for (int slot = 0; slot < 6; slot++) {
            cu[slot] = -1;
            if ((b >> slot) & 1u) {
                const int d = slot >> 1;
                cu[slot] = cid_of((slot & 1) ? m + g.stride[d] : m - g.stride[d]);
            }
        }
    };
    // external in-edges per component; the components without any start
    for (int32_t c = threadIdx.x; c - (int32_t)threadIdx.x < nc; c += blockDim.x) {
        bool start = false;
        if (c < nc) {
            int32_t n_in = 0;
            bool own = true;
            int32_t j0 = -1, j1 = 0;     // one member: c itself
            if (c >= N) {
                j0 = k.bptr[c - N];
                j1 = k.bptr[c - N + 1];
            } else if (!IDENT && k.cid[c] != c) {
                own = false;             // a member of a nontrivial component
                j1 = -1;
            }
            for (int32_t j = j0; j < j1; j++) {
                const int64_t m = j < 0 ? c : k.bmem[j];
                int32_t cu[6];
                nbr_ids(m, inm[m], cu);
#pragma unroll
                for (int slot = 0; slot < 6; slot++) n_in += (cu[slot] >= 0 && cu[slot] != c) ? 1 : 0;
            }
            cnt[c] = n_in;
            lev[c] = own ? -1 : -2;
            start = own && n_in == 0;
        }
        frontier_push(F, &s_n, start, c);
    }
    __syncthreads();
    int cur = s_n;
    // KU frontier entries per thread with their loads in flight together
    // (entries, then masks, then the neighbours' component ids, then the
    // counter decrements), so that a round takes a few memory round trips
    // whatever the frontier's size
    constexpr int KU = 4;
    for (int32_t r = 0; cur > 0; r++) {
        __syncthreads();
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        const int step = (int)blockDim.x * KU;
        for (int base = 0; base < cur; base += step) {
            int32_t c[KU];
            bool live[KU];
#pragma unroll
            for (int u = 0; u < KU; u++) {
                const int i = base + u * (int)blockDim.x + (int)threadIdx.x;
                live[u] = i < cur;
                c[u] = live[u] ? F[i] : 0;
            }
            uint32_t mk[KU];
#pragma unroll
            for (int u = 0; u < KU; u++) {
                if (live[u]) lev[c[u]] = r;
                mk[u] = (live[u] && c[u] < N) ? (uint32_t)outm[c[u]] : 0u;     // singletons here, blocks below
            }
            int32_t cu[KU][6];
#pragma unroll
            for (int u = 0; u < KU; u++) nbr_ids(c[u], mk[u], cu[u]);
            bool ready[KU][6];
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int slot = 0; slot < 6; slot++)
                    ready[u][slot] = cu[u][slot] >= 0 && cu[u][slot] != c[u] && atomicSub(cnt + cu[u][slot], 1) == 1;
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int slot = 0; slot < 6; slot++) frontier_push(Fn, &s_n, ready[u][slot], cu[u][slot]);
            // nontrivial components: one member per step, every lane of the
            // wave at the same pushes
            for (int u = 0; u < KU; u++) {
                const bool blk = live[u] && c[u] >= N;
                if (!__any(blk)) continue;
                int32_t j = blk ? k.bptr[c[u] - N] : 0;
                const int32_t j1 = blk ? k.bptr[c[u] - N + 1] : 0;
                for (;;) {
                    const bool has = j < j1;
                    if (!__any(has)) break;
                    int32_t cb[6];
                    bool rb[6];
#pragma unroll
                    for (int slot = 0; slot < 6; slot++) {
                        cb[slot] = 0;
                        rb[slot] = false;
                    }
                    if (has) {
                        const int64_t m = k.bmem[j];
                        nbr_ids(m, outm[m], cb);
#pragma unroll
                        for (int slot = 0; slot < 6; slot++)
                            rb[slot] = cb[slot] >= 0 && cb[slot] != c[u] && atomicSub(cnt + cb[slot], 1) == 1;
                    }
#pragma unroll
                    for (int slot = 0; slot < 6; slot++) frontier_push(Fn, &s_n, rb[slot], cb[slot]);
                    j++;
                }
            }
        }
        __syncthreads();
        cur = s_n;
        int32_t* t = F;
        F = Fn;
        Fn = t;
    }
}

// One source per workgroup, its arrays at the workgroup's offset.
template <bool REV, bool IDENT>
__global__ __launch_bounds__(1024) void k_kahn(KahnArgs k) {
    const int32_t nc = (int32_t)k.g.N + (IDENT ? 0 : k.nblk);
    kahn_run<REV, IDENT>(k, (int64_t)blockIdx.x * nc, (int64_t)blockIdx.x * k.g.N);
}

// Trimming of n sources in one launch: workgroups [0, n) run the forward
// eliminations, [n, 2n) the reverse ones (each direction with counters and
// frontiers of its own, so the two run side by side).
__global__ __launch_bounds__(1024) void k_kahn_trim(KahnArgs kf, KahnArgs kr, int32_t n) {
    const bool rev = (int32_t)blockIdx.x >= n;
    const int64_t off = (int64_t)(rev ? blockIdx.x - n : blockIdx.x) * kf.g.N;
    if (rev) kahn_run<true, true>(kr, off, off);
    else kahn_run<false, true>(kf, off, off);
}

// Several sources' eliminations over their components in one launch: one
// workgroup per job, each with arrays of its own; jobs [0, n) forward,
// [n, 2n) reverse.
__global__ __launch_bounds__(1024) void k_kahn_jobs(const KahnArgs* __restrict__ jobs, int32_t n) {
    const KahnArgs k = jobs[blockIdx.x];
    if ((int32_t)blockIdx.x >= n) kahn_run<true, false>(k, 0, 0);
    else kahn_run<false, false>(k, 0, 0);
}

// Nodes removed by the forward (bit 0) and the reverse (bit 1) elimination.
__global__ void k_trim_flags(int64_t total, const int32_t* __restrict__ lf, const int32_t* __restrict__ lr,
                             uint8_t* __restrict__ flags) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        flags[t] = (uint8_t)((lf[t] >= 0 ? 1 : 0) | (lr[t] >= 0 ? 2 : 0));
}

// The host threads' level eliminations, batched: each thread hands over
// the arguments of its two eliminations (inputs already on the device) and
// waits; the server launches every job pending at that moment in one launch
// per direction, so that the small one-workgroup eliminations of many
// sources run side by side instead of queueing behind each other.
struct LevelServer {
    struct Job {
        KahnArgs f, r;
        bool done = false;
        hipError_t err = hipSuccess;
    };
    std::mutex mu;
    std::condition_variable cv_job, cv_done;
    std::vector<Job*> pending;
    bool stop = false;
    int device = 0;
    std::thread th;
    void run() {
        hipStream_t st = nullptr;
        KahnArgs* dargs = nullptr;
        size_t cap = 0;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        for (;;) {
            std::vector<Job*> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_job.wait(lk, [&]() { return stop || !pending.empty(); });
                if (pending.empty()) break;
                batch.swap(pending);
            }
            const size_t n = batch.size();
            std::vector<KahnArgs> h(2 * n);
            for (size_t i = 0; i < n; i++) {
                h[i] = batch[i]->f;
                h[n + i] = batch[i]->r;
            }
            if (e == hipSuccess && cap < 2 * n) {
                if (dargs) (void)hipFree(dargs);
                dargs = nullptr;
                cap = std::max<size_t>(2 * n, 32);
                e = hipMalloc(&dargs, sizeof(KahnArgs) * cap);
            }
            if (e == hipSuccess) e = hipMemcpyAsync(dargs, h.data(), sizeof(KahnArgs) * 2 * n, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_kahn_jobs, dim3((unsigned)(2 * n)), dim3(1024), 0, st, (const KahnArgs*)dargs,
                                   (int32_t)n);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            {
                std::lock_guard<std::mutex> lk(mu);
                for (Job* j : batch) {
                    j->err = e;
                    j->done = true;
                }
            }
            cv_done.notify_all();
        }
        if (dargs) (void)hipFree(dargs);
        if (st) (void)hipStreamDestroy(st);
    }
    hipError_t submit(Job& j) {
        std::unique_lock<std::mutex> lk(mu);
        pending.push_back(&j);
        cv_job.notify_one();
        cv_done.wait(lk, [&]() { return j.done; });
        return j.err;
    }
    void start(int dev) {
        device = dev;
        th = std::thread([this]() { run(); });
    }
    void finish() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_job.notify_all();
        if (th.joinable()) th.join();
    }
};

// Per host thread: a stream, device buffers and pinned host staging for the
// condensation levels and the records of the states it finishes.
struct LevelCtx {
    LevelServer* server = nullptr;
    SetupDims g;
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t cap = 0;             // N + the most nontrivial components seen
    int32_t *cid = nullptr, *bptr = nullptr, *bmem = nullptr, *cnt = nullptr, *f0 = nullptr, *f1 = nullptr,
            *lf = nullptr, *lr = nullptr;
    int32_t *cnt_r = nullptr, *f0_r = nullptr, *f1_r = nullptr;   // the reverse elimination's own
    uint8_t *pm = nullptr, *sm = nullptr;
    char* host = nullptr;        // pinned: cid, masks, block lists in; levels out
    // records: placement, components, weights, calibration, receiver flags,
    // external masks, overflow counts and their block sums
    int32_t *pos = nullptr, *comp = nullptr, *bsum = nullptr;
    double *w6 = nullptr, *cal = nullptr;
    uint8_t *rcv = nullptr, *extm = nullptr;
    // the current source's couplings, kept on the device since the couplings
    // pass (not owned)
    const double *src_w6 = nullptr, *src_cal = nullptr;
    const uint8_t* src_pm = nullptr;
    void release() {
        for (void* p : {(void*)cid, (void*)bptr, (void*)bmem, (void*)cnt, (void*)f0, (void*)f1, (void*)lf, (void*)lr,
                        (void*)cnt_r, (void*)f0_r, (void*)f1_r,
                        (void*)pm, (void*)sm, (void*)pos, (void*)comp, (void*)bsum, (void*)w6, (void*)cal, (void*)rcv,
                        (void*)extm})
            if (p) (void)hipFree(p);
        if (host) (void)hipHostFree(host);
        if (stream) (void)hipStreamDestroy(stream);
        cid = bptr = bmem = cnt = f0 = f1 = lf = lr = nullptr;
        cnt_r = f0_r = f1_r = nullptr;
        pm = sm = nullptr;
        pos = comp = bsum = nullptr;
        w6 = cal = nullptr;
        rcv = extm = nullptr;
        host = nullptr;
        stream = nullptr;
        cap = 0;
    }
};

// ---- records on the device (the host's packing format, bit for bit) ----

// External-neighbour masks (a block member lists only neighbours outside
// its component) and the overflow count (neighbours past the third) at each
// node's position.
template <bool FWD>
__global__ void k_pack_count(SetupDims g, const int32_t* __restrict__ pos, const int32_t* __restrict__ comp,
                             const uint8_t* __restrict__ pm, const uint8_t* __restrict__ sm, uint8_t* __restrict__ extm,
                             int32_t* __restrict__ cnt) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * blockDim.x) {
        uint32_t full = FWD ? pm[v] : sm[v], m = 0;
        const int32_t cv = comp[v];
        while (full) {
            const int slot = __builtin_ctz(full);
            full &= full - 1u;
            const int d = slot >> 1;
            const int64_t u = (slot & 1) ? v + g.stride[d] : v - g.stride[d];
            if (comp[u] != cv) m |= 1u << slot;
        }
        extm[v] = (uint8_t)m;
        const int t = __builtin_popcount(m);
        cnt[pos[v]] = t > 3 ? t - 3 : 0;
    }
}

// Exclusive prefix sums of cnt in place, blocks of 1024 (block totals to bsum).
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t* __restrict__ cnt, int64_t n, int32_t* __restrict__ bsum) {
    __shared__ int32_t t[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int32_t x = i < n ? cnt[i] : 0;
    t[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t y = threadIdx.x >= (unsigned)o ? t[threadIdx.x - o] : 0;
        __syncthreads();
        t[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) cnt[i] = t[threadIdx.x] - x;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = t[1023];
}

// The block totals scanned by one workgroup (exclusive; the grand total after them).
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t* __restrict__ bsum, int32_t nb) {
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t b0 = 0; b0 < nb; b0 += 1024) {
        __shared__ int32_t t[1024];
        const int32_t i = b0 + (int32_t)threadIdx.x;
        const int32_t x = i < nb ? bsum[i] : 0;
        t[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t y = threadIdx.x >= (unsigned)o ? t[threadIdx.x - o] : 0;
            __syncthreads();
            t[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + t[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += t[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

// Meta words and value records: [c, w1, w2, w3] per position (unused
// entries 0), further weights in the overflow area after the N records;
// reverse records list successors u with weight w_{u,v} and mark receivers.
template <bool FWD>
__global__ void k_pack_write(SetupDims g, const int32_t* __restrict__ pos, const uint8_t* __restrict__ extm,
                             const int32_t* __restrict__ off, const int32_t* __restrict__ bsum,
                             const double* __restrict__ w6, const double* __restrict__ cal,
                             const uint8_t* __restrict__ rcv, uint64_t* __restrict__ meta, double* __restrict__ wts) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = pos[v];
        const uint32_t mask = extm[v];
        const int64_t o = __builtin_popcount(mask) > 3 ? (int64_t)off[q] + bsum[q >> 10] : 0;
        double* rec = wts + q * 4;
        rec[0] = cal[v];
        double r[3] = {0.0, 0.0, 0.0};
        uint32_t m = mask;
        for (int t = 0; m; t++) {
            const int slot = __builtin_ctz(m);
            m &= m - 1u;
            const int d = slot >> 1;
            const int64_t u = (slot & 1) ? v + g.stride[d] : v - g.stride[d];
            const double w = FWD ? w6[v * 6 + slot] : w6[u * 6 + (slot ^ 1)];
            if (t < 3) r[t] = w;
            else wts[g.N * 4 + o + (t - 3)] = w;
        }
        rec[1] = r[0];
        rec[2] = r[1];
        rec[3] = r[2];
        meta[q] = (uint64_t)(uint32_t)v | ((uint64_t)o << kOffShift) | ((uint64_t)mask << kMaskShift) |
                  (!FWD && rcv[v] ? kRcvFlag : 0ull);
    }
}

int device_pack(void* ctxp, bool fwd, int64_t N, const int32_t* pos_of, const int32_t* comp, const uint32_t* pmask,
                const uint32_t* smask, const double* w6, const double* cal, const uint8_t* rcvflag,
                Packed::DeviceRecords* out) {
    LevelCtx& x = *static_cast<LevelCtx*>(ctxp);
    hipError_t e = hipSuccess;
    if (!x.stream) e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
    const int64_t nb = (N + 1023) / 1024;
    if (e == hipSuccess && !x.pos) {
        e = hipMalloc(&x.pos, sizeof(int32_t) * (size_t)N);
        if (e == hipSuccess) e = hipMalloc(&x.comp, sizeof(int32_t) * (size_t)N);
        if (e == hipSuccess) e = hipMalloc(&x.bsum, sizeof(int32_t) * (size_t)(nb + 1));
        if (e == hipSuccess && !x.src_w6) e = hipMalloc(&x.w6, sizeof(double) * 6 * (size_t)N);
        if (e == hipSuccess && !x.src_cal) e = hipMalloc(&x.cal, sizeof(double) * (size_t)N);
        if (e == hipSuccess) e = hipMalloc(&x.rcv, (size_t)N);
        if (e == hipSuccess) e = hipMalloc(&x.extm, (size_t)N);
        if (e == hipSuccess && !x.pm) e = hipMalloc(&x.pm, (size_t)N);
        if (e == hipSuccess && !x.sm) e = hipMalloc(&x.sm, (size_t)N);
        if (e == hipSuccess && !x.cnt) e = hipMalloc(&x.cnt, sizeof(int32_t) * (size_t)N);
    }
    hipStream_t s = x.stream;
    const int d = fwd ? 0 : 1;
    std::vector<uint8_t> m8;
    const double* dw6 = x.src_w6 ? x.src_w6 : x.w6;
    const double* dcal = x.src_cal ? x.src_cal : x.cal;
    if (e == hipSuccess && fwd) {
        // per state, with the forward direction (always packed first); the
        // masks (made by the level pass) and the couplings are on the device
        // already when the couplings pass kept them there
        if (!x.src_pm) {
            m8.resize(2 * (size_t)N);
            for (int64_t v = 0; v < N; v++) {
                m8[v] = (uint8_t)pmask[v];
                m8[N + v] = (uint8_t)smask[v];
            }
            e = hipMemcpyAsync(x.pm, m8.data(), (size_t)N, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(x.sm, m8.data() + N, (size_t)N, hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(x.comp, comp, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !x.src_w6)
            e = hipMemcpyAsync(x.w6, w6, sizeof(double) * 6 * (size_t)N, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !x.src_cal)
            e = hipMemcpyAsync(x.cal, cal, sizeof(double) * (size_t)N, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(x.rcv, rcvflag, (size_t)N, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(x.pos, pos_of, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, s);
    const int grid = (int)std::min<int64_t>((N + 255) / 256, 65535);
    if (e == hipSuccess) {
        if (fwd) hipLaunchKernelGGL(k_pack_count<true>, dim3(grid), dim3(256), 0, s, x.g, x.pos, x.comp, x.pm, x.sm, x.extm, x.cnt);
        else hipLaunchKernelGGL(k_pack_count<false>, dim3(grid), dim3(256), 0, s, x.g, x.pos, x.comp, x.pm, x.sm, x.extm, x.cnt);
        hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(1024), 0, s, x.cnt, N, x.bsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, x.bsum, (int32_t)nb);
        e = hipGetLastError();
    }
    int32_t total = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&total, x.bsum + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && (int64_t)total > (int64_t)kOffMask + 1) {
        set_error("state too large for the packed format: record overflow area too large");
        return FM_EINVAL;
    }
    const int64_t nw = 4 * N + total + 4;
    if (e == hipSuccess) e = hipMalloc(&out->meta[d], sizeof(uint64_t) * (size_t)N);
    if (e == hipSuccess) e = hipMalloc(&out->wts[d], sizeof(double) * (size_t)nw);
    if (e == hipSuccess) e = hipMemsetAsync((double*)out->wts[d] + (nw - 4), 0, 4 * sizeof(double), s);
    if (e == hipSuccess) {
        if (fwd)
            hipLaunchKernelGGL(k_pack_write<true>, dim3(grid), dim3(256), 0, s, x.g, x.pos, x.extm, x.cnt, x.bsum, dw6,
                               dcal, x.rcv, (uint64_t*)out->meta[d], (double*)out->wts[d]);
        else
            hipLaunchKernelGGL(k_pack_write<false>, dim3(grid), dim3(256), 0, s, x.g, x.pos, x.extm, x.cnt, x.bsum,
                               dw6, dcal, x.rcv, (uint64_t*)out->meta[d], (double*)out->wts[d]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("GPU setup pass (records): %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    out->nwts[d] = nw;
    out->device = x.device;
    return FM_OK;
}

int device_levels(void* ctxp, int64_t N, int32_t ncomp, const int32_t* comp, const int32_t* cptr, const int32_t* cnodes,
                  const uint32_t* pmask, const uint32_t* smask, int32_t* clev_f, int32_t* clev_r) {
    LevelCtx& x = *static_cast<LevelCtx*>(ctxp);
    // component ids for the device: node ids for singletons, N + b for the
    // b-th nontrivial component (in comp order)
    int32_t nblk = 0;
    int64_t nmem = 0;
    for (int32_t c = 0; c < ncomp; c++)
        if (cptr[c + 1] - cptr[c] > 1) {
            nblk++;
            nmem += cptr[c + 1] - cptr[c];
        }
    const int64_t need = N + nblk;
    hipError_t e = hipSuccess;
    if (!x.stream) e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
    if (e == hipSuccess && x.cap < need) {
        const int64_t cap = std::max<int64_t>(need, N + N / 64 + 64);
        x.release();
        e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
        x.cap = cap;
        for (int32_t** p : {&x.cid, &x.bmem, &x.cnt, &x.f0, &x.f1, &x.lf, &x.lr, &x.cnt_r, &x.f0_r, &x.f1_r})
            if (e == hipSuccess) e = hipMalloc(p, sizeof(int32_t) * (size_t)cap);
        if (e == hipSuccess) e = hipMalloc(&x.bptr, sizeof(int32_t) * ((size_t)cap + 1));
        if (e == hipSuccess) e = hipMalloc(&x.pm, (size_t)N);
        if (e == hipSuccess) e = hipMalloc(&x.sm, (size_t)N);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.host, sizeof(int32_t) * (size_t)(4 * cap + 2) + 2 * (size_t)N);
    }
    if (e != hipSuccess) {
        set_error("GPU setup pass (levels): %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    int32_t* h_cid = (int32_t*)x.host;                 // [N]
    int32_t* h_bptr = h_cid + N;                        // [nblk + 1]
    int32_t* h_bmem = h_bptr + (nblk + 1);              // [nmem]
    uint8_t* h_pm = (uint8_t*)(h_bmem + nmem);          // [N]
    uint8_t* h_sm = h_pm + N;                           // [N]
    int32_t* h_lf = (int32_t*)x.host;                   // out: [need] twice, after the inputs are consumed
    int32_t* h_lr = h_lf + need;
    {
        int32_t b = 0;
        h_bptr[0] = 0;
        for (int32_t c = 0; c < ncomp; c++) {
            const int32_t k = cptr[c + 1] - cptr[c];
            if (k == 1) {
                h_cid[cnodes[cptr[c]]] = cnodes[cptr[c]];
                continue;
            }
            for (int32_t j = cptr[c]; j < cptr[c + 1]; j++) {
                h_cid[cnodes[j]] = (int32_t)N + b;
                h_bmem[h_bptr[b] + (j - cptr[c])] = cnodes[j];
            }
            h_bptr[b + 1] = h_bptr[b] + k;
            b++;
        }
        if (!x.src_pm)
            for (int64_t v = 0; v < N; v++) {
                h_pm[v] = (uint8_t)pmask[v];
                h_sm[v] = (uint8_t)smask[v];
            }
    }
    hipStream_t s = x.stream;
    e = hipMemcpyAsync(x.cid, h_cid, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(x.bptr, h_bptr, sizeof(int32_t) * ((size_t)nblk + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nmem) e = hipMemcpyAsync(x.bmem, h_bmem, sizeof(int32_t) * (size_t)nmem, hipMemcpyHostToDevice, s);
    if (x.src_pm) {
        // the masks from the source's couplings on the device
        const int grid = (int)std::min<int64_t>((N + 255) / 256, 65535);
        if (e == hipSuccess) e = hipMemcpyAsync(x.pm, x.src_pm, (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_setup_smask, dim3(grid), dim3(256), 0, s, x.g, 1, x.pm, x.sm);
            e = hipGetLastError();
        }
    } else {
        if (e == hipSuccess) e = hipMemcpyAsync(x.pm, h_pm, (size_t)N, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(x.sm, h_sm, (size_t)N, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) {
        KahnArgs k{};
        k.g = x.g;
        k.pmask = x.pm;
        k.smask = x.sm;
        k.cid = x.cid;
        k.bptr = x.bptr;
        k.bmem = x.bmem;
        k.nblk = nblk;
        k.cnt = x.cnt;
        k.f0 = x.f0;
        k.f1 = x.f1;
        if (x.server) {
            // inputs on the device first, then the batched eliminations
            e = hipStreamSynchronize(s);
            LevelServer::Job job;
            job.f = k;
            job.f.lev = x.lf;
            job.r = k;
            job.r.cnt = x.cnt_r;
            job.r.f0 = x.f0_r;
            job.r.f1 = x.f1_r;
            job.r.lev = x.lr;
            if (e == hipSuccess) e = x.server->submit(job);
        } else {
            k.lev = x.lf;
            hipLaunchKernelGGL((k_kahn<false, false>), dim3(1), dim3(1024), 0, s, k);
            k.lev = x.lr;
            hipLaunchKernelGGL((k_kahn<true, false>), dim3(1), dim3(1024), 0, s, k);
            e = hipGetLastError();
        }
    }
    // the inputs in the staging area are consumed once the kernels have run
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_lf, x.lf, sizeof(int32_t) * (size_t)need, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_lr, x.lr, sizeof(int32_t) * (size_t)need, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("GPU setup pass (levels): %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    int32_t b = 0;
    for (int32_t c = 0; c < ncomp; c++) {
        const int32_t id = cptr[c + 1] - cptr[c] > 1 ? (int32_t)N + b++ : cnodes[cptr[c]];
        clev_f[c] = h_lf[id];
        clev_r[c] = h_lr[id];
        if (clev_f[c] < 0 || clev_r[c] < 0) {
            set_error("GPU setup pass: component %d was never eliminated (the partition leaves a cycle)", c);
            return FM_EHIP;
        }
    }
    return FM_OK;
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
    // (couplings 57 bytes per node, the eliminations' masks, counters,
    // frontiers and levels 22 more, the reverse elimination's own counters
    // and frontiers 12 more outside this budget)
    const int32_t chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t)(2LL << 30) / (N * 79)));
    double *dG = nullptr, *ds = nullptr, *dw = nullptr, *dc = nullptr;
    uint8_t *dm = nullptr, *dsm = nullptr, *dtr = nullptr;
    int32_t *dcnt = nullptr, *df0 = nullptr, *df1 = nullptr, *dlf = nullptr, *dlr = nullptr;
    int32_t *dcnt_r = nullptr, *df0_r = nullptr, *df1_r = nullptr;
    int64_t* dsrc = nullptr;
    unsigned long long* dnv = nullptr;
    int* dbad = nullptr;
    char* hst = nullptr;         // pinned staging of one chunk's couplings and trim flags
    int dev = 0;
    std::vector<LevelCtx> lctx(nt);
    LevelServer server;
    for (LevelCtx& x : lctx) {
        x.g = d;
        x.server = &server;
    }
    auto release = [&]() {
        for (void* p : {(void*)dG, (void*)ds, (void*)dw, (void*)dc, (void*)dm, (void*)dsrc, (void*)dnv, (void*)dbad,
                        (void*)dsm, (void*)dtr, (void*)dcnt, (void*)df0, (void*)df1, (void*)dlf, (void*)dlr,
                        (void*)dcnt_r, (void*)df0_r, (void*)df1_r})
            if (p) (void)hipFree(p);
        for (LevelCtx& x : lctx) x.release();
        if (hst) (void)hipHostFree(hst);
    };
    hipError_t e = hipGetDevice(&dev);
    for (LevelCtx& x : lctx) x.device = dev;
    if (e == hipSuccess) e = hipMalloc(&dG, sizeof(double) * (size_t)N * d.ncomp_g);
    if (e == hipSuccess) e = hipMalloc(&ds, sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = hipMalloc(&dw, sizeof(double) * 6 * (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dc, sizeof(double) * (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dm, (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dsm, (size_t)N * chunk);
    if (e == hipSuccess) e = hipMalloc(&dtr, (size_t)N * chunk);
    for (int32_t** p : {&dcnt, &df0, &df1, &dlf, &dlr, &dcnt_r, &df0_r, &df1_r})
        if (e == hipSuccess) e = hipMalloc(p, sizeof(int32_t) * (size_t)N * chunk);
    if (e == hipSuccess) e = hipHostMalloc((void**)&hst, (size_t)N * chunk * (2 + 7 * sizeof(double)));
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
        std::vector<uint8_t> m, t;
        std::vector<double> w, c;
        void* dev = nullptr;     // device copy of w [N][6], c [N], m [N] for the host thread's device work
    };
    std::vector<Couplings> buf(S);
    // device copies of the couplings, recycled between sources
    std::mutex pool_mu;
    std::vector<void*> pool_free, pool_all;
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
    auto worker = [&](int id) {
        if (hipSetDevice(dev) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
            return;
        }
        for (;;) {
            int32_t a;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&]() { return stop || next.load() < ready || next.load() >= S; });
                if (next.load() >= S || (stop && next.load() >= ready)) return;
                a = next.fetch_add(1);
            }
            Assembled pre{buf[a].m.data(), buf[a].w.data(), buf[a].c.data(), (int64_t)nv[a]};
            pre.trim = buf[a].t.data();
            pre.levels = device_levels;
            pre.pack = device_pack;
            pre.ctx = &lctx[id];
            if (buf[a].dev) {
                lctx[id].src_w6 = (const double*)buf[a].dev;
                lctx[id].src_cal = lctx[id].src_w6 + (size_t)N * 6;
                lctx[id].src_pm = (const uint8_t*)(lctx[id].src_cal + (size_t)N);
            } else {
                lctx[id].src_w6 = lctx[id].src_cal = nullptr;
                lctx[id].src_pm = nullptr;
            }
            fm_state* stt = nullptr;
            const int r = build_state(g, nullptr, s, src_nodes[a],
                                      n_rcv > 0 ? rcv_nodes + (size_t)a * per_src : nullptr,
                                      n_rcv > 0 && rcv_weights ? rcv_weights + (size_t)a * per_src : nullptr,
                                      n_rcv, k_per_rcv, &stt, nullptr, &pre);
            rcs[a] = r;
            res[a] = stt;
            if (r != FM_OK) msgs[a] = fm_last_error();
            std::vector<uint8_t>().swap(buf[a].m);
            std::vector<uint8_t>().swap(buf[a].t);
            if (buf[a].dev) {
                // back to the pool (a hipFree here would wait for the whole device)
                std::lock_guard<std::mutex> lk(pool_mu);
                pool_free.push_back(buf[a].dev);
                buf[a].dev = nullptr;
            }
            lctx[id].src_w6 = lctx[id].src_cal = nullptr;
            lctx[id].src_pm = nullptr;
            std::vector<double>().swap(buf[a].w);
            std::vector<double>().swap(buf[a].c);
        }
    };
    server.start(dev);
    std::vector<std::thread> th;
    for (int i = 0; i < nt; i++) th.emplace_back(worker, i);
    int rc = FM_OK;
    std::string msg;
    // the device work of one chunk: couplings, successor masks, trimming
    auto launch_chunk = [&](int32_t a0) {
        const int32_t n = std::min(chunk, S - a0);
        const int64_t total = (int64_t)n * N;
        const int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        hipLaunchKernelGGL(k_setup_couplings, dim3(grid), dim3(256), 0, st, d, n, dG, T_dev + (size_t)a0 * N, ds,
                           dsrc + a0, dw, dm, dc, dnv + a0, dbad + a0);
        // trimming: Kahn's elimination forward and backward, one workgroup
        // per source; the nodes neither removes hold every cycle
        hipLaunchKernelGGL(k_setup_smask, dim3(grid), dim3(256), 0, st, d, n, dm, dsm);
        KahnArgs kf{};
        kf.g = d;
        kf.pmask = dm;
        kf.smask = dsm;
        kf.cnt = dcnt;
        kf.f0 = df0;
        kf.f1 = df1;
        kf.lev = dlf;
        KahnArgs kr = kf;
        kr.cnt = dcnt_r;
        kr.f0 = df0_r;
        kr.f1 = df1_r;
        kr.lev = dlr;
        hipLaunchKernelGGL(k_kahn_trim, dim3((unsigned)(2 * n)), dim3(1024), 0, st, kf, kr, n);
        hipLaunchKernelGGL(k_trim_flags, dim3(grid), dim3(256), 0, st, total, dlf, dlr, dtr);
        return hipGetLastError();
    };
    e = launch_chunk(0);
    for (int32_t a0 = 0; a0 < S; a0 += chunk) {
        const int32_t n = std::min(chunk, S - a0);
        // one copy per array into pinned staging, then into each source's
        // own buffers for the host threads
        uint8_t* hm = (uint8_t*)hst;
        uint8_t* ht = hm + (size_t)chunk * N;
        double* hw = (double*)(ht + (size_t)chunk * N);
        double* hc = hw + (size_t)chunk * N * 6;
        if (e == hipSuccess) e = hipMemcpyAsync(hm, dm, (size_t)n * N, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ht, dtr, (size_t)n * N, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hw, dw, sizeof(double) * 6 * (size_t)n * N, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hc, dc, sizeof(double) * (size_t)n * N, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(nv.data() + a0, dnv + a0, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(bad.data() + a0, dbad + a0, sizeof(int) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            rc = FM_EHIP;
            msg = std::string("GPU setup pass failed: ") + hipGetErrorString(e);
            break;
        }
        // each source's couplings stay on the device for its host thread
        // (their device work then needs no upload); without the memory for
        // it the host thread uploads them
        for (int32_t k = 0; k < n && e == hipSuccess; k++) {
            void* p = nullptr;
            {
                std::lock_guard<std::mutex> lk(pool_mu);
                if (!pool_free.empty()) {
                    p = pool_free.back();
                    pool_free.pop_back();
                }
            }
            if (!p) {
                if (hipMalloc(&p, (size_t)N * (6 * sizeof(double) + sizeof(double) + 1)) != hipSuccess) {
                    (void)hipGetLastError();
                    break;
                }
                std::lock_guard<std::mutex> lk(pool_mu);
                pool_all.push_back(p);
            }
            buf[a0 + k].dev = p;
            e = hipMemcpyAsync(p, dw + (size_t)k * N * 6, sizeof(double) * 6 * (size_t)N, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync((double*)p + (size_t)N * 6, dc + (size_t)k * N, sizeof(double) * (size_t)N,
                                   hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync((double*)p + (size_t)N * 7, dm + (size_t)k * N, (size_t)N, hipMemcpyDeviceToDevice, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        // the next chunk's device work runs while this one is copied out of
        // the staging (one host thread per source)
        if (e == hipSuccess && a0 + chunk < S) e = launch_chunk(a0 + chunk);
        {
            std::vector<std::thread> cps;
            for (int32_t k = 0; k < n; k++)
                cps.emplace_back([&, k]() {
                    Couplings& cp = buf[a0 + k];
                    cp.m.assign(hm + (size_t)k * N, hm + (size_t)(k + 1) * N);
                    cp.t.assign(ht + (size_t)k * N, ht + (size_t)(k + 1) * N);
                    cp.w.assign(hw + (size_t)k * N * 6, hw + (size_t)(k + 1) * N * 6);
                    cp.c.assign(hc + (size_t)k * N, hc + (size_t)(k + 1) * N);
                });
            for (auto& t : cps) t.join();
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
    server.finish();
    for (int32_t a = 0; a < S && rc == FM_OK; a++)
        if (res[a] == nullptr || rcs[a] != FM_OK) {
            rc = rcs[a] != FM_OK ? rcs[a] : FM_EHIP;
            msg = "source " + std::to_string(a) + ": " + msgs[a];
        }
    for (void* p : pool_all) (void)hipFree(p);
    release();
    if (rc != FM_OK) {
        for (auto* p : res) fm_state_free(p);
        set_error("%s", msg.c_str());
        return rc;
    }
    std::copy(res.begin(), res.end(), out);
    return FM_OK;
}
