// Comparison baseline: directional Gauss-Seidel sweeping of the frozen
// transport on the GPU (Section 3.6, repeated directional sweeping as a
// stationary matrix splitting).  Included by device.hip only.
//
// It solves the same systems as the condensation-DAG traversal but the way
// the sweeping prior art does: no graph analysis, every right-hand side swept
// over the 2^dim axis orderings until a whole cycle changes no entry by more
// than tol * max|x|.  Under one ordering the nodes of a hyperplane
// a + b + c = h (coordinates flipped per ordering) depend only on the previous
// hyperplane, so a workgroup updates a hyperplane in parallel and then moves
// on - exactly the Gauss-Seidel pass with the newest values.  One workgroup
// owns one (source, group of RG right-hand sides), as in the main kernels.
#pragma once

namespace fm {

struct NatDev {
    const uint64_t* fmeta;   // natural-order records of W (predecessors)
    const void* frec;
    const uint64_t* rmeta;   // natural-order records of W^T (successors)
    const void* rrec;
};

struct GsArgs {
    ApplyArgs a;
    const NatDev* nat;
    int32_t max_cycles;
    double tol;
    int32_t* cycles;         // [items]: cycles used, negative when not converged
    int32_t m0, m1, m2;      // nodes per logical axis (2-D: n1, n3, 1)
    int32_t dim;
};

template <int DIR, typename V, int RG, int VW, int NT>
__global__ __launch_bounds__(NT) void k_gs_sweep(GsArgs g) {
    constexpr int LPN = RG / VW;
    constexpr int SLOTS = NT / LPN;
    const ApplyArgs& a = g.a;
    int alpha, grp, item;
    {
        const int w = blockIdx.x;
        item = a.xcd_aware ? (w % 8) * a.per_xcd + (w / 8) : w;
        if (item >= a.items) return;
        alpha = item / a.ngroups;
        grp = item - alpha * a.ngroups;
    }
    __shared__ unsigned long long red[2 * RG];
    __shared__ int done;
    const NatDev nd = g.nat[alpha];
    const uint64_t* __restrict__ meta = DIR == kFwd ? nd.fmeta : nd.rmeta;
    const V* __restrict__ wts = (const V*)(DIR == kFwd ? nd.frec : nd.rrec);
    const V* __restrict__ ovf_base = wts + a.N * 4;
    const SrcDev sd = a.src[alpha];
    const int sub = threadIdx.x % LPN;
    const int slot0 = threadIdx.x / LPN;
    const int64_t NB = a.N * a.B;
    Ctx cx;
    cx.B = a.B;
    cx.rhs0 = grp * RG + sub * VW;
    cx.R = a.R;
    cx.st1 = a.st1;
    cx.st2 = a.st2;
    cx.N = a.N;
    cx.rcv_in = false;
    cx.cube = false;          // face-stencil states only
    const V* __restrict__ in = (const V*)a.in +
        ((DIR == kFwd && a.in_mode == FM_DS_BROADCAST) ? 0 : (size_t)alpha * NB);
    V* __restrict__ X = (V*)a.work + (size_t)alpha * NB;
    LevelDesc none{0, 0, 0, 0, 0, 0};

    Pack<V, VW> zero;
#pragma unroll
    for (int v = 0; v < VW; ++v) zero.v[v] = (V)0;
    for (int64_t n = slot0; n < a.N; n += SLOTS) st<V, VW>(X + n * cx.B + cx.rhs0, zero);
    const int H = (g.m0 - 1) + (g.m1 - 1) + (g.m2 - 1);
    int cyc = 1;
    bool converged = false;
    for (; cyc <= g.max_cycles; ++cyc) {
        if (threadIdx.x < 2 * RG) red[threadIdx.x] = 0ull;
        double dmax[VW], xmax[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) dmax[v] = xmax[v] = 0.0;
        __syncthreads();
        for (int o = 0; o < (1 << g.dim); ++o) {
            for (int h = 0; h <= H; ++h) {
                const int cmin = max(0, h - (g.m0 - 1) - (g.m1 - 1));
                const int cmax = min(g.m2 - 1, h);
                const int rows = cmax - cmin + 1;
                for (int idx = slot0; idx < rows * g.m1; idx += SLOTS) {
                    const int c = cmin + idx / g.m1;
                    const int b = idx % g.m1;
                    const int aa = h - b - c;
                    if (aa < 0 || aa >= g.m0) continue;
                    const int i = (o & 1) ? g.m0 - 1 - aa : aa;
                    const int j = (o & 2) ? g.m1 - 1 - b : b;
                    const int k = (o & 4) ? g.m2 - 1 - c : c;
                    const int64_t node = (int64_t)i + (int64_t)g.m0 * ((int64_t)j + (int64_t)g.m1 * k);
                    NodeOps<V, VW> p;
                    fetch_static<DIR, V, VW>(p, meta[node], (int)node, wts, in, cx, sd, none);
                    V res[VW];
                    combine<DIR, V, VW, V>(p, ovf_base, X, cx, res);
                    V* xp = X + node * cx.B + cx.rhs0;
                    const Pack<V, VW> old = ld<V, VW>(xp);
                    Pack<V, VW> o2;
#pragma unroll
                    for (int v = 0; v < VW; ++v) {
                        o2.v[v] = res[v];
                        dmax[v] = fmax(dmax[v], fabs((double)res[v] - (double)old.v[v]));
                        xmax[v] = fmax(xmax[v], fabs((double)res[v]));
                    }
                    st<V, VW>(xp, o2);
                }
                __syncthreads();
            }
        }
        // non-negative doubles order like their bit patterns
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            atomicMax(&red[sub * VW + v], (unsigned long long)__double_as_longlong(dmax[v]));
            atomicMax(&red[RG + sub * VW + v], (unsigned long long)__double_as_longlong(xmax[v]));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int ok = 1;
            for (int rr = 0; rr < RG; ++rr)
                if (!(__longlong_as_double((long long)red[rr]) <= g.tol * __longlong_as_double((long long)red[RG + rr])))
                    ok = 0;
            done = ok;
        }
        __syncthreads();
        converged = done != 0;
        __syncthreads();
        if (converged) break;
    }
    if (g.cycles && threadIdx.x == 0) g.cycles[item] = converged ? cyc : -g.max_cycles;
}

// out[alpha][n][b] = c_alpha[n] * lambda_alpha[n][b]
template <typename V>
__global__ void k_scale_per_source(ApplyArgs a, const void* const* cal) {
    const int64_t NB = a.N * a.B;
    const int64_t total = (int64_t)a.S * NB;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t alpha = t / NB;
        const int64_t node = (t - alpha * NB) / a.B;
        ((V*)a.out)[t] = ((const V*)cal[alpha])[node] * ((const V*)a.work)[t];
    }
}

}  // namespace fm
