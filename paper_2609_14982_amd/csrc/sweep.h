// Level-walking kernels for the primal (A x = q) and transpose (A^T y = r)
// traversals of the condensation DAG.  Included by device.hip only.
//
// One workgroup owns one (source, group of RG right-hand sides).  A node's RG
// values are one contiguous segment of the [N][B] vectors; each lane moves VW
// of them with one vector access, so LPN = RG / VW lanes serve a node and a
// workgroup of NT threads covers SLOTS = NT / LPN nodes per pass.  Vector
// accesses matter here: the address unit handles few lanes per clock for
// scattered accesses, so fewer, wider lane accesses per node move more data
// per address-unit cycle.
//
// Every level is processed in batches of SLOTS * U nodes.  Only the
// predecessor (successor) values depend on earlier levels; a node's meta word
// is static, so the next batch's meta words (possibly the next level's) are
// requested before the current batch's operands, and each batch waits on one
// round trip.
#pragma once

namespace fm {

enum : int { kFwd = 0, kRev = 1 };
constexpr int kSlots = 6;   // neighbour slots per node (-x,+x,-y,+y,-z,+z)

struct LevelDesc {
    int p0, nsc, b0, b1, e0, e1;
};

template <int DIR>
__device__ __forceinline__ LevelDesc load_desc(const SrcDev& sd, int l) {
    LevelDesc d;
    if (DIR == kFwd) {
        d.p0 = gld(sd.flvl_ptr + (l));
        d.nsc = gld(sd.flvl_nsc + (l));
        d.b0 = gld(sd.fblk_ptr + (l));
        d.b1 = gld(sd.fblk_ptr + (l + 1));
        d.e0 = d.e1 = 0;
    } else {
        d.p0 = gld(sd.rlvl_ptr + (l));
        d.nsc = gld(sd.rlvl_nsc + (l));
        d.b0 = gld(sd.rblk_ptr + (l));
        d.b1 = gld(sd.rblk_ptr + (l + 1));
        d.e0 = gld(sd.rcvlvl_ptr + (l));
        d.e1 = gld(sd.rcvlvl_ptr + (l + 1));
    }
    return d;
}

// VW consecutive values, aligned for one vector access.
template <typename V, int VW>
struct alignas(sizeof(V) * VW) Pack {
    V v[VW];
};

template <typename V, int VW>
__device__ __forceinline__ Pack<V, VW> ld(const V* p) {
    return *reinterpret_cast<const Pack<V, VW>*>(p);
}

template <typename V, int VW>
__device__ __forceinline__ void st(V* p, const Pack<V, VW>& x) {
    *reinterpret_cast<Pack<V, VW>*>(p) = x;
}

struct Ctx {
    int B, rhs0, R;         // rhs0: first right-hand side of this lane
    int64_t st1, st2;
    int64_t N;
    bool rcv_in;            // transpose input given at receivers
    bool cube;              // cube-stencil records (26-bit masks)
};

__device__ __forceinline__ int64_t slot_off(int slot, int64_t st1, int64_t st2) {
    int64_t st = (slot >> 1) == 0 ? 1 : ((slot >> 1) == 1 ? st1 : st2);
    return (slot & 1) ? st : -st;
}

// Cube-stencil slot b: node offset of the logical offset o in {-1,0,1}^3
// whose base-3 number (o_0 + 1) + 3 (o_1 + 1) + 9 (o_2 + 1), centre left
// out, is b.
__device__ __forceinline__ int64_t cube_slot_off(int slot, int64_t st1, int64_t st2) {
    const int b = slot + (slot >= 13 ? 1 : 0);
    const int o0 = b % 3 - 1, o1 = (b / 3) % 3 - 1, o2 = b / 9 - 1;
    return (int64_t)o0 + (int64_t)o1 * st1 + (int64_t)o2 * st2;
}

// Everything one lane needs for one node of a traversal step.
template <typename V, int VW>
struct NodeOps {
    int64_t node;   // -1 when the slot is empty
    uint32_t mask;
    uint32_t ovf;   // offset of the extra weights (> 3 neighbours)
    Pack<V, 4> rec; // c, w1, w2, w3
    Pack<V, VW> inp;
};

// Static part of a node's operands: record and input values.
template <int DIR, typename V, int VW>
__device__ __forceinline__ void fetch_static(NodeOps<V, VW>& p, uint64_t m, int pos, const V* __restrict__ wts,
                                             const V* __restrict__ in, const Ctx& cx, const SrcDev& sd,
                                             const LevelDesc& d) {
    p.node = (int64_t)(m & kNodeMask);
    if (cx.cube) {
        p.mask = (uint32_t)((m >> kCubeMaskShift) & kCubeMask);
        p.ovf = __builtin_popcount(p.mask) > 3 ? (uint32_t)(DIR == kFwd ? sd.fovf : sd.rovf)[pos] : 0u;
    } else {
        p.ovf = (uint32_t)((m >> kOffShift) & kOffMask);
        p.mask = (uint32_t)(m >> kMaskShift);
    }
    p.rec = ld<V, 4>(wts + (size_t)pos * 4);
    if (DIR == kFwd || !cx.rcv_in) {
        p.inp = ld<V, VW>(in + p.node * cx.B + cx.rhs0);
    } else {
#pragma unroll
        for (int v = 0; v < VW; ++v) p.inp.v[v] = (V)0;
        if (m & kRcvFlag)
            for (int e = d.e0; e < d.e1; ++e)
                if (sd.rcv_pos[e] == pos) {
                    const Pack<V, VW> y = ld<V, VW>(in + (int64_t)sd.rcv_idx[e] * cx.B + cx.rhs0);
                    const V w = (V)sd.rcv_ew[e];
#pragma unroll
                    for (int v = 0; v < VW; ++v) p.inp.v[v] += w * y.v[v];
                }
    }
}

// x_node = c*ds + sum_j w_j x_j (primal) or lambda = r + sum_i w_i lambda_i
// (transpose), neighbours in slot order; T is the accumulation type.
template <int DIR, typename V, int VW, typename T>
__device__ __forceinline__ void combine(const NodeOps<V, VW>& p, const V* __restrict__ ovf_base,
                                        const V* __restrict__ X, const Ctx& cx, T acc[VW]) {
    if (cx.cube) {
        // the k-th set bit (ascending slot) takes the k-th weight
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] = (DIR == kFwd) ? (T)p.rec.v[0] * (T)p.inp.v[v] : (T)p.inp.v[v];
        uint32_t m = p.mask;
        for (int t = 0; m != 0u; ++t) {
            const int s = __builtin_ctz(m);
            m &= m - 1u;
            const Pack<V, VW> x = ld<V, VW>(X + (p.node + cube_slot_off(s, cx.st1, cx.st2)) * cx.B + cx.rhs0);
            const V w = t == 0 ? p.rec.v[1] : (t == 1 ? p.rec.v[2] : (t == 2 ? p.rec.v[3] : ovf_base[p.ovf + (t - 3)]));
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[v] += (T)w * (T)x.v[v];
        }
        return;
    }
    Pack<V, VW> xv[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if ((p.mask >> s) & 1u) xv[s] = ld<V, VW>(X + (p.node + slot_off(s, cx.st1, cx.st2)) * cx.B + cx.rhs0);
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = (DIR == kFwd) ? (T)p.rec.v[0] * (T)p.inp.v[v] : (T)p.inp.v[v];
    // the k-th set mask bit takes the k-th weight: w1..w3 from the record,
    // later ones from the overflow area
    const uint32_t m = p.mask;
    const int n1 = __builtin_popcount(m & 1u), n2 = __builtin_popcount(m & 3u), n3 = __builtin_popcount(m & 7u);
    const int n4 = __builtin_popcount(m & 15u), n5 = __builtin_popcount(m & 31u);
    const int before[kSlots] = {0, n1, n2, n3, n4, n5};
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if ((m >> s) & 1u) {
            const int t = before[s];
            V w;
            if (s < 3 || t < 3) w = t == 0 ? p.rec.v[1] : (t == 1 ? p.rec.v[2] : p.rec.v[3]);
            else w = ovf_base[p.ovf + (t - 3)];
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[v] += (T)w * (T)xv[s].v[v];
        }
    }
}

// One nontrivial SCC block of the current level (all threads take part).
// Phase 1 stages b_C = q_C + sum_ext w x (or r_C + sum_ext w lambda) in LDS,
// phase 2 applies A_C^{-1} (primal) or A_C^{-T} (transpose); each output sums
// in ascending index order whatever the schedule.
template <int DIR, typename V, int RG, int VW, int NT>
__device__ __forceinline__ void block_solve(const SrcDev& sd, int blk, const uint64_t* __restrict__ meta,
                                            const V* __restrict__ wts, const V* __restrict__ in,
                                            V* __restrict__ X, V* __restrict__ outp, const Ctx& cx,
                                            const LevelDesc& d, double* lds, int slot0, int sub) {
    constexpr int LPN = RG / VW;
    constexpr int SLOTS = NT / LPN;
    const V* ovf_base = wts + cx.N * 4;
    const int k = sd.blk_k[blk];
    const int bp = DIR == kFwd ? sd.blk_fpos[blk] : sd.blk_rpos[blk];
    for (int mi = slot0; mi < k; mi += SLOTS) {
        NodeOps<V, VW> p;
        fetch_static<DIR, V, VW>(p, meta[bp + mi], bp + mi, wts, in, cx, sd, d);
        double acc[VW];
        combine<DIR, V, VW, double>(p, ovf_base, X, cx, acc);
#pragma unroll
        for (int v = 0; v < VW; ++v) lds[mi * RG + sub * VW + v] = acc[v];
    }
    __syncthreads();
    const int m_it = sd.blk_it[2 * blk + (DIR == kFwd ? 0 : 1)];
    if (m_it) {
        // a large block solved by its Neumann series (as in the node split):
        // x^0 = b, x^j = b + W_CC x^{j-1} (transpose: W_CC^T), j = 1..m, the
        // iterates in two more LDS buffers of k x RG values, the last one
        // straight to the node rows
        const int64_t sp = sd.blk_sp[blk];
        const int32_t* __restrict__ rp = (DIR == kFwd ? sd.sp_ptr : sd.spt_ptr) + sp;
        const int32_t* __restrict__ cl = DIR == kFwd ? sd.sp_col : sd.spt_col;
        const double* __restrict__ wv = DIR == kFwd ? sd.sp_w : sd.spt_w;
        double* buf[2] = {lds + (size_t)k * RG, lds + (size_t)2 * k * RG};
        const int g0 = cx.rhs0 - sub * VW;
        for (int j = 1; j <= m_it; ++j) {
            const double* cur = j == 1 ? lds : buf[(j - 1) & 1];
            double* nxt = buf[j & 1];
            for (int i = threadIdx.x; i < k; i += NT) {
                double acc[RG];
#pragma unroll
                for (int rr = 0; rr < RG; ++rr) acc[rr] = lds[i * RG + rr];
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    const double w = wv[e];
                    const double* src = cur + (size_t)cl[e] * RG;
#pragma unroll
                    for (int rr = 0; rr < RG; ++rr) acc[rr] += w * src[rr];
                }
                if (j < m_it) {
#pragma unroll
                    for (int rr = 0; rr < RG; ++rr) nxt[i * RG + rr] = acc[rr];
                } else {
                    const int64_t node = (int64_t)(meta[bp + i] & kNodeMask);
                    const V c = wts[(size_t)(bp + i) * 4];
                    V* dst = X + node * cx.B + g0;
#pragma unroll
                    for (int rr = 0; rr < RG; ++rr) dst[rr] = (V)acc[rr];
                    if (DIR == kRev && outp) {
                        V* o = outp + node * cx.B + g0;
#pragma unroll
                        for (int rr = 0; rr < RG; ++rr) o[rr] = c * (V)acc[rr];
                    }
                }
            }
            __syncthreads();
        }
        return;
    }
    // phase 2: thread t owns outputs t, t + NT, ... and all RG right-hand
    // sides of each, so consecutive lanes read consecutive matrix entries:
    // primal x_i = sum_j Minv(i, j) b_j reads the column-major inverse,
    // transpose y_j = sum_i Minv(i, j) b_i reads the row-major copy.
    const double* __restrict__ Mx = DIR == kFwd ? sd.inv + sd.blk_inv[blk] : sd.invt + sd.blk_inv[blk];
    const int g0 = cx.rhs0 - sub * VW;   // first right-hand side of the group
    for (int i = threadIdx.x; i < k; i += NT) {
        double acc[RG];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) acc[rr] = 0.0;
#pragma unroll 4
        for (int j = 0; j < k; ++j) {
            const double m = Mx[(size_t)j * k + i];
#pragma unroll
            for (int rr = 0; rr < RG; ++rr) acc[rr] += m * lds[j * RG + rr];
        }
        const uint64_t m = meta[bp + i];
        const int64_t node = (int64_t)(m & kNodeMask);
        const V c = wts[(size_t)(bp + i) * 4];
        V* dst = X + node * cx.B + g0;
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) dst[rr] = (V)acc[rr];
        if (DIR == kRev && outp) {
            V* o = outp + node * cx.B + g0;
#pragma unroll
            for (int rr = 0; rr < RG; ++rr) o[rr] = c * (V)acc[rr];
        }
    }
    __syncthreads();
}

template <int DIR, typename V, int RG, int VW, int NT, int U>
__global__ __launch_bounds__(NT) void k_sweep(ApplyArgs a) {
    constexpr int LPN = RG / VW;
    constexpr int SLOTS = NT / LPN;
    constexpr int BATCH = SLOTS * U;
    int alpha, grp;
    {
        const int w = blockIdx.x;
        const int item = a.xcd_aware ? (w % 8) * a.per_xcd + (w / 8) : w;
        if (item >= a.items) return;
        alpha = item / a.ngroups;
        grp = item - alpha * a.ngroups;
    }
    extern __shared__ double lds[];
    const SrcDev sd = a.src[alpha];
    const uint64_t* __restrict__ meta = DIR == kFwd ? sd.fmeta : sd.rmeta;
    const V* __restrict__ wts = (const V*)(DIR == kFwd ? sd.fwts : sd.rwts);
    const V* __restrict__ ovf_base = wts + a.N * 4;
    const int L = DIR == kFwd ? sd.L_f : sd.L_r;
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
    cx.rcv_in = DIR == kRev && a.in_mode == FM_W_RECEIVERS;
    cx.cube = a.cube != 0;
    const V* __restrict__ in;
    V* __restrict__ X = (V*)a.work + (size_t)alpha * NB;
    V* __restrict__ outp = nullptr;
    if (DIR == kFwd) {
        in = (const V*)a.in + (a.in_mode == FM_DS_PER_PAIR ? (size_t)alpha * NB : 0);
    } else {
        in = (const V*)a.in + (cx.rcv_in ? (size_t)alpha * a.R * a.B : (size_t)alpha * NB);
        if (a.out_mode == FM_JT_PER_SOURCE) outp = (V*)a.out + (size_t)alpha * NB;
    }

    // The batches of all levels form one sequence; the meta words of the next
    // batch (possibly the first batch of the next level) are requested before
    // the current batch's operands.
    LevelDesc cur = load_desc<DIR>(sd, 0);
    LevelDesc nxt = cur;
    if (L > 1) nxt = load_desc<DIR>(sd, 1);
    uint64_t mcur[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int u = slot0 + q * SLOTS;
        mcur[q] = u < cur.nsc ? meta[cur.p0 + u] : ~0ull;
    }
    int l = 0;
    int base = 0;
    for (;;) {
        const bool same_level = base + BATCH < cur.nsc;
        const bool has_next = same_level || l + 1 < L;
        uint64_t mnxt[U];
        const int np0 = same_level ? cur.p0 : nxt.p0;
        const int nnsc = same_level ? cur.nsc : nxt.nsc;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int u = (same_level ? base + BATCH : 0) + slot0 + q * SLOTS;
            mnxt[q] = (has_next && u < nnsc) ? meta[np0 + u] : ~0ull;
        }
        {
            NodeOps<V, VW> ops[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                ops[q].node = -1;
                if (mcur[q] != ~0ull)
                    fetch_static<DIR, V, VW>(ops[q], mcur[q], cur.p0 + base + slot0 + q * SLOTS, wts, in, cx, sd, cur);
            }
            V res[U][VW];
#pragma unroll
            for (int q = 0; q < U; ++q)
                if (ops[q].node >= 0) combine<DIR, V, VW, V>(ops[q], ovf_base, X, cx, res[q]);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (ops[q].node >= 0) {
                    Pack<V, VW> o;
#pragma unroll
                    for (int v = 0; v < VW; ++v) o.v[v] = res[q][v];
                    st<V, VW>(X + ops[q].node * cx.B + cx.rhs0, o);
                    if (DIR == kRev && outp) {
#pragma unroll
                        for (int v = 0; v < VW; ++v) o.v[v] = ops[q].rec.v[0] * res[q][v];
                        st<V, VW>(outp + ops[q].node * cx.B + cx.rhs0, o);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) mcur[q] = mnxt[q];
        if (same_level) {
            base += BATCH;
            continue;
        }
        // end of level l: its nontrivial SCC blocks, then the level barrier
        for (int bi = cur.b0; bi < cur.b1; ++bi) {
            const int blk = DIR == kFwd ? sd.fblk_id[bi] : sd.rblk_id[bi];
            block_solve<DIR, V, RG, VW, NT>(sd, blk, meta, wts, in, X, outp, cx, cur, lds, slot0, sub);
        }
        __syncthreads();
        if (++l >= L) break;
        cur = nxt;
        if (l + 1 < L) nxt = load_desc<DIR>(sd, l + 1);
        base = 0;
    }
}

}  // namespace fm
