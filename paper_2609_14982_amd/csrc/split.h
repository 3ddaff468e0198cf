// Node-split level walk: P workgroups share one source and all B right-hand
// sides.  Included by device.hip only, after sweep.h.
//
// Why.  A level step is bound by the number of cache-line requests each CU
// keeps in flight, not by bytes.  With the rhs-group split every node's
// 128-byte line of B = 16 FP64 values is requested by B / RG workgroups that
// each use RG of them; here one workgroup takes a node and all B values, so
// every line request carries a full line, and the P workgroups of a source
// take disjoint slices of each level instead.
//
// Synchronisation.  Nodes of one level are independent (Section 4.1,
// Proposition 3), so the P workgroups only meet at the end of a level: each
// waits for its own stores to complete, one thread adds 1 to the source's
// arrival counter and polls it until all P have arrived.  The counter is only
// touched by device-scope atomics, which every XCD sees.  The node values are
// exchanged through the L2 of the XCD the P workgroups run on (workgroups are
// dispatched to XCDs round-robin and the P of one source sit P-aligned in one
// XCD's share of the grid); whether they really share an XCD is checked at
// the first barrier from the XCC_ID hardware register, and if not, every
// barrier adds the device-scope release (L2 write-back) and acquire (cache
// invalidate) so that the result is right either way.  A node's values are
// written once per launch and read only after the barrier that follows, and
// with rows of a multiple of 128 bytes no cache line holds two nodes, so no
// stale line can sit in a CU's L1.  The batch's own node-value scratch and the
// block staging rows are therefore padded to whole lines (FP32 with 16 rhs,
// FP64 with 8); only a caller's output array with shorter rows (J to all
// nodes) takes the cache-invalidating acquire at every barrier.  Every wait
// is bounded: after ~10 s without progress the wave sets the launch's abort
// word, so that all later barriers of that launch return at
// once and the launch always ends, and the batch's sticky failure word, which
// fm_batch_status reports.  The abort word is cleared before every launch, so
// one failed launch never shortens the waits of the next.
//
// Nontrivial SCC blocks (Section 4.3) take two phases.  Phase 1 computes the
// block right-hand sides b_C = q_C + sum_ext w x for the members (members
// split over the P workgroups, like singletons) into a per-source staging
// area; a barrier; phase 2 splits the block's rows over the P workgroups, each
// row owned by one thread that accumulates all B right-hand sides while b_C
// streams through LDS in chunks; a second barrier.
#pragma once

namespace fm {

struct SplitArgs {
    unsigned* ctr;      // [S] arrival counters, one per 128-byte line (32 words apart)
    unsigned* xmask;    // [S] XCDs seen per source, one per 128-byte line
    unsigned* abort_w;  // one word: set when a barrier wait of this launch timed out
    unsigned* fail_w;   // one word, sticky until fm_batch_status: some launch timed out
    void* stage;        // [S][stage_rows][stage_B] block right-hand sides (FP64)
    int64_t stage_rows;
    int32_t stage_B;    // doubles per staged row: B rounded up to whole 128-byte lines, so
                        // no line holds two rows (read by other workgroups after a barrier)
    int32_t P;          // workgroups per source
    int32_t lds_rows;   // rows of b_C per LDS chunk (vector block path)
    int32_t inv_l1;     // rows are not a multiple of 128 bytes
    int32_t rcv_lds;    // receiver inputs of the transpose staged in LDS
    int32_t stage_off;  // first LDS double of the block staging area
    const int32_t* wg_map;  // NULL, or per workgroup source << 8 | part (-1: idle)
    const int32_t* src_P;   // with wg_map: workgroups of each source
};

constexpr int kCtrStride = 32;                 // words between counters
constexpr uint64_t kBarrierTicks = 1000000000; // 10 s of the 100 MHz realtime clock

struct GroupSync {
    unsigned* ctr;
    unsigned* abort_w;
    unsigned* fail_w;
    unsigned target;
    bool agent;       // device-scope release/acquire around every barrier
    bool inv_l1;      // acquire at every barrier
    bool dead;        // a wait of this launch timed out somewhere
};

__device__ __forceinline__ unsigned xcc_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xfu;
}

// All threads of the workgroup call this at the same point.
__device__ __forceinline__ void group_barrier(GroupSync& g, int P) {
    __shared__ unsigned s_dead;
    g.target += (unsigned)P;
    // this wave's stores have reached the L2 before the arrival is counted
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (g.agent) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned dead = g.dead ? 1u : 0u;
        // the last workgroup to arrive learns it from the add and does not poll
        const unsigned old = __hip_atomic_fetch_add(g.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!dead && (int)(old + 1u - g.target) < 0) {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                const unsigned c = __hip_atomic_load(g.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((int)(c - g.target) >= 0) break;
                if (__hip_atomic_load(g.abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { dead = 1u; break; }
                if (wall_clock64() - t0 > kBarrierTicks) {
                    __hip_atomic_fetch_or(g.fail_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_or(g.abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    dead = 1u;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_dead = dead;
    }
    __syncthreads();
    g.dead = s_dead != 0u;
    if (g.agent || g.inv_l1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// [lo, hi) of n items for part p of P (contiguous, sizes differ by <= 1)
__device__ __forceinline__ void share(int n, int P, int p, int& lo, int& hi) {
    const int q = n / P, r = n % P;
    lo = p * q + (p < r ? p : r);
    hi = lo + q + (p < r ? 1 : 0);
}

// Streaming loads: records, meta words and inputs are read once per launch,
// so they are loaded non-temporally and leave the L2 to the node values that
// later levels read again.
// The pointers are cast to the global address space: a generic pointer
// would give FLAT loads, which also count against the LDS/scalar wait
// counter, so every wait for a scalar or LDS access would wait for them too.
template <typename V, int VW>
__device__ __forceinline__ Pack<V, VW> ld_stream(const V* p) {
    typedef V vec __attribute__((ext_vector_type(VW)));
    typedef const __attribute__((address_space(1))) vec gvec;
    const vec x = __builtin_nontemporal_load((gvec*)(p));
    Pack<V, VW> r;
#pragma unroll
    for (int v = 0; v < VW; ++v) r.v[v] = x[v];
    return r;
}

__device__ __forceinline__ uint64_t ld_meta(const uint64_t* p) {
    typedef const __attribute__((address_space(1))) uint64_t gu64;
    return __builtin_nontemporal_load((gu64*)(p));
}

// Singleton operands with 32-bit byte offsets: every array of one source
// (a [N][B] vector, the [N][4] records) spans less than 4 GiB, so an access
// is a uniform base pointer plus one 32-bit lane offset (the "saddr" form of
// the global loads) and a neighbour's offset is the node's plus a signed
// axis stride.  This keeps the per-node address arithmetic to a few 32-bit
// instructions.
template <typename V, int VW>
struct Node32 {
    uint32_t row;    // byte offset of this lane's values in the node-value array X (rows of xrowb bytes)
    uint32_t mask;   // neighbour mask (0 for an empty slot)
    uint32_t ovf;
    bool ok;
    Pack<V, 4> rec;
    Pack<V, VW> inp;
};

// byte stride of one step along each logical axis in a [N][B] array, kept
// as three scalars (a struct or array indexed by the slot ends up in scratch
// memory)
struct Strides32 {
    int32_t a0, a1, a2;
};

__device__ __forceinline__ uint32_t nbr_row(uint32_t row, int slot, int32_t a0, int32_t a1, int32_t a2) {
    const int32_t m = slot < 2 ? a0 : (slot < 4 ? a1 : a2);
    return row + (uint32_t)((slot & 1) ? m : -m);
}

// Cube-stencil slot b: the offset o in {-1,0,1}^3 whose base-3 number
// (o_0 + 1) + 3 (o_1 + 1) + 9 (o_2 + 1), centre left out, is b.
__device__ __forceinline__ uint32_t nbr_row_cube(uint32_t row, int slot, int32_t a0, int32_t a1, int32_t a2) {
    const int b = slot + (slot >= 13 ? 1 : 0);
    const int q = (b * 11) >> 5;          // b / 3 for 0 <= b < 27
    const int o0 = b - 3 * q - 1;
    const int q2 = (q * 11) >> 5;         // q / 3
    const int o1 = q - 3 * q2 - 1;
    const int o2 = q2 - 1;
    return row + (uint32_t)(o0 * a0 + o1 * a1 + o2 * a2);
}

template <bool CUBE>
__device__ __forceinline__ uint32_t nbr_at(uint32_t row, int slot, const Strides32& sx) {
    return CUBE ? nbr_row_cube(row, slot, sx.a0, sx.a1, sx.a2) : nbr_row(row, slot, sx.a0, sx.a1, sx.a2);
}

template <typename V, int VW>
__device__ __forceinline__ Pack<V, VW> ldb(const char* base, uint32_t off) {
    return ld<V, VW>(reinterpret_cast<const V*>(base + off));
}

template <typename V, int VW>
__device__ __forceinline__ Pack<V, VW> ldb_stream(const char* base, uint32_t off) {
    return ld_stream<V, VW>(reinterpret_cast<const V*>(base + off));
}

// Receiver inputs of the transpose (r = P^T y, duplicates added in entry
// order), either from the LDS copy made at kernel start (rv values per entry,
// rpos reverse positions) or from global memory.
struct RcvLds {
    const double* rv;
    const int32_t* rpos;
    bool on;
};

template <int DIR, typename V, int VW, bool CUBE>
__device__ __forceinline__ void fetch32(Node32<V, VW>& p, uint64_t m, int pos, const char* __restrict__ wtc,
                                        const char* __restrict__ inc, uint32_t rowb, uint32_t xrowb, uint32_t lane_off,
                                        const Ctx& cx, const SrcDev& sd, const LevelDesc& d, const V* in,
                                        const RcvLds& rl) {
    const uint32_t node = (uint32_t)(m & kNodeMask);
    p.row = node * xrowb + lane_off;
    if (CUBE) {
        // 26-bit mask; the overflow offset of a node with more than three
        // neighbours is in the per-position array
        p.mask = (uint32_t)((m >> kCubeMaskShift) & kCubeMask);
        p.ovf = __builtin_popcount(p.mask) > 3 ? (uint32_t)gld((DIR == kFwd ? sd.fovf : sd.rovf) + pos) : 0u;
    } else {
        p.ovf = (uint32_t)((m >> kOffShift) & kOffMask);
        p.mask = (uint32_t)(m >> kMaskShift);
    }
    p.rec = ldb_stream<V, 4>(wtc, (uint32_t)pos * (uint32_t)(4 * sizeof(V)));
    if (DIR == kFwd || !cx.rcv_in) {
        p.inp = ldb_stream<V, VW>(inc, node * rowb + lane_off);
    } else {
#pragma unroll
        for (int v = 0; v < VW; ++v) p.inp.v[v] = (V)0;
        // with the LDS copy the receiver values are added later by
        // rcv_add, after every load of the batch has been issued
        if (!rl.on && (m & kRcvFlag)) {
            {
                for (int e = d.e0; e < d.e1; ++e)
                    if (gld(sd.rcv_pos + (e)) == pos) {
                        const Pack<V, VW> y = ld<V, VW>(in + (int64_t)gld(sd.rcv_idx + (e)) * cx.B + cx.rhs0);
                        const V w = (V)gld(sd.rcv_ew + (e));
#pragma unroll
                        for (int v = 0; v < VW; ++v) p.inp.v[v] += w * y.v[v];
                    }
            }
        }
    }
}

// Receiver inputs from the LDS copy (duplicates in entry order): every lane
// walks the level's few receiver entries (uniform bounds) and keeps the
// matching ones.
template <typename V, int VW>
__device__ __forceinline__ void rcv_add(Node32<V, VW>& p, int pos, const LevelDesc& d, const RcvLds& rl, int B,
                                        int rhs0) {
    for (int e = d.e0; e < d.e1; ++e) {
        const bool hit = rl.rpos[e] == pos;
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const V y = (V)rl.rv[e * B + rhs0 + v];
            p.inp.v[v] = hit ? p.inp.v[v] + y : p.inp.v[v];
        }
    }
}

template <typename V, int VW, bool CUBE>
__device__ __forceinline__ void nbrs32(const Node32<V, VW>& p, const char* __restrict__ Xc, const Strides32 sx,
                                       Pack<V, VW> xv[3]) {
    uint32_t m = p.mask;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (m != 0u) xv[t] = ldb<V, VW>(Xc, nbr_at<CUBE>(p.row, __builtin_ctz(m), sx));
        m &= m - 1u;
    }
}

// x_node = c*ds + sum_j w_j x_j (primal) or r + sum_i w_i lambda_i
// (transpose) in ascending slot order (the order of the rhs-group kernel,
// hence the same bits); neighbours past the third (rare) are loaded here.
template <int DIR, typename V, int VW, typename T, bool CUBE>
__device__ __forceinline__ void acc32(const Node32<V, VW>& p, const Pack<V, VW> xv[3], const V* __restrict__ ovf_base,
                                      const char* __restrict__ Xc, const Strides32 sx, T acc[VW]) {
    uint32_t m = p.mask;
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = (DIR == kFwd) ? (T)p.rec.v[0] * (T)p.inp.v[v] : (T)p.inp.v[v];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (m != 0u) {
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[v] += (T)p.rec.v[1 + t] * (T)xv[t].v[v];
        }
        m &= m - 1u;
    }
    for (int t = 3; m != 0u; ++t) {
        const Pack<V, VW> x = ldb<V, VW>(Xc, nbr_at<CUBE>(p.row, __builtin_ctz(m), sx));
        m &= m - 1u;
        const T w = (T)gld(ovf_base + p.ovf + (t - 3));
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += w * (T)x.v[v];
    }
}

// Phase 1 of the level's blocks: b_C of this workgroup's share of every
// block's members into the staging rows (LPN lanes per member), summed in
// FP64 whatever the vector precision.
template <int DIR, typename V, int LPN, int NT, bool CUBE>
__device__ __forceinline__ void split_block_rhs(const SrcDev& sd, const LevelDesc& d, const uint64_t* __restrict__ meta,
                                                const char* __restrict__ wtc, const char* __restrict__ inc,
                                                const V* __restrict__ in, const V* __restrict__ ovf_base,
                                                const char* __restrict__ Xc, const Strides32 sx, uint32_t xrowb,
                                                uint32_t lane_off, double* __restrict__ stage, int SB, const Ctx& cx,
                                                int P, int part, int slot0, const RcvLds& rl) {
    constexpr int VW = 16 / (int)sizeof(V);
    constexpr int SLOTS = NT / LPN;
    constexpr uint32_t ROWB = LPN * VW * sizeof(V);
    for (int bi = d.b0; bi < d.b1; ++bi) {
        const int blk = DIR == kFwd ? gld(sd.fblk_id + (bi)) : gld(sd.rblk_id + (bi));
        const int k = gld(sd.blk_k + (blk));
        const int bp = DIR == kFwd ? gld(sd.blk_fpos + (blk)) : gld(sd.blk_rpos + (blk));
        const int64_t moff = gld(sd.blk_moff + (blk));
        int lo, hi;
        share(k, P, part, lo, hi);
        for (int mi = lo + slot0; mi < hi; mi += SLOTS) {
            Node32<V, VW> p;
            fetch32<DIR, V, VW, CUBE>(p, ld_meta(meta + bp + mi), bp + mi, wtc, inc, ROWB, xrowb, lane_off, cx, sd, d, in,
                                rl);
            Pack<V, VW> xv[3];
            nbrs32<V, VW, CUBE>(p, Xc, sx, xv);
            if (DIR == kRev && cx.rcv_in && rl.on) rcv_add<V, VW>(p, bp + mi, d, rl, cx.B, cx.rhs0);
            Pack<double, VW> o;
            acc32<DIR, V, VW, double, CUBE>(p, xv, ovf_base, Xc, sx, o.v);
            st<double, VW>(stage + (moff + mi) * SB + cx.rhs0, o);
        }
    }
}

// Phase 2: rows of this workgroup's share of each block,
// x_i = sum_j Minv(i, j) b_j (primal, column-major inverse) or
// y_j = sum_i Minv(i, j) b_i (transpose, row-major copy), in ascending
// order of the summation index.  Each thread owns a row and all B
// right-hand sides (consecutive threads take consecutive rows, so a wave
// reads a contiguous piece of each matrix column) and keeps G matrix entries
// in flight; b_C streams through LDS in chunks that every thread loads with
// all its requests issued at once.
// Phase 2 on the matrix cores (B a multiple of 16): the share's rows of
// X_C = Minv * B_C form a (rows x k) by (k x 16) FP64 product per 16
// right-hand sides, computed with v_mfma_f64_16x16x4f64.  Lane layout of that
// instruction: A(16 x 4) lane l holds A[l % 16][l / 16], B(4 x 16) lane l
// holds B[l / 16][l % 16], and D(16 x 16) lane l register r holds
// D[4 r + l / 16][l % 16].  A wave owns TW tiles of 16 rows; per step of 4
// columns it loads one matrix entry per lane and tile (a contiguous 128-byte
// piece of each column) and one staged right-hand-side value per lane, with
// clamped in-range addresses and a zero select past the last column, so the
// loop has no divergent branches.  The four products of a step are summed by
// the instruction, steps in ascending column order (a fixed order for every
// schedule of the node split).
template <int DIR, typename V, int B, int NT>
__device__ __forceinline__ void split_block_solve_mfma(const SrcDev& sd, const LevelDesc& d,
                                                       const uint64_t* __restrict__ meta, const V* __restrict__ wts,
                                                       const double* __restrict__ stage, int SB, V* __restrict__ X,
                                                       int XB, V* __restrict__ outp, int P, int part) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int WAVES = NT / 64;
    constexpr int TW = 4;                       // 16-row tiles per wave
    constexpr int G = 4;                        // column steps in flight
    constexpr int ROWS = WAVES * TW * 16;       // rows per pass
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    for (int bi = d.b0; bi < d.b1; ++bi) {
        const int blk = DIR == kFwd ? gld(sd.fblk_id + (bi)) : gld(sd.rblk_id + (bi));
        if (gld(sd.blk_it + 2 * blk)) continue;   // solved iteratively
        const int k = gld(sd.blk_k + (blk));
        const int bp = DIR == kFwd ? gld(sd.blk_fpos + (blk)) : gld(sd.blk_rpos + (blk));
        const int64_t moff = gld(sd.blk_moff + (blk));
        const __attribute__((address_space(1))) double* __restrict__ Mx =
            gptr(DIR == kFwd ? sd.inv + gld(sd.blk_inv + (blk)) : sd.invt + gld(sd.blk_inv + (blk)));
        int lo, hi;
        share(k, P, part, lo, hi);
        for (int r0 = lo; r0 < hi; r0 += ROWS) {
            for (int ct = 0; ct < B; ct += 16) {
                const double* __restrict__ bsrc = stage + moff * SB + ct + lr;
                int rowc[TW];
#pragma unroll
                for (int t = 0; t < TW; ++t) rowc[t] = min(r0 + (wave * TW + t) * 16 + lr, hi - 1);
                d4 acc[TW];
#pragma unroll
                for (int t = 0; t < TW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
                for (int j = 0; j < k; j += 4 * G) {
                    double av[G][TW], bv[G];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const int col = j + 4 * g + lk;
                        const int cc = min(col, k - 1);
                        bv[g] = bsrc[(int64_t)cc * SB];
#pragma unroll
                        for (int t = 0; t < TW; ++t) av[g][t] = Mx[(size_t)cc * k + rowc[t]];
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const bool in = j + 4 * g + lk < k;
                        const double b = in ? bv[g] : 0.0;
#pragma unroll
                        for (int t = 0; t < TW; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g][t], b, acc[t], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int t = 0; t < TW; ++t) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = r0 + (wave * TW + t) * 16 + 4 * r + lk;
                        if (i < hi) {
                            const uint64_t mw = gld(meta + bp + i);
                            const int64_t node = (int64_t)(mw & kNodeMask);
                            X[node * XB + ct + lr] = (V)acc[t][r];
                            if (DIR == kRev && outp) outp[node * B + ct + lr] = gld(wts + (size_t)(bp + i) * 4) * (V)acc[t][r];
                        }
                    }
                }
            }
        }
    }
}

// Blocks solved iteratively (large SCCs; Section 6 names iterative block
// solvers for them): with rho(W_CC) < 1 (Theorem 1) the block solution is the
// Neumann series x = sum_j W_CC^j b, summed as x^0 = b, x^j = b + W_CC x^{j-1}
// for j = 1..m (transpose: W_CC^T), m fixed at setup so that the tail is
// below FP64 rounding.  The iterates live in FP64 in the two staging buffers
// after b (k rows each), the last one goes straight to the node rows.  The
// P workgroups split the block's rows; all of them pass the m - 1 barriers
// between iterates, which invalidate the L1 (the two buffers are rewritten
// every other iterate).  Each row sums its couplings in one fixed order, so
// every schedule gives the same bits.
template <int DIR, typename V, int B, int NT>
__device__ __forceinline__ void split_block_iterate(const SrcDev& sd, const LevelDesc& d,
                                                    const uint64_t* __restrict__ meta, const V* __restrict__ wts,
                                                    double* __restrict__ stage, int SB, V* __restrict__ X, int XB,
                                                    V* __restrict__ outp, int P, int part, GroupSync& g) {
    constexpr int H = B / 2;   // pairs of right-hand sides per row
    for (int bi = d.b0; bi < d.b1; ++bi) {
        const int blk = DIR == kFwd ? gld(sd.fblk_id + (bi)) : gld(sd.rblk_id + (bi));
        const int m = gld(sd.blk_it + 2 * blk + (DIR == kFwd ? 0 : 1));
        if (!m) continue;
        const int k = gld(sd.blk_k + (blk));
        const int bp = DIR == kFwd ? gld(sd.blk_fpos + (blk)) : gld(sd.blk_rpos + (blk));
        const int64_t moff = gld(sd.blk_moff + (blk));
        const int64_t sp = gld(sd.blk_sp + (blk));
        const int32_t* __restrict__ rp = (DIR == kFwd ? sd.sp_ptr : sd.spt_ptr) + sp;
        const int32_t* __restrict__ cl = DIR == kFwd ? sd.sp_col : sd.spt_col;
        const double* __restrict__ wv = DIR == kFwd ? sd.sp_w : sd.spt_w;
        double* __restrict__ b0 = stage + moff * SB;
        double* __restrict__ buf[2] = {b0 + (int64_t)k * SB, b0 + (int64_t)2 * k * SB};
        int lo, hi;
        share(k, P, part, lo, hi);
        const int items = (hi - lo) * H;
        for (int j = 1; j <= m; ++j) {
            const double* __restrict__ cur = j == 1 ? b0 : buf[(j - 1) & 1];
            double* __restrict__ nxt = buf[j & 1];
            for (int t = (int)threadIdx.x; t < items; t += NT) {
                const int i = lo + t / H;
                const int c = 2 * (t % H);
                double a0 = gld(b0 + (int64_t)i * SB + c), a1 = gld(b0 + (int64_t)i * SB + c + 1);
                const int e1 = gld(rp + i + 1);
                for (int e = gld(rp + i); e < e1; ++e) {
                    const int64_t r = (int64_t)gld(cl + e) * SB + c;
                    const double w = gld(wv + e);
                    a0 += w * gld(cur + r);
                    a1 += w * gld(cur + r + 1);
                }
                if (j < m) {
                    nxt[(int64_t)i * SB + c] = a0;
                    nxt[(int64_t)i * SB + c + 1] = a1;
                } else {
                    const int64_t node = (int64_t)(gld(meta + bp + i) & kNodeMask);
                    X[node * XB + c] = (V)a0;
                    X[node * XB + c + 1] = (V)a1;
                    if (DIR == kRev && outp) {
                        const V cc = gld(wts + (size_t)(bp + i) * 4);
                        outp[node * B + c] = cc * (V)a0;
                        outp[node * B + c + 1] = cc * (V)a1;
                    }
                }
            }
            if (j < m) {
                const bool keep = g.inv_l1;
                g.inv_l1 = true;
                group_barrier(g, P);
                g.inv_l1 = keep;
            }
        }
    }
}

template <int DIR, typename V, int B, int NT>
__device__ __forceinline__ void split_block_solve(const SrcDev& sd, const LevelDesc& d, const uint64_t* __restrict__ meta,
                                                  const V* __restrict__ wts, const double* __restrict__ stage, int SB,
                                                  V* __restrict__ X, int XB, V* __restrict__ outp, int P, int part,
                                                  int lds_rows, double* lds) {
    constexpr int G = 16;
    constexpr int CH = 8;    // staged values per thread and round
    for (int bi = d.b0; bi < d.b1; ++bi) {
        const int blk = DIR == kFwd ? gld(sd.fblk_id + (bi)) : gld(sd.rblk_id + (bi));
        if (gld(sd.blk_it + 2 * blk)) continue;   // solved iteratively
        const int k = gld(sd.blk_k + (blk));
        const int bp = DIR == kFwd ? gld(sd.blk_fpos + (blk)) : gld(sd.blk_rpos + (blk));
        const int64_t moff = gld(sd.blk_moff + (blk));
        const __attribute__((address_space(1))) double* __restrict__ Mx =
            gptr(DIR == kFwd ? sd.inv + gld(sd.blk_inv + (blk)) : sd.invt + gld(sd.blk_inv + (blk)));
        const double* __restrict__ bsrc = stage + moff * SB;
        int lo, hi;
        share(k, P, part, lo, hi);
        // every thread of the workgroup passes the same barriers: the row
        // loop runs the same number of times in all of them
        for (int r0 = lo; r0 < hi; r0 += NT) {
            const int i = r0 + (int)threadIdx.x;
            const bool own = i < hi;
            double acc[B];
#pragma unroll
            for (int rr = 0; rr < B; ++rr) acc[rr] = 0.0;
            for (int j0 = 0; j0 < k; j0 += lds_rows) {
                const int jn = min(lds_rows, k - j0);
                const int nv = jn * B;
                const double* __restrict__ bs = bsrc + (int64_t)j0 * SB;
                __syncthreads();
                for (int t0 = 0; t0 < nv; t0 += NT * CH) {
                    double v[CH];
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const int t = t0 + c * NT + (int)threadIdx.x;
                        v[c] = t < nv ? bs[(t / B) * SB + (t % B)] : 0.0;
                    }
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const int t = t0 + c * NT + (int)threadIdx.x;
                        if (t < nv) lds[t] = v[c];
                    }
                }
                __syncthreads();
                if (own) {
                    const __attribute__((address_space(1))) double* __restrict__ col = Mx + (size_t)j0 * k + i;
                    int j = 0;
                    for (; j + G <= jn; j += G) {
                        double m[G];
#pragma unroll
                        for (int t = 0; t < G; ++t) m[t] = col[(size_t)(j + t) * k];
#pragma unroll
                        for (int t = 0; t < G; ++t) {
                            const double* bj = lds + (j + t) * B;
#pragma unroll
                            for (int rr = 0; rr < B; ++rr) acc[rr] += m[t] * bj[rr];
                        }
                    }
                    for (; j < jn; ++j) {
                        const double m = col[(size_t)j * k];
                        const double* bj = lds + j * B;
#pragma unroll
                        for (int rr = 0; rr < B; ++rr) acc[rr] += m * bj[rr];
                    }
                }
            }
            if (own) {
                const uint64_t mw = gld(meta + bp + i);
                const int64_t node = (int64_t)(mw & kNodeMask);
                const V c = gld(wts + (size_t)(bp + i) * 4);
                V* dst = X + node * XB;
#pragma unroll
                for (int rr = 0; rr < B; ++rr) dst[rr] = (V)acc[rr];
                if (DIR == kRev && outp) {
                    V* o = outp + node * B;
#pragma unroll
                    for (int rr = 0; rr < B; ++rr) o[rr] = c * (V)acc[rr];
                }
            }
        }
    }
}

// Position of this workgroup in its source's sequence of batches: every
// level has at least one batch (possibly empty), so that every level ends
// with its barrier.
struct Cursor {
    int l, base, lo, hi;
    LevelDesc d;
};

template <int DIR, int BATCH>
__device__ __forceinline__ void cursor_next(Cursor& c, const SrcDev& sd, int L, int P, int part) {
    if (c.base + BATCH < c.hi) {
        c.base += BATCH;
        return;
    }
    if (++c.l < L) {
        c.d = load_desc<DIR>(sd, c.l);
        share(c.d.nsc, P, part, c.lo, c.hi);
        c.base = c.lo;
    }
}

// MODE bit 0 (transpose only): input given at the receivers; bit 1: the
// records of a cube-stencil state (26-bit neighbour masks).  The two input modes
// are separate kernels; with a run-time choice between them inside the batch
// loop the compiler placed its memory waits for one path only, and the
// receiver path ran 15 % slower.  (The optional per-source output stays a
// run-time choice: compiled out, the same loop measured slower.)
// At least two waves per SIMD (at most 256 registers per lane), so that two
// 256-thread workgroups of different sources share a CU and one streams
// while the other waits at a level barrier.
template <int DIR, typename V, int LPN, int NT, int U, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_split(ApplyArgs a, SplitArgs s) {
    constexpr bool RCV = DIR == kRev && (MODE & 1) != 0;
    constexpr bool CUBE = (MODE & 2) != 0;   // 26-neighbour stencil records
    constexpr int VW = 16 / (int)sizeof(V);
    constexpr int B = LPN * VW;
    constexpr int SLOTS = NT / LPN;
    constexpr int BATCH = SLOTS * U;
    int P = s.P;
    int alpha, part;
    if (s.wg_map) {
        // balanced split: the host's table (workgroup w runs on XCD w % 8,
        // where all workgroups of its source are placed)
        const int code = s.wg_map[blockIdx.x];
        if (code < 0) return;          // idle slot: touches no counter
        alpha = code >> 8;
        part = code & 255;
        P = s.src_P[alpha];
    } else {
        const int w = blockIdx.x;
        const int item = (w % 8) * a.per_xcd + (w / 8);
        if (item >= a.items) return;   // not part of any source's group: touches no counter
        alpha = item / P;
        part = item - alpha * P;
    }
    extern __shared__ double lds[];
    __shared__ unsigned s_xmask;
    const SrcDev sd = a.src[alpha];
    const uint64_t* __restrict__ meta = DIR == kFwd ? sd.fmeta : sd.rmeta;
    const V* __restrict__ wts = (const V*)(DIR == kFwd ? sd.fwts : sd.rwts);
    const V* __restrict__ ovf_base = wts + a.N * 4;
    const int L = DIR == kFwd ? sd.L_f : sd.L_r;
    const int sub = threadIdx.x % LPN;
    const int slot0 = threadIdx.x / LPN;
    const int64_t NB = a.N * B;
    Ctx cx;
    cx.B = B;
    cx.rhs0 = sub * VW;
    cx.R = a.R;
    cx.st1 = a.st1;
    cx.st2 = a.st2;
    cx.N = a.N;
    cx.rcv_in = RCV;
    cx.cube = CUBE;
    const V* __restrict__ in;
    // node values: rows of a.xB >= B values (padded to whole 128-byte lines
    // when the array is the batch's own scratch, so no line holds two nodes)
    V* __restrict__ X = (V*)a.work + (size_t)alpha * a.N * a.xB;
    V* __restrict__ outp = nullptr;
    if (DIR == kFwd) {
        in = (const V*)a.in + (a.in_mode == FM_DS_PER_PAIR ? (size_t)alpha * NB : 0);
    } else {
        in = (const V*)a.in + (cx.rcv_in ? (size_t)alpha * a.R * B : (size_t)alpha * NB);
        if (a.out_mode == FM_JT_PER_SOURCE) outp = (V*)a.out + (size_t)alpha * NB;
    }
    // staged rows: a compile-time B when B doubles already fill whole lines
    const int SB = (B * 8) % 128 == 0 ? B : s.stage_B;
    double* __restrict__ stage = (double*)s.stage + (size_t)alpha * s.stage_rows * SB;
    // byte-offset views of the same arrays (each spans < 4 GiB, checked on the host)
    constexpr uint32_t ROWB = B * sizeof(V);                 // input and per-source output rows
    // node-value rows (a compile-time ROWB when B values already fill whole lines)
    const uint32_t XROWB = ROWB % 128 == 0 ? ROWB : (uint32_t)a.xB * sizeof(V);
    const int xsh = ROWB % 128 == 0 || a.xB == B ? 0 : 1;   // XROWB = ROWB << xsh
    const uint32_t lane_off = (uint32_t)(cx.rhs0 * sizeof(V));
    const char* __restrict__ Xc = reinterpret_cast<const char*>(X);
    char* __restrict__ Xw = reinterpret_cast<char*>(X);
    const char* __restrict__ inc = reinterpret_cast<const char*>(in);
    const char* __restrict__ wtc = reinterpret_cast<const char*>(wts);
    Strides32 sx;
    sx.a0 = (int32_t)XROWB;
    sx.a1 = (int32_t)(a.st1 * XROWB);
    sx.a2 = (int32_t)(a.st2 * XROWB);
    // transpose from receiver data: copy this source's receiver entries (in
    // the order of the reverse levels), each input value times the entry's
    // weight, and their positions to LDS
    RcvLds rl;
    rl.on = DIR == kRev && cx.rcv_in && s.rcv_lds != 0;
    rl.rv = lds;
    rl.rpos = reinterpret_cast<const int32_t*>(lds + (size_t)sd.n_ent * B);
    if (rl.on) {
        double* rv = lds;
        int32_t* rpos = reinterpret_cast<int32_t*>(lds + (size_t)sd.n_ent * B);
        for (int t = threadIdx.x; t < sd.n_ent * B; t += NT) {
            const int e = t / B, b = t - e * B;
            rv[t] = gld(sd.rcv_ew + (e)) * (double)in[(int64_t)gld(sd.rcv_idx + (e)) * B + b];
        }
        for (int t = threadIdx.x; t < sd.n_ent; t += NT) rpos[t] = gld(sd.rcv_pos + (t));
        __syncthreads();
    }

    GroupSync g;
    g.ctr = s.ctr + (size_t)alpha * kCtrStride;
    g.abort_w = s.abort_w;
    g.fail_w = s.fail_w;
    g.target = 0;
    g.agent = true;          // until the XCD check at the first barrier
    g.inv_l1 = s.inv_l1 != 0;
    g.dead = false;
    if (threadIdx.x == 0)
        s_xmask = __hip_atomic_fetch_or(s.xmask + (size_t)alpha * kCtrStride, 1u << xcc_id(), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    bool first = true;

    // The meta words of the next batch (possibly the next level's first)
    // are requested before the current batch's operands; a batch then waits
    // on one round trip for its records, inputs and neighbour values.  The
    // batch (SLOTS * U nodes) is sized so that a workgroup's share of a
    // typical level is one batch.
    auto meta_of = [&](const Cursor& c, uint64_t mw[U]) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int u = c.base + slot0 + q * SLOTS;
            mw[q] = (c.l < L && u < c.hi) ? ld_meta(meta + c.d.p0 + u) : ~0ull;
        }
    };

    Cursor cC;
    cC.l = 0;
    cC.d = load_desc<DIR>(sd, 0);
    share(cC.d.nsc, P, part, cC.lo, cC.hi);
    cC.base = cC.lo;
    Cursor cN = cC;
    cursor_next<DIR, BATCH>(cN, sd, L, P, part);
    uint64_t mC[U];
    meta_of(cC, mC);
    // records and inputs of a batch (static data)
    Node32<V, VW> ops[U];
    auto fetch_batch = [&](const Cursor& c, const uint64_t mw[U]) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            ops[q].ok = mw[q] != ~0ull;
            if (ops[q].ok)
                fetch32<DIR, V, VW, CUBE>(ops[q], mw[q], c.d.p0 + c.base + slot0 + q * SLOTS, wtc, inc, ROWB, XROWB, lane_off, cx,
                                    sd, c.d, in, rl);
        }
    };
    bool pre = false;   // ops already hold the current batch's static data
    for (;;) {
        const bool last = cC.base + BATCH >= cC.hi;          // last batch of level cC.l
        const bool blocks = last && cC.d.b1 > cC.d.b0;
        const bool more = cC.l + 1 < L;
        uint64_t mN[U];
        meta_of(cN, mN);
        {
            Pack<V, VW> xv[U][3];
            if (!pre) fetch_batch(cC, mC);
#pragma unroll
            for (int q = 0; q < U; ++q)
                if (ops[q].ok) nbrs32<V, VW, CUBE>(ops[q], Xc, sx, xv[q]);
            if (RCV && rl.on) {
#pragma unroll
                for (int q = 0; q < U; ++q)
                    if (ops[q].ok) rcv_add<V, VW>(ops[q], cC.d.p0 + cC.base + slot0 + q * SLOTS, cC.d, rl, B, cx.rhs0);
            }
            Pack<V, VW> o[U];
            uint32_t orow[U];
            V oscale[U];
            bool ook[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                ook[q] = ops[q].ok;
                orow[q] = ops[q].row;
                oscale[q] = ops[q].rec.v[0];
                if (ook[q]) acc32<DIR, V, VW, V, CUBE>(ops[q], xv[q], ovf_base, Xc, sx, o[q].v);
            }
            // The next level's first batch reads records and inputs that no
            // level writes.  At the end of a level without blocks they are
            // requested before this batch's stores (its meta words arrived
            // with the neighbour values), so that the barrier's wait for the
            // stores and the wait for these loads are one round trip.
            if (last && !blocks && more) fetch_batch(cN, mN);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (ook[q]) {
                    st<V, VW>(reinterpret_cast<V*>(Xw + orow[q]), o[q]);
                    if (DIR == kRev && outp) {
                        Pack<V, VW> os;
#pragma unroll
                        for (int v = 0; v < VW; ++v) os.v[v] = oscale[q] * o[q].v[v];
                        const uint32_t irow = ((orow[q] - lane_off) >> xsh) + lane_off;
                        st<V, VW>(reinterpret_cast<V*>(reinterpret_cast<char*>(outp) + irow), os);
                    }
                }
            }
        }
        if (last) {
            // a level with blocks fetches the next level's first batch after
            // its block products (that state is not kept live across them)
            if (blocks)
                split_block_rhs<DIR, V, LPN, NT, CUBE>(sd, cC.d, meta, wtc, inc, in, ovf_base, Xc, sx, XROWB, lane_off, stage,
                                                 SB, cx, P, part, slot0, rl);
            group_barrier(g, P);
            if (first) {
                first = false;
                const unsigned xm = __hip_atomic_load(s.xmask + (size_t)alpha * kCtrStride, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                g.agent = __builtin_popcount(xm) != 1;
            }
            if (blocks) {
                if constexpr (B % 16 == 0)
                    split_block_solve_mfma<DIR, V, B, NT>(sd, cC.d, meta, wts, stage, SB, X, a.xB, outp, P, part);
                else
                    split_block_solve<DIR, V, B, NT>(sd, cC.d, meta, wts, stage, SB, X, a.xB, outp, P, part,
                                                     s.lds_rows, lds + s.stage_off);
                split_block_iterate<DIR, V, B, NT>(sd, cC.d, meta, wts, stage, SB, X, a.xB, outp, P, part, g);
                if (more) fetch_batch(cN, mN);
                group_barrier(g, P);
            }
            if (!more) break;
        }
        pre = last;
        cC = cN;
#pragma unroll
        for (int q = 0; q < U; ++q) mC[q] = mN[q];
        cursor_next<DIR, BATCH>(cN, sd, L, P, part);
    }
}

// Counters, XCD masks and the launch's abort word start from zero at every
// launch (a kernel, not a memset, so that the launch can be captured in a
// graph).  The sticky failure word is left alone: it stays set until the host
// has read it.
__global__ void k_split_reset(SplitArgs s, int S) {
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0) *s.abort_w = 0u;
    for (int t = t0; t < S; t += gridDim.x * blockDim.x) {
        s.ctr[(size_t)t * kCtrStride] = 0u;
        s.xmask[(size_t)t * kCtrStride] = 0u;
    }
}

}  // namespace fm
