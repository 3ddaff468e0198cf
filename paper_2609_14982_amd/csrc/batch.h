// Device-side structures shared by the HIP translation units of fmbtf.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace fm {

// An off-grid point source (Section 3.1 source-seed rows, the direct term of
// eq. (source-jacobian)); a state whose source sits on a node has none.
struct PtDev {
    const int32_t* seed_node;   // [n_seed] identity rows the forward walk skips
    const int32_t* seed_ptr;    // [n_seed + 1] their right-hand-side entries
    const int32_t* seed_col;    //   node of each entry
    const double* seed_w;       //   weight of each entry
    const int32_t* d_ptr;       // [R + 1] entries of D per receiver (none: not direct)
    const int32_t* d_col;
    const double* d_w;
    const int32_t* sc_tgt;      // [n_tgt] targets of the transposes of both, ascending
    const int32_t* sc_ptr;      // [n_tgt + 1]
    const int32_t* sc_idx;      //   seed node (kind 0) or receiver (kind 1)
    const uint8_t* sc_kind;
    const double* sc_w;
    int32_t n_seed, n_tgt;
};

// The same transposes of every off-grid source of a batch, grouped by target
// node over the batch (J^T summed over sources): target tgt[t] receives
// sum_i w[i] v_i over i in [ptr[t], ptr[t+1]), sources ascending.
struct UnionDev {
    const int32_t* tgt;
    const int32_t* ptr;
    const int32_t* alpha;
    const int32_t* idx;
    const uint8_t* kind;
    const double* w;
    int32_t n;
};

struct SrcDev {
    const uint64_t* fmeta;
    const void* fwts;
    const int32_t* flvl_ptr;
    const int32_t* flvl_nsc;
    const int32_t* fblk_ptr;
    const int32_t* fblk_id;
    const uint64_t* rmeta;
    const void* rwts;
    const int32_t* rlvl_ptr;
    const int32_t* rlvl_nsc;
    const int32_t* rblk_ptr;
    const int32_t* rblk_id;
    const int32_t* blk_k;
    const int32_t* blk_fpos;
    const int32_t* blk_rpos;
    const int64_t* blk_inv;
    const int64_t* blk_moff;    // first staging row of each block (prefix sum of k, 3k iterative)
    const int32_t* blk_it;      // [2 nblk] series terms, primal and transpose (0: dense inverse)
    const int64_t* blk_sp;      // [nblk] first row pointer of an iterative block's couplings
    const int32_t* sp_ptr;      // in-block couplings, primal rows (member order)
    const int32_t* sp_col;
    const double* sp_w;
    const int32_t* spt_ptr;     // the same, transpose rows
    const int32_t* spt_col;
    const double* spt_w;
    const double* inv;
    const double* invt;
    const void* cal_nat;
    const int32_t* rcv_ptr;     // [R + 1] entries of each receiver
    const int32_t* rcv_node;    // [E] node of each entry
    const double* rcv_wt;       // [E] weight of each entry
    const int32_t* rcvlvl_ptr;  // [L_r + 1] sorted entries per reverse level
    const int32_t* rcv_pos;     // [E] reverse position of each sorted entry
    const int32_t* rcv_idx;     // [E] receiver of each sorted entry
    const double* rcv_ew;       // [E] weight of each sorted entry
    const PtDev* pt;            // off-grid source tables, or nullptr
    const int32_t* fovf;        // cube stencil: overflow offset per position, or nullptr
    const int32_t* rovf;
    int32_t L_f, L_r, n_rcv, n_ent;
};

struct DeviceState {
    void* blob_nat = nullptr;    // natural-order records for the sweeping baseline
    void* blob_nat32 = nullptr;
    const void* nat[4] = {nullptr, nullptr, nullptr, nullptr};     // fmeta, frec, rmeta, rrec
    const void* nat32[2] = {nullptr, nullptr};                     // frec, rrec in FP32
    void* blob = nullptr;        // all FP64 arrays and integer tables
    void* blob32 = nullptr;      // FP32 copies of the records and calibration
    SrcDev d{};                  // pointers into blob (FP64 records)
    const void* fwts32 = nullptr;
    const void* rwts32 = nullptr;
    const void* cal32 = nullptr;
    size_t nwts[2] = {0, 0};     // doubles in the forward / reverse value records
    int device = -1;
};

}  // namespace fm

struct fm_batch {
    std::vector<fm::HostState*> states;
    int32_t S = 0, B = 0, prec = 64, R = 0;
    fm_tuning tun{};
    hipStream_t stream = nullptr;
    fm::SrcDev* d_src = nullptr;     // [S]
    void* scratch = nullptr;         // [S][N][xB] of the batch precision
    int32_t xB = 0;                  // values per scratch row (B, or B padded to whole 128-byte lines)
    int64_t N = 0;
    int64_t st1 = 1, st2 = 1;
    int device = -1;
    size_t lds_bytes = 0;
    int32_t grid = 0, per_xcd = 0, items = 0;
    void* nat_dev = nullptr;         // [S] NatDev, created by the first sweeping-baseline call
    int32_t* cycles_dev = nullptr;   // [items]
    // node split (tun.split > 1)
    int32_t split_grid = 0, split_per_xcd = 0, split_items = 0, split_lds_rows = 0;
    int32_t split_rcv_lds = 0, split_stage_off = 0;
    size_t split_lds = 0;
    int64_t stage_rows = 0;
    void* stage = nullptr;           // [S][stage_rows][B] FP64 block right-hand sides
    unsigned* sync = nullptr;        // counters [S*32], XCD masks [S*32], abort word
    int32_t* wg_map = nullptr;       // balanced split: [grid] source << 8 | part (-1 idle), then [S] P per source
    // off-grid sources: the most seed rows and transpose targets of one source
    int32_t max_seed = 0, max_tgt = 0;
    void* union_blob = nullptr;      // UnionDev arrays (J^T summed)
    fm::UnionDev uni{};
};

namespace fm {

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                    \
            return FM_EHIP;                                                              \
        }                                                                                \
    } while (0)

// Loads through the pointers stored in SrcDev: the compiler cannot infer
// their address space and would emit FLAT loads, which also count against the
// LDS/scalar wait counter; these name the global address space explicitly.
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)(p);
}

template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)(p);
}

struct ApplyArgs {
    const SrcDev* src;
    int32_t S, B, ngroups, items, per_xcd, xcd_aware;
    int64_t N;
    int64_t st1, st2;       // node strides of logical axes 1 and 2
    int32_t R;              // receivers per source (receiver layouts)
    int32_t in_mode, out_mode;
    int32_t cube;           // cube-stencil records (26-bit neighbour masks)
    int32_t xB;             // values per row of work ([S][N][xB], xB >= B; rows padded to 128 bytes
                            // when work is the batch's own scratch of a node-split batch)
    const void* in;         // J: ds ; J^T: w
    void* out;              // J: nodes output (or unused) ; J^T: per-source output
    void* work;             // J: X (out or scratch) ; J^T: lambda scratch
};

// device.hip
int apply_J(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode);
int apply_JT(fm_batch* b, const void* w, int32_t w_mode, void* out, int32_t out_mode);
ApplyArgs batch_args(const fm_batch* b);
const void* const* batch_calibration(const fm_batch* b);

}  // namespace fm
