// Internal declarations of the fmbtf library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fmbtf.h"

namespace fm {

// Thread-local error message behind fm_last_error().
void set_error(const char* fmt, ...);
void clear_error();

// ---------------------------------------------------------------------------
// Packed record format shared by the host packer and the kernels.
//
// Every node owns one record per traversal direction, stored in that
// direction's level order (position q):
//   meta word (uint64): bits 0..30  node id
//                       bit  31     node is a receiver (reverse records only)
//                       bits 32..57 offset of the node's extra weights in the
//                                   overflow area (only with > 3 neighbours)
//                       bits 58..63 neighbour mask
//   value record:       rec[q] = [c_node, w_1, w_2, w_3] (fixed 4 entries,
//                       unused entries 0); weights w_4.. of a node with more
//                       than three neighbours follow in the overflow area that
//                       starts after the N fixed records.
// Weights are listed in increasing mask-bit order.  Neighbour slot b: axis =
// b >> 1; side = b & 1; side 0 is node - stride[axis], side 1 is node +
// stride[axis].  In forward records the mask lists the predecessors j of the
// node with weight w_{node,j}; in reverse records it lists the successors i
// with weight w_{i,node}.  For members of a nontrivial SCC only the
// neighbours outside the component are listed; couplings inside the
// component live in the block's dense factors.
//
// States of the 26-neighbour (cube) stencil use a 26-bit mask in bits 32..57
// instead (bits 58..63 zero); slot b is the logical offset o in {-1,0,1}^3
// whose base-3 number (o_0 + 1) + 3 (o_1 + 1) + 9 (o_2 + 1), centre left out,
// is b (ascending slots are ascending node ids; the opposite of b is 25 - b).
// Their overflow offsets are in a per-position array of their own (fovf /
// rovf).
// ---------------------------------------------------------------------------
constexpr int kNodeBits = 31;
constexpr uint64_t kNodeMask = (1ull << kNodeBits) - 1;
constexpr uint64_t kRcvFlag = 1ull << 31;
constexpr int kOffShift = 32;
constexpr int kOffBits = 26;
constexpr uint64_t kOffMask = (1ull << kOffBits) - 1;
constexpr int kMaskShift = 58;
constexpr int kCubeMaskShift = 32;
constexpr uint64_t kCubeMask = (1ull << 26) - 1;

// Neighbour slots of the cube stencil: offset of slot b along each axis.
inline void cube_offset(int slot, int o[3]) {
    const int b = slot + (slot >= 13 ? 1 : 0);
    o[0] = b % 3 - 1;
    o[1] = (b / 3) % 3 - 1;
    o[2] = b / 9 - 1;
}

struct Packed {
    int32_t L_f = 0, L_r = 0, nblk = 0;
    // forward traversal
    std::vector<uint64_t> fmeta;       // [N]
    std::vector<double> fwts;          // [N][4] records, then the overflow area
    std::vector<int32_t> flvl_ptr;     // [L_f + 1] position range per level
    std::vector<int32_t> flvl_nsc;     // [L_f] scalar nodes at the start of each level
    std::vector<int32_t> fblk_ptr;     // [L_f + 1] range into fblk_id
    std::vector<int32_t> fblk_id;      // [nblk] blocks in forward level order
    // reverse traversal
    std::vector<uint64_t> rmeta;
    std::vector<double> rwts;
    std::vector<int32_t> rlvl_ptr, rlvl_nsc, rblk_ptr, rblk_id;
    // nontrivial SCC blocks: member m sits at fpos+m / rpos+m
    std::vector<int32_t> blk_k, blk_fpos, blk_rpos;
    std::vector<int64_t> blk_inv;      // offset of the k x k inverse in inv and invt
    std::vector<double> inv;           // A_C^{-1}, column-major (entry (i,j) at j*k + i)
    std::vector<double> invt;          // the same matrix row-major (entry (i,j) at i*k + j)
    std::vector<double> cal_nat;       // [N] calibration in natural order
    // receivers: receiver r samples sum_e rcv_wt[e] x[rcv_node[e]] over its
    // entries e in [rcv_ptr[r], rcv_ptr[r+1]) (a selection: one entry of weight 1)
    std::vector<int32_t> rcv_ptr;      // [R + 1]
    std::vector<int32_t> rcv_node;     // [E] node of each entry
    std::vector<double> rcv_wt;        // [E] weight of each entry
    std::vector<int32_t> rcvlvl_ptr;   // [L_r + 1] range of the sorted entries per reverse level
    std::vector<int32_t> rcv_pos;      // [E] reverse position of each entry (sorted)
    std::vector<int32_t> rcv_idx;      // [E] receiver of each sorted entry
    std::vector<double> rcv_ew;        // [E] weight of each sorted entry
    int32_t max_blk_k = 0;
    int64_t max_level_nodes = 0;
    // Large blocks solved iteratively (Neumann series of W_CC, no inverse):
    // blk_it[2b], blk_it[2b+1] = iterations of the primal and transpose solve
    // (both 0: a dense block with an inverse at blk_inv[b]; blk_inv[b] = -1
    // otherwise).  The in-block couplings of such a block, member order:
    // primal row i in sp_ptr[blk_sp[b] + i .. + i + 1) lists members j with
    // w_ij > 0 (sp_col, sp_w); transpose row j in spt_* the same way lists
    // members i with weight w_ij.
    std::vector<int32_t> blk_it;
    std::vector<int64_t> blk_sp;
    std::vector<int32_t> sp_ptr, sp_col, spt_ptr, spt_col;
    std::vector<double> sp_w, spt_w;
    int64_t max_blk_rows = 0;          // most FP64 rows one block stages (k, or 3k iterative)
    // cube stencil only: overflow offset of each position's further weights
    std::vector<int32_t> fovf, rovf;
    // records packed on the device by the GPU setup pass (fmeta / fwts /
    // rmeta / rwts then stay empty): device buffers the state owns until its
    // device state is built from them (index 0 forward, 1 reverse)
    struct DeviceRecords {
        void* meta[2] = {nullptr, nullptr};   // uint64 [N]
        void* wts[2] = {nullptr, nullptr};    // double [N * 4 + overflow + 4]
        int64_t nwts[2] = {0, 0};
        int device = -1;
    } drec;
    // off-grid point source (all empty for an on-grid source).  Seed node
    // seed_node[e] is an identity row whose right-hand side is
    // sum_i seed_w[i] ds[seed_col[i]] over i in [seed_ptr[e], seed_ptr[e+1]);
    // it has no forward position inside a level (the forward walk never
    // computes it: a pass before the walk writes it).
    std::vector<int32_t> seed_node, seed_ptr, seed_col;
    std::vector<double> seed_w;
    // direct term D_alpha: receiver r adds sum_i d_w[i] ds[d_col[i]] over
    // i in [d_ptr[r], d_ptr[r+1]) (its P entries are dropped)
    std::vector<int32_t> d_ptr, d_col;
    std::vector<double> d_w;
    // the transposes of both, grouped by target node for J^T: target
    // sc_tgt[t] receives sum_i sc_w[i] v_i over i in [sc_ptr[t], sc_ptr[t+1]),
    // v_i = lambda at node sc_idx[i] (sc_kind 0) or y at receiver sc_idx[i] (1)
    std::vector<int32_t> sc_tgt, sc_ptr, sc_idx;
    std::vector<uint8_t> sc_kind;
    std::vector<double> sc_w;
};

// An off-grid point source: logical coordinates xi, the seed region of
// max-norm radius rho around it, and the physical node coordinates X the
// straight-ray seed times are measured in.
struct PointSource {
    const double* X;   // [N][dim]
    double xi[3];
    double rho;
};

// Couplings computed elsewhere (the GPU setup pass) for an on-grid source:
// pmask [N], w6 [N][6], cal [N] exactly as parts 1-2 of build_state write
// them, and the count of violating edges (T_j > T_i over the edges j -> i).
// Optionally the graph work too: trim [N] marks the nodes that Kahn's
// elimination removes forward (bit 0: not on or downstream of a cycle) and
// backward (bit 1: not on or upstream of one), so the SCC search runs on
// the rest only (every cycle lies in it); levels() then computes the
// longest-path levels of the condensation DAG for the partition given as
// comp [N] (ncomp components, members cnodes[cptr[c] .. cptr[c+1])), with
// the predecessor / successor masks, into clev_f / clev_r [ncomp];
// it returns FM_OK or an FM_E* code with the message set.
struct Assembled {
    const uint8_t* pmask;
    const double* w6;
    const double* cal;
    int64_t n_vio;
    const uint8_t* trim = nullptr;
    int (*levels)(void* ctx, int64_t N, int32_t ncomp, const int32_t* comp, const int32_t* cptr,
                  const int32_t* cnodes, const uint32_t* pmask, const uint32_t* smask, int32_t* clev_f,
                  int32_t* clev_r) = nullptr;
    // and the records: pack() writes one direction's meta words and value
    // records (the host's format, bit for bit) on the device from the
    // placement pos_of [N], the components, masks, weights [N][6] and
    // calibration, rcv [N] marking receiver nodes (reverse direction)
    int (*pack)(void* ctx, bool fwd, int64_t N, const int32_t* pos_of, const int32_t* comp, const uint32_t* pmask,
                const uint32_t* smask, const double* w6, const double* cal, const uint8_t* rcv,
                Packed::DeviceRecords* out) = nullptr;
    void* ctx = nullptr;
};

struct DeviceState;   // defined in the HIP translation unit

struct HostState {
    int dim = 3;
    int64_t n[3] = {1, 1, 1};       // nodes per logical axis (axis 0 fastest)
    int64_t stride[3] = {1, 1, 1};
    int64_t N = 0;
    int64_t src = 0;
    int stencil = 6;                // 6: face-based upwinding; 26: cube stencil
    // natural-order operator: predecessor and successor slot masks, and the
    // weights, per slot ([N][6], 0 if none) for the face stencil, by rank in
    // ascending slot order ([N][3]) for the cube stencil (see weight())
    std::vector<uint32_t> pmask, smask;
    std::vector<double> wrow;
    std::vector<double> cal;        // [N]
    int nslot() const { return stencil == 26 ? 26 : 2 * dim; }
    // w_{p, neighbour in slot}
    double weight(int64_t p, int slot) const {
        if (stencil == 26) return wrow[(size_t)p * 3 + __builtin_popcount(pmask[p] & ((1u << slot) - 1u))];
        return wrow[(size_t)p * 6 + slot];
    }
    int64_t neighbour(int64_t p, int slot) const {
        if (stencil == 26) {
            int o[3];
            cube_offset(slot, o);
            return p + o[0] * stride[0] + o[1] * stride[1] + o[2] * stride[2];
        }
        return (slot & 1) ? p + stride[slot >> 1] : p - stride[slot >> 1];
    }
    int opposite(int slot) const { return stencil == 26 ? 25 - slot : slot ^ 1; }
    // graph
    std::vector<int32_t> comp;      // component id: ascending forward level, then smallest member
    int32_t ncomp = 0;
    std::vector<int32_t> cptr, cnodes;      // members per component (ascending node id)
    std::vector<int32_t> clev_f, clev_r;    // per component
    Packed pk;
    fm_stats stats{};
    DeviceState* dev = nullptr;
    // the grid shape, to check that the states of one batch agree
    bool same_grid(const HostState& o) const {
        return dim == o.dim && n[0] == o.n[0] && n[1] == o.n[1] && n[2] == o.n[2] && stencil == o.stencil;
    }
};

}  // namespace fm

// The opaque handle of the C ABI is the host state itself.
struct fm_state : fm::HostState {};

namespace fm {

// Host setup (setup.cpp).  Returns FM_OK or an FM_E* code with the message set.
// Receiver r is sum_k rcv_w[r*K + k] x[rcv[r*K + k]] (rcv_w NULL: weights 1);
// entries of weight 0 are dropped.
// With pre (on-grid sources only), parts 1-2 take its couplings and T may
// be NULL (the caller has checked it).
int build_state(const fm_grid* g, const double* T, const double* s, int64_t src,
                const int64_t* rcv, const double* rcv_w, int32_t n_rcv, int32_t K, fm_state** out,
                const PointSource* ps = nullptr, const Assembled* pre = nullptr);

// Staging rows of block b: its right-hand sides, plus two iterate buffers
// when it is solved iteratively.
inline int64_t block_stage_rows(const Packed& pk, int32_t b) {
    return (int64_t)pk.blk_k[b] * (pk.blk_it[2 * (size_t)b] ? 3 : 1);
}

// Blocks of at least this many nodes are solved iteratively when the Neumann
// series reaches full precision within kNeumannMax terms (<= 0: never).
constexpr int32_t kIterativeMinDefault = 1024;
constexpr int32_t kNeumannMax = 200;
void set_iterative_min(int32_t k_min);
int32_t iterative_min();

// Natural-order records of the full operator (W for fwd, W^T otherwise) in
// the packed record format, for the directional-sweeping comparison baseline.
void pack_natural(const HostState* st, bool fwd, std::vector<uint64_t>& meta, std::vector<double>& rec);

// Device side (device.hip).
int upload_state(HostState* st);
void free_device_state(HostState* st);   // also frees records packed on the device

}  // namespace fm
