// Device side of fmbtf for gfx950 (CDNA4): state upload, batches and the
// apply kernels.
//
// Work decomposition.  One workgroup owns one (source, group of RG
// right-hand sides) pair and walks that source's condensation levels in
// order (primal: Section 4.1, Proposition 3; transpose: Section 4.3).  Inside
// a level every singleton is independent, so the workgroup's threads take the
// level's nodes RG lanes per node (one lane per right-hand side, so a node's
// RG values are one contiguous segment of the [N][B] vectors), and every
// nontrivial SCC block of the level is solved cooperatively with its
// right-hand sides staged in LDS.  A workgroup barrier separates levels; no
// workgroup ever waits on another, so the launch needs no global
// synchronisation, no atomics and no cross-XCD cache maintenance.  The
// workgroups of one source are placed on one XCD so that they share that
// XCD's L2 copy of the source's records.
//
// SCC blocks apply A_C^{-1}, formed once on the host from the pivoted LU
// P_C A_C = L_C U_C of Section 4.3, as a dense matvec; the transpose solve
// uses the same matrix read transposed (no second factorisation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"

namespace fm {

// ---------------------------------------------------------------------------
// upload
// ---------------------------------------------------------------------------
namespace {

struct Arena {
    size_t off = 0;
    template <class T>
    size_t add(size_t count) {
        off = (off + 255) & ~size_t(255);
        size_t at = off;
        off += count * sizeof(T);
        return at;
    }
};

template <class T>
int put(char* base, size_t at, const std::vector<T>& v) {
    if (v.empty()) return FM_OK;
    hipError_t e = hipMemcpy(base + at, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("hipMemcpy of state arrays failed: %s", hipGetErrorString(e));
        return FM_EHIP;
    }
    return FM_OK;
}

}  // namespace

static void free_device_records(Packed& pk) {
    for (int d = 0; d < 2; d++) {
        if (pk.drec.meta[d]) (void)hipFree(pk.drec.meta[d]);
        if (pk.drec.wts[d]) (void)hipFree(pk.drec.wts[d]);
        pk.drec.meta[d] = pk.drec.wts[d] = nullptr;
    }
}

int upload_state(HostState* st) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (st->dev && st->dev->device == dev) return FM_OK;
    if (st->dev) {
        set_error("state already lives on device %d (current device %d)", st->dev->device, dev);
        return FM_ESTATE;
    }
    const Packed& pk = st->pk;
    Arena ar;
    // records packed on the device by the GPU setup pass are copied from there
    const bool drec = pk.drec.meta[0] != nullptr;
    if (drec && pk.drec.device != dev) {
        set_error("the state's records were packed on device %d, not the current device %d", pk.drec.device, dev);
        return FM_EINVAL;
    }
    const size_t n_fmeta = drec ? (size_t)st->N : pk.fmeta.size(), n_rmeta = drec ? (size_t)st->N : pk.rmeta.size();
    const size_t n_fwts = drec ? (size_t)pk.drec.nwts[0] : pk.fwts.size();
    const size_t n_rwts = drec ? (size_t)pk.drec.nwts[1] : pk.rwts.size();
    size_t o_fmeta = ar.add<uint64_t>(n_fmeta);
    size_t o_fwts = ar.add<double>(n_fwts);
    size_t o_flp = ar.add<int32_t>(pk.flvl_ptr.size());
    size_t o_fln = ar.add<int32_t>(pk.flvl_nsc.size());
    size_t o_fbp = ar.add<int32_t>(pk.fblk_ptr.size());
    size_t o_fbi = ar.add<int32_t>(pk.fblk_id.size());
    size_t o_rmeta = ar.add<uint64_t>(n_rmeta);
    size_t o_rwts = ar.add<double>(n_rwts);
    size_t o_rlp = ar.add<int32_t>(pk.rlvl_ptr.size());
    size_t o_rln = ar.add<int32_t>(pk.rlvl_nsc.size());
    size_t o_rbp = ar.add<int32_t>(pk.rblk_ptr.size());
    size_t o_rbi = ar.add<int32_t>(pk.rblk_id.size());
    size_t o_bk = ar.add<int32_t>(pk.blk_k.size());
    size_t o_bfp = ar.add<int32_t>(pk.blk_fpos.size());
    size_t o_brp = ar.add<int32_t>(pk.blk_rpos.size());
    size_t o_binv = ar.add<int64_t>(pk.blk_inv.size());
    std::vector<int64_t> moff(pk.blk_k.size());
    {
        int64_t acc = 0;
        for (size_t i = 0; i < pk.blk_k.size(); i++) { moff[i] = acc; acc += block_stage_rows(pk, (int32_t)i); }
    }
    size_t o_moff = ar.add<int64_t>(moff.size());
    size_t o_bit = ar.add<int32_t>(pk.blk_it.size());
    size_t o_bsp = ar.add<int64_t>(pk.blk_sp.size());
    size_t o_spp = ar.add<int32_t>(pk.sp_ptr.size());
    size_t o_spc = ar.add<int32_t>(pk.sp_col.size());
    size_t o_spw = ar.add<double>(pk.sp_w.size());
    size_t o_stp = ar.add<int32_t>(pk.spt_ptr.size());
    size_t o_stc = ar.add<int32_t>(pk.spt_col.size());
    size_t o_stw = ar.add<double>(pk.spt_w.size());
    size_t o_inv = ar.add<double>(pk.inv.size());
    size_t o_invt = ar.add<double>(pk.invt.size());
    size_t o_cal = ar.add<double>(pk.cal_nat.size());
    size_t o_rptr = ar.add<int32_t>(pk.rcv_ptr.size());
    size_t o_rn = ar.add<int32_t>(pk.rcv_node.size());
    size_t o_rwt = ar.add<double>(pk.rcv_wt.size());
    size_t o_rlv = ar.add<int32_t>(pk.rcvlvl_ptr.size());
    size_t o_rp = ar.add<int32_t>(pk.rcv_pos.size());
    size_t o_ri = ar.add<int32_t>(pk.rcv_idx.size());
    size_t o_rew = ar.add<double>(pk.rcv_ew.size());
    // an off-grid source's tables and the PtDev that points at them
    const bool has_pt = !pk.seed_node.empty();
    size_t o_sn = ar.add<int32_t>(pk.seed_node.size());
    size_t o_sp = ar.add<int32_t>(pk.seed_ptr.size());
    size_t o_sc = ar.add<int32_t>(pk.seed_col.size());
    size_t o_sw = ar.add<double>(pk.seed_w.size());
    size_t o_dp = ar.add<int32_t>(pk.d_ptr.size());
    size_t o_dc = ar.add<int32_t>(pk.d_col.size());
    size_t o_dw = ar.add<double>(pk.d_w.size());
    size_t o_tt = ar.add<int32_t>(pk.sc_tgt.size());
    size_t o_tp = ar.add<int32_t>(pk.sc_ptr.size());
    size_t o_ti = ar.add<int32_t>(pk.sc_idx.size());
    size_t o_tk = ar.add<uint8_t>(pk.sc_kind.size());
    size_t o_tw = ar.add<double>(pk.sc_w.size());
    size_t o_pt = ar.add<PtDev>(has_pt ? 1 : 0);
    size_t o_fovf = ar.add<int32_t>(pk.fovf.size());
    size_t o_rovf = ar.add<int32_t>(pk.rovf.size());
    size_t total = ar.add<char>(0) + 256;
    DeviceState* ds = new DeviceState();
    hipError_t e = hipMalloc(&ds->blob, total);
    if (e != hipSuccess) {
        delete ds;
        set_error("hipMalloc(%zu) for a state failed: %s", total, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    char* b = (char*)ds->blob;
    int rc = FM_OK;
    if (drec) {
        const void* src[4] = {pk.drec.meta[0], pk.drec.wts[0], pk.drec.meta[1], pk.drec.wts[1]};
        const size_t at[4] = {o_fmeta, o_fwts, o_rmeta, o_rwts};
        const size_t bytes[4] = {8 * n_fmeta, 8 * n_fwts, 8 * n_rmeta, 8 * n_rwts};
        for (int i = 0; i < 4 && rc == FM_OK; i++) {
            const hipError_t ce = hipMemcpy(b + at[i], src[i], bytes[i], hipMemcpyDeviceToDevice);
            if (ce != hipSuccess) {
                set_error("copy of device-packed records failed: %s", hipGetErrorString(ce));
                rc = FM_EHIP;
            }
        }
    } else {
        rc = rc ? rc : put(b, o_fmeta, pk.fmeta);
        rc = rc ? rc : put(b, o_fwts, pk.fwts);
    }
    rc = rc ? rc : put(b, o_flp, pk.flvl_ptr);
    rc = rc ? rc : put(b, o_fln, pk.flvl_nsc);
    rc = rc ? rc : put(b, o_fbp, pk.fblk_ptr);
    rc = rc ? rc : put(b, o_fbi, pk.fblk_id);
    if (!drec) {
        rc = rc ? rc : put(b, o_rmeta, pk.rmeta);
        rc = rc ? rc : put(b, o_rwts, pk.rwts);
    }
    rc = rc ? rc : put(b, o_rlp, pk.rlvl_ptr);
    rc = rc ? rc : put(b, o_rln, pk.rlvl_nsc);
    rc = rc ? rc : put(b, o_rbp, pk.rblk_ptr);
    rc = rc ? rc : put(b, o_rbi, pk.rblk_id);
    rc = rc ? rc : put(b, o_bk, pk.blk_k);
    rc = rc ? rc : put(b, o_bfp, pk.blk_fpos);
    rc = rc ? rc : put(b, o_brp, pk.blk_rpos);
    rc = rc ? rc : put(b, o_binv, pk.blk_inv);
    rc = rc ? rc : put(b, o_moff, moff);
    rc = rc ? rc : put(b, o_bit, pk.blk_it);
    rc = rc ? rc : put(b, o_bsp, pk.blk_sp);
    rc = rc ? rc : put(b, o_spp, pk.sp_ptr);
    rc = rc ? rc : put(b, o_spc, pk.sp_col);
    rc = rc ? rc : put(b, o_spw, pk.sp_w);
    rc = rc ? rc : put(b, o_stp, pk.spt_ptr);
    rc = rc ? rc : put(b, o_stc, pk.spt_col);
    rc = rc ? rc : put(b, o_stw, pk.spt_w);
    rc = rc ? rc : put(b, o_inv, pk.inv);
    rc = rc ? rc : put(b, o_invt, pk.invt);
    rc = rc ? rc : put(b, o_cal, pk.cal_nat);
    rc = rc ? rc : put(b, o_rptr, pk.rcv_ptr);
    rc = rc ? rc : put(b, o_rn, pk.rcv_node);
    rc = rc ? rc : put(b, o_rwt, pk.rcv_wt);
    rc = rc ? rc : put(b, o_rlv, pk.rcvlvl_ptr);
    rc = rc ? rc : put(b, o_rp, pk.rcv_pos);
    rc = rc ? rc : put(b, o_ri, pk.rcv_idx);
    rc = rc ? rc : put(b, o_rew, pk.rcv_ew);
    rc = rc ? rc : put(b, o_fovf, pk.fovf);
    rc = rc ? rc : put(b, o_rovf, pk.rovf);
    if (has_pt) {
        rc = rc ? rc : put(b, o_sn, pk.seed_node);
        rc = rc ? rc : put(b, o_sp, pk.seed_ptr);
        rc = rc ? rc : put(b, o_sc, pk.seed_col);
        rc = rc ? rc : put(b, o_sw, pk.seed_w);
        rc = rc ? rc : put(b, o_dp, pk.d_ptr);
        rc = rc ? rc : put(b, o_dc, pk.d_col);
        rc = rc ? rc : put(b, o_dw, pk.d_w);
        rc = rc ? rc : put(b, o_tt, pk.sc_tgt);
        rc = rc ? rc : put(b, o_tp, pk.sc_ptr);
        rc = rc ? rc : put(b, o_ti, pk.sc_idx);
        rc = rc ? rc : put(b, o_tk, pk.sc_kind);
        rc = rc ? rc : put(b, o_tw, pk.sc_w);
        PtDev h{};
        h.seed_node = (const int32_t*)(b + o_sn);
        h.seed_ptr = (const int32_t*)(b + o_sp);
        h.seed_col = (const int32_t*)(b + o_sc);
        h.seed_w = (const double*)(b + o_sw);
        h.d_ptr = (const int32_t*)(b + o_dp);
        h.d_col = (const int32_t*)(b + o_dc);
        h.d_w = (const double*)(b + o_dw);
        h.sc_tgt = (const int32_t*)(b + o_tt);
        h.sc_ptr = (const int32_t*)(b + o_tp);
        h.sc_idx = (const int32_t*)(b + o_ti);
        h.sc_kind = (const uint8_t*)(b + o_tk);
        h.sc_w = (const double*)(b + o_tw);
        h.n_seed = (int32_t)pk.seed_node.size();
        h.n_tgt = (int32_t)pk.sc_tgt.size();
        rc = rc ? rc : put(b, o_pt, std::vector<PtDev>(1, h));
    }
    if (rc != FM_OK) {
        (void)hipFree(ds->blob);
        delete ds;
        return rc;
    }
    SrcDev& d = ds->d;
    d.fmeta = (const uint64_t*)(b + o_fmeta);
    d.fwts = b + o_fwts;
    d.flvl_ptr = (const int32_t*)(b + o_flp);
    d.flvl_nsc = (const int32_t*)(b + o_fln);
    d.fblk_ptr = (const int32_t*)(b + o_fbp);
    d.fblk_id = (const int32_t*)(b + o_fbi);
    d.rmeta = (const uint64_t*)(b + o_rmeta);
    d.rwts = b + o_rwts;
    d.rlvl_ptr = (const int32_t*)(b + o_rlp);
    d.rlvl_nsc = (const int32_t*)(b + o_rln);
    d.rblk_ptr = (const int32_t*)(b + o_rbp);
    d.rblk_id = (const int32_t*)(b + o_rbi);
    d.blk_k = (const int32_t*)(b + o_bk);
    d.blk_fpos = (const int32_t*)(b + o_bfp);
    d.blk_rpos = (const int32_t*)(b + o_brp);
    d.blk_inv = (const int64_t*)(b + o_binv);
    d.blk_moff = (const int64_t*)(b + o_moff);
    d.blk_it = (const int32_t*)(b + o_bit);
    d.blk_sp = (const int64_t*)(b + o_bsp);
    d.sp_ptr = (const int32_t*)(b + o_spp);
    d.sp_col = (const int32_t*)(b + o_spc);
    d.sp_w = (const double*)(b + o_spw);
    d.spt_ptr = (const int32_t*)(b + o_stp);
    d.spt_col = (const int32_t*)(b + o_stc);
    d.spt_w = (const double*)(b + o_stw);
    d.inv = (const double*)(b + o_inv);
    d.invt = (const double*)(b + o_invt);
    d.cal_nat = b + o_cal;
    d.rcv_ptr = (const int32_t*)(b + o_rptr);
    d.rcv_node = (const int32_t*)(b + o_rn);
    d.rcv_wt = (const double*)(b + o_rwt);
    d.rcvlvl_ptr = (const int32_t*)(b + o_rlv);
    d.rcv_pos = (const int32_t*)(b + o_rp);
    d.rcv_idx = (const int32_t*)(b + o_ri);
    d.rcv_ew = (const double*)(b + o_rew);
    d.pt = has_pt ? (const PtDev*)(b + o_pt) : nullptr;
    d.fovf = pk.fovf.empty() ? nullptr : (const int32_t*)(b + o_fovf);
    d.rovf = pk.rovf.empty() ? nullptr : (const int32_t*)(b + o_rovf);
    d.L_f = pk.L_f;
    d.L_r = pk.L_r;
    d.n_rcv = (int32_t)pk.rcv_ptr.size() - 1;
    d.n_ent = (int32_t)pk.rcv_node.size();
    ds->device = dev;
    ds->nwts[0] = n_fwts;
    ds->nwts[1] = n_rwts;
    st->dev = ds;
    if (drec) {
        (void)hipDeviceSynchronize();   // the copies out of them are done
        free_device_records(st->pk);
    }
    return FM_OK;
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

static int upload_fp32(HostState* st) {
    DeviceState* ds = st->dev;
    if (ds->blob32) return FM_OK;
    const Packed& pk = st->pk;
    // records packed on the device exist only there: converted there
    const bool on_dev = pk.fwts.empty() && ds->nwts[0] > 0;
    std::vector<float> f, r;
    if (!on_dev) {
        f.assign(pk.fwts.begin(), pk.fwts.end());
        r.assign(pk.rwts.begin(), pk.rwts.end());
    }
    std::vector<float> c(pk.cal_nat.begin(), pk.cal_nat.end());
    Arena ar;
    size_t of = ar.add<float>(on_dev ? ds->nwts[0] : f.size()), orr = ar.add<float>(on_dev ? ds->nwts[1] : r.size()),
           oc = ar.add<float>(c.size());
    size_t total = ar.add<char>(0) + 256;
    hipError_t e = hipMalloc(&ds->blob32, total);
    if (e != hipSuccess) {
        ds->blob32 = nullptr;
        set_error("hipMalloc(%zu) for FP32 records failed: %s", total, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    char* b = (char*)ds->blob32;
    int rc = FM_OK;
    if (on_dev) {
        const int64_t nn[2] = {(int64_t)ds->nwts[0], (int64_t)ds->nwts[1]};
        const void* srcs[2] = {ds->d.fwts, ds->d.rwts};
        const size_t offs[2] = {of, orr};
        for (int i = 0; i < 2; i++) {
            const int grid = (int)std::min<int64_t>((nn[i] + 255) / 256, 65535);
            hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(256), 0, nullptr, (const double*)srcs[i],
                               (float*)(b + offs[i]), nn[i]);
        }
        const hipError_t ce = hipGetLastError();
        if (ce != hipSuccess) {
            set_error("FP32 conversion of the records failed: %s", hipGetErrorString(ce));
            return FM_EHIP;
        }
    } else {
        rc = put(b, of, f);
        rc = rc ? rc : put(b, orr, r);
    }
    rc = rc ? rc : put(b, oc, c);
    if (rc) return rc;
    ds->fwts32 = b + of;
    ds->rwts32 = b + orr;
    ds->cal32 = b + oc;
    return FM_OK;
}

void free_device_state(HostState* st) {
    free_device_records(st->pk);
    if (!st->dev) return;
    if (st->dev->blob_nat) (void)hipFree(st->dev->blob_nat);
    if (st->dev->blob_nat32) (void)hipFree(st->dev->blob_nat32);
    if (st->dev->blob) (void)hipFree(st->dev->blob);
    if (st->dev->blob32) (void)hipFree(st->dev->blob32);
    delete st->dev;
    st->dev = nullptr;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

}  // namespace fm

#include "sweep.h"
#include "split.h"
#include "baseline.h"

namespace fm {

// out[alpha][r][b] = sum_e w_e X[alpha][node_e][b] over receiver r's
// entries, in entry order (P_alpha, Section 4.4; a selection when each
// receiver has one entry of weight 1)
template <typename V>
__global__ void k_gather_receivers(ApplyArgs a) {
    const int64_t total = (int64_t)a.S * a.R * a.B;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t % a.B;
        const int64_t rr = (t / a.B) % a.R;
        const int64_t alpha = t / ((int64_t)a.B * a.R);
        const SrcDev& sd = a.src[alpha];
        const V* x = (const V*)a.work + alpha * a.N * a.xB + b;
        V acc = (V)0;
        for (int32_t e = sd.rcv_ptr[rr]; e < sd.rcv_ptr[rr + 1]; ++e)
            acc += (V)sd.rcv_wt[e] * x[(int64_t)sd.rcv_node[e] * a.xB];
        if (sd.pt) {
            // a receiver an off-grid source reaches directly: its row of D
            // applied to ds (it has no entries above)
            const PtDev* pt = sd.pt;
            const V* ds = (const V*)a.in + (a.in_mode == FM_DS_PER_PAIR ? alpha * a.N * a.B : 0) + b;
            for (int32_t i = pt->d_ptr[rr]; i < pt->d_ptr[rr + 1]; ++i)
                acc += (V)pt->d_w[i] * ds[(int64_t)pt->d_col[i] * a.B];
        }
        ((V*)a.out)[t] = acc;
    }
}

// The seed rows of off-grid sources, before the forward walk (which skips
// them): X[alpha][p][b] = sum_i seed_w[i] ds[seed_col[i]][b], the derivative
// of the straight-ray seed time (Section 3.2's right-hand side for
// source-seed rows).
template <typename V>
__global__ void k_seed_rows(ApplyArgs a, int32_t max_seed) {
    const int64_t total = (int64_t)a.S * max_seed * a.B;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t % a.B;
        const int32_t e = (int32_t)((t / a.B) % max_seed);
        const int64_t alpha = t / ((int64_t)a.B * max_seed);
        const PtDev* pt = a.src[alpha].pt;
        if (!pt || e >= pt->n_seed) continue;
        const V* ds = (const V*)a.in + (a.in_mode == FM_DS_PER_PAIR ? alpha * a.N * a.B : 0) + b;
        double acc = 0.0;
        for (int32_t i = pt->seed_ptr[e]; i < pt->seed_ptr[e + 1]; ++i)
            acc += pt->seed_w[i] * (double)ds[(int64_t)pt->seed_col[i] * a.B];
        ((V*)a.work)[(alpha * a.N + pt->seed_node[e]) * a.xB + b] = (V)acc;
    }
}

// J^T per source, after the reverse walk wrote c lambda: each off-grid
// source adds the transposes of its seed rows (lambda at the seeds) and of
// D (receiver data, when the input is receiver data) at their targets,
// one thread per (source, target, rhs), so no two threads share an output.
template <typename V>
__global__ void k_seed_scatter(ApplyArgs a, int32_t max_tgt) {
    const int64_t total = (int64_t)a.S * max_tgt * a.B;
    const bool rcv = a.in_mode == FM_W_RECEIVERS;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t % a.B;
        const int32_t e = (int32_t)((t / a.B) % max_tgt);
        const int64_t alpha = t / ((int64_t)a.B * max_tgt);
        const PtDev* pt = a.src[alpha].pt;
        if (!pt || e >= pt->n_tgt) continue;
        const V* lam = (const V*)a.work + alpha * a.N * a.xB + b;
        const V* y = (const V*)a.in + alpha * (int64_t)a.R * a.B + b;
        double acc = 0.0;
        for (int32_t i = pt->sc_ptr[e]; i < pt->sc_ptr[e + 1]; ++i) {
            if (pt->sc_kind[i] == 0) acc += pt->sc_w[i] * (double)lam[(int64_t)pt->sc_idx[i] * a.xB];
            else if (rcv) acc += pt->sc_w[i] * (double)y[(int64_t)pt->sc_idx[i] * a.B];
        }
        V* o = (V*)a.out + (alpha * a.N + pt->sc_tgt[e]) * a.B + b;
        *o = (V)((double)*o + acc);
    }
}

// J^T summed over sources, after the source sum: the same transposes of
// every off-grid source, grouped by target over the batch (sources
// ascending inside a target), one thread per (target, rhs).
template <typename V>
__global__ void k_union_scatter(ApplyArgs a, UnionDev u) {
    const int64_t total = (int64_t)u.n * a.B;
    const bool rcv = a.in_mode == FM_W_RECEIVERS;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t % a.B;
        const int64_t e = t / a.B;
        double acc = 0.0;
        for (int32_t i = u.ptr[e]; i < u.ptr[e + 1]; ++i) {
            const int64_t alpha = u.alpha[i];
            if (u.kind[i] == 0)
                acc += u.w[i] * (double)((const V*)a.work)[(alpha * a.N + u.idx[i]) * a.xB + b];
            else if (rcv)
                acc += u.w[i] * (double)((const V*)a.in)[(alpha * a.R + u.idx[i]) * a.B + b];
        }
        V* o = (V*)a.out + (int64_t)u.tgt[e] * a.B + b;
        *o = (V)((double)*o + acc);
    }
}

// g[n][b] = sum_alpha c_alpha[n] lambda_alpha[n][b], sources in ascending
// order (Section 4.4).  A streaming reduction: each thread takes VW
// consecutive values of one node (one 16-byte access per source) and keeps
// the accesses of SU sources in flight; lambda is read once, so its loads
// are non-temporal, and every load names the global address space.
// PAD: work rows hold a.xB > B values (padded scratch); otherwise xB = B and
// the addressing is the plain [S][N][B] one.
template <typename V, bool PAD>
__global__ void k_sum_sources(ApplyArgs a, const void* const* cal) {
    constexpr int VW = 16 / (int)sizeof(V);
    constexpr int SU = 16;
    const int64_t NB = a.N * a.B;
    const int64_t NXB = a.N * a.xB;          // one source's rows in work (xB >= B values each)
    const V* __restrict__ work = (const V*)a.work;
    V* __restrict__ out = (V*)a.out;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (a.B % VW == 0) {
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NB / VW; t += stride) {
            const int64_t e0 = t * VW;
            const int64_t node = e0 / a.B;
            const int64_t w0 = PAD ? node * a.xB + (e0 - node * a.B) : e0;
            V acc[VW];
#pragma unroll
            for (int v = 0; v < VW; ++v) acc[v] = (V)0;
            for (int a0 = 0; a0 < a.S; a0 += SU) {
                Pack<V, VW> x[SU];
                V c[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    if (a0 + u < a.S) {
                        x[u] = ld_stream<V, VW>(work + (int64_t)(a0 + u) * NXB + w0);
                        c[u] = gld((const V*)gld(cal + (a0 + u)) + node);
                    }
                }
#pragma unroll
                for (int u = 0; u < SU; ++u)
                    if (a0 + u < a.S) {
#pragma unroll
                        for (int v = 0; v < VW; ++v) acc[v] += c[u] * x[u].v[v];
                    }
            }
            Pack<V, VW> o;
#pragma unroll
            for (int v = 0; v < VW; ++v) o.v[v] = acc[v];
            st<V, VW>(out + e0, o);
        }
    } else {
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NB; t += stride) {
            const int64_t node = t / a.B;
            V acc = (V)0;
            const int64_t w0 = PAD ? node * a.xB + (t - node * a.B) : t;
            for (int alpha = 0; alpha < a.S; ++alpha) acc += ((const V*)cal[alpha])[node] * work[alpha * NXB + w0];
            out[t] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// batch and launches
// ---------------------------------------------------------------------------

// VW values per lane access: 16 bytes (2 doubles, 4 floats) or the whole
// group when it is smaller.
template <typename V, int RG>
constexpr int lane_width() {
    return RG < (int)(16 / sizeof(V)) ? RG : (int)(16 / sizeof(V));
}

template <int DIR, typename V, int RG, int NT, int U>
static hipError_t launch_one(const ApplyArgs& a, int grid, size_t lds, hipStream_t s) {
    constexpr int VW = lane_width<V, RG>();
    // raise the dynamic-LDS limit once per kernel and device, outside any
    // stream capture that later launches may be part of
    static int attr_device = -1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (attr_device != dev) {
        e = hipFuncSetAttribute((const void*)k_sweep<DIR, V, RG, VW, NT, U>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_device = dev;
    }
    hipLaunchKernelGGL((k_sweep<DIR, V, RG, VW, NT, U>), dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <int DIR, typename V, int RG, int NT>
static hipError_t launch_u(int u, const ApplyArgs& a, int grid, size_t lds, hipStream_t s) {
    switch (u) {
        case 1: return launch_one<DIR, V, RG, NT, 1>(a, grid, lds, s);
        case 2: return launch_one<DIR, V, RG, NT, 2>(a, grid, lds, s);
        case 4: return launch_one<DIR, V, RG, NT, 4>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

template <int DIR, typename V, int NT>
static hipError_t launch_rg(const fm_tuning& t, const ApplyArgs& a, int grid, size_t lds, hipStream_t s) {
    switch (t.rhs_per_group) {
        case 1: return launch_u<DIR, V, 1, NT>(t.unroll, a, grid, lds, s);
        case 2: return launch_u<DIR, V, 2, NT>(t.unroll, a, grid, lds, s);
        case 4: return launch_u<DIR, V, 4, NT>(t.unroll, a, grid, lds, s);
        case 8: return launch_u<DIR, V, 8, NT>(t.unroll, a, grid, lds, s);
        case 16: return launch_u<DIR, V, 16, NT>(t.unroll, a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

template <typename V>
static hipError_t launch_sweep(bool fwd, const fm_tuning& t, const ApplyArgs& a, int grid, size_t lds,
                               hipStream_t s) {
    if (fwd) {
        switch (t.threads) {
            case 256: return launch_rg<kFwd, V, 256>(t, a, grid, lds, s);
            case 512: return launch_rg<kFwd, V, 512>(t, a, grid, lds, s);
            case 1024: return launch_rg<kFwd, V, 1024>(t, a, grid, lds, s);
        }
    } else {
        switch (t.threads) {
            case 256: return launch_rg<kRev, V, 256>(t, a, grid, lds, s);
            case 512: return launch_rg<kRev, V, 512>(t, a, grid, lds, s);
            case 1024: return launch_rg<kRev, V, 1024>(t, a, grid, lds, s);
        }
    }
    return hipErrorInvalidValue;
}

static constexpr size_t kLdsMax = 160 * 1024;
template <int DIR, typename V, int LPN, int NT, int U, int MODE>
static const void* split_fn() {
    return (const void*)k_split<DIR, V, LPN, NT, U, MODE>;
}

// The node-split kernels that are built (lanes per node, threads, unroll),
// for face-stencil states and, fewer, for cube-stencil states (the library
// defaults for every lane count and the 256-thread shapes).
#define FM_SPLIT_SHAPES(X)                                             \
    X(4, 256, 4) X(4, 512, 2) X(4, 512, 3) X(4, 512, 4)                \
    X(8, 256, 3) X(8, 256, 4) X(8, 512, 2) X(8, 512, 4)                \
    X(16, 256, 2) X(16, 256, 3) X(16, 512, 2)
#define FM_SPLIT_SHAPES_CUBE(X)                                        \
    X(4, 256, 4) X(4, 512, 3) X(8, 256, 3) X(8, 512, 4)                \
    X(16, 256, 2) X(16, 512, 2)

// kind 0: primal; 1: transpose from nodes; 2: transpose from receivers;
// mode bit 1 (2) added for the cube-stencil records
template <typename V, int L_, int N_, int U_, int CUBE>
static const void* split_kind(int kind) {
    switch (kind) {
        case 0: return split_fn<kFwd, V, L_, N_, U_, 2 * CUBE>();
        case 1: return split_fn<kRev, V, L_, N_, U_, 2 * CUBE>();
        case 2: return split_fn<kRev, V, L_, N_, U_, 2 * CUBE + 1>();
    }
    return nullptr;
}

static const void* split_kernel(int kind, bool fp64, bool cube, int lpn, int nt, int u) {
#define FM_SPLIT_PTR(L_, N_, U_) \
    if (lpn == L_ && nt == N_ && u == U_) return fp64 ? split_kind<double, L_, N_, U_, 0>(kind) : split_kind<float, L_, N_, U_, 0>(kind);
#define FM_SPLIT_PTR_CUBE(L_, N_, U_) \
    if (lpn == L_ && nt == N_ && u == U_) return fp64 ? split_kind<double, L_, N_, U_, 1>(kind) : split_kind<float, L_, N_, U_, 1>(kind);
    if (cube) {
        FM_SPLIT_SHAPES_CUBE(FM_SPLIT_PTR_CUBE)
        return nullptr;
    }
    FM_SPLIT_SHAPES(FM_SPLIT_PTR)
#undef FM_SPLIT_PTR
#undef FM_SPLIT_PTR_CUBE
    return nullptr;
}

template <int DIR, typename V, int LPN, int NT, int U, int MODE>
static hipError_t launch_split_one(const ApplyArgs& a, const SplitArgs& s, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((k_split<DIR, V, LPN, NT, U, MODE>), dim3(grid), dim3(NT), lds, st, a, s);
    return hipGetLastError();
}

template <int DIR, typename V, int MODE>
static hipError_t launch_split_dir(int lpn, int nt, int u, const ApplyArgs& a, const SplitArgs& s, int grid,
                                   size_t lds, hipStream_t st) {
#define FM_SPLIT_LAUNCH(L_, N_, U_) \
    if (lpn == L_ && nt == N_ && u == U_) return launch_split_one<DIR, V, L_, N_, U_, MODE>(a, s, grid, lds, st);
    if constexpr ((MODE & 2) != 0) {
        FM_SPLIT_SHAPES_CUBE(FM_SPLIT_LAUNCH)
    } else {
        FM_SPLIT_SHAPES(FM_SPLIT_LAUNCH)
    }
#undef FM_SPLIT_LAUNCH
    return hipErrorInvalidValue;
}

// mode bit 0: transpose input at the receivers; bit 1: cube-stencil records
template <typename V>
static hipError_t launch_split_v(bool fwd, int mode, int lpn, int nt, int u, const ApplyArgs& a, const SplitArgs& s,
                                 int grid, size_t lds, hipStream_t st) {
    switch (mode | (fwd ? 4 : 0)) {
        case 4: return launch_split_dir<kFwd, V, 0>(lpn, nt, u, a, s, grid, lds, st);
        case 6: return launch_split_dir<kFwd, V, 2>(lpn, nt, u, a, s, grid, lds, st);
        case 0: return launch_split_dir<kRev, V, 0>(lpn, nt, u, a, s, grid, lds, st);
        case 1: return launch_split_dir<kRev, V, 1>(lpn, nt, u, a, s, grid, lds, st);
        case 2: return launch_split_dir<kRev, V, 2>(lpn, nt, u, a, s, grid, lds, st);
        case 3: return launch_split_dir<kRev, V, 3>(lpn, nt, u, a, s, grid, lds, st);
    }
    return hipErrorInvalidValue;
}

static int split_lpn(const fm_batch* b) {
    const int vw = b->prec == FM_FP64 ? 2 : 4;
    return b->B / vw;
}

// Reset the counters, then one node-split sweep; a.work is the X/lambda array.
static hipError_t launch_split(const fm_batch* b, bool fwd, const ApplyArgs& a0) {
    ApplyArgs a = a0;
    a.items = b->split_items;
    a.per_xcd = b->split_per_xcd;
    SplitArgs s{};
    s.ctr = b->sync;
    s.xmask = b->sync + (size_t)b->S * kCtrStride;
    s.abort_w = b->sync + (size_t)2 * b->S * kCtrStride;
    s.fail_w = s.abort_w + kCtrStride;
    s.stage = b->stage;
    s.stage_rows = b->stage_rows;
    s.stage_B = (int32_t)(((b->B * sizeof(double) + 127) / 128) * 128 / sizeof(double));
    s.P = b->tun.split;
    s.lds_rows = b->split_lds_rows;
    s.rcv_lds = b->split_rcv_lds;
    s.stage_off = b->split_stage_off;
    s.wg_map = b->wg_map;
    s.src_P = b->wg_map ? b->wg_map + b->split_grid : nullptr;
    const size_t vbytes = b->prec == FM_FP64 ? 8 : 4;
    s.inv_l1 = ((size_t)a.xB * vbytes) % 128 != 0 || ((uintptr_t)a.work & 127u) != 0;
    hipLaunchKernelGGL(k_split_reset, dim3(1), dim3(256), 0, b->stream, s, b->S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int lpn = split_lpn(b), nt = b->tun.threads, u = b->tun.unroll;
    const int mode = (!fwd && a.in_mode == FM_W_RECEIVERS ? 1 : 0) | (b->states[0]->stencil == 26 ? 2 : 0);
    if (b->prec == FM_FP64)
        return launch_split_v<double>(fwd, mode, lpn, nt, u, a, s, b->split_grid, b->split_lds, b->stream);
    return launch_split_v<float>(fwd, mode, lpn, nt, u, a, s, b->split_grid, b->split_lds, b->stream);
}

// Choose and prepare the node split of a new batch (tun.split resolved in
// place: 1 when the rhs-group kernel runs).  Every workgroup of the launch
// must be resident at once, since the workgroups of a source wait on each
// other: the grid is checked against the occupancy of the kernel.
static int prepare_split(fm_batch* b, fm_tuning& t, const fm_tuning& asked) {
    const bool fp64 = b->prec == FM_FP64;
    const int vw = fp64 ? 2 : 4;
    const int lpn = b->B % vw == 0 ? b->B / vw : 0;
    if (t.split == 1) return FM_OK;
    // the node split defaults to 512 threads and batches of 256-384 nodes (a
    // workgroup's share of a typical level in one round trip)
    const int nt = asked.threads ? asked.threads : 512;
    const int u = asked.unroll ? asked.unroll : (lpn == 16 ? 2 : lpn == 8 ? 4 : 3);
    const bool cube = b->states[0]->stencil == 26;
    const void* kf = split_kernel(0, fp64, cube, lpn, nt, u);
    const void* kr = split_kernel(1, fp64, cube, lpn, nt, u);
    const void* kq = split_kernel(2, fp64, cube, lpn, nt, u);
    const bool built = kf && kr && kq;
    if (t.split != 0 && t.split != 2 && t.split != 4 && t.split != 8 && t.split != 16) {
        set_error("split must be 0, 1, 2, 4, 8 or 16");
        return FM_EINVAL;
    }
    // the kernel addresses one source's [N][B] arrays with 32-bit byte offsets
    const uint64_t xrow = (((uint64_t)b->B * (fp64 ? 8u : 4u) + 127u) / 128u) * 128u;   // padded node-value row
    const bool fits32 = (uint64_t)b->N * xrow < (1ull << 32) &&
                        (uint64_t)b->N * 4u * (fp64 ? 8u : 4u) < (1ull << 32);
    if (!built || !fits32) {
        if (t.split == 0) { t.split = 1; return FM_OK; }
        if (!fits32) {
            set_error("node split: one source's vectors (N=%lld x B=%d) exceed 4 GiB", (long long)b->N, b->B);
            return FM_EINVAL;
        }
        set_error("no node-split kernel for B=%d in this precision with %d threads and unroll %d (B must be %s; "
                  "see the built shapes)", b->B, nt, u, fp64 ? "8, 16 or 32" : "16, 32 or 64");
        return FM_EINVAL;
    }
    // the kernel's few bytes of static LDS come out of the same 160 KB
    // (the rhs-group kernel's 96 KB default is not applied here: with the
    // caller's request, or 16 KB, two 256-thread workgroups fit on a CU)
    const int64_t lds_cap = (int64_t)kLdsMax - 1024;
    const size_t lds = (size_t)std::min<int64_t>(std::max<int64_t>(asked.min_lds_bytes, 16 * 1024), lds_cap);
    int dev = b->device, cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int occ = 1 << 30;
    for (const void* k : {kf, kr, kq}) {
        HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap));
        int nb = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, nt, lds));
        occ = std::min(occ, nb);
    }
    const int64_t cap = (int64_t)occ * cus;
    const int64_t per8 = (b->S + 7) / 8;
    auto fits = [&](int P) { return 8 * per8 * P <= cap; };
    int P = t.split;
    std::vector<int32_t> wg_map, src_P;     // balanced split only
    if (asked.balance) {
        const int64_t slots = cap / 8;          // resident workgroups per XCD
        if (slots < 2 * per8) {
            set_error("balanced split: %lld sources per XCD need 2 workgroups each; an XCD holds %lld",
                      (long long)per8, (long long)slots);
            return FM_EINVAL;
        }
        // predicted time of a source on p workgroups (us).  balance 1..5:
        // node work / p (a workgroup streams ~0.094 * threads nodes per us)
        // plus a fixed cost per level (3, 4.5, 6, 7.5, 9 us); balance 6..10:
        // level by level, max(share / rate, t_min) plus a barrier each
        // (t_min, barrier = 3, 2 / 3, 4 / 5, 2 / 3, 6 / 4, 4 us), so that levels smaller
        // than a round trip do not get faster with more workgroups.  Both add
        // the block products (8 sum k^2 bytes at ~18 GB/s per 512 threads) / p.
        if (asked.balance < 0 || asked.balance > 10) { set_error("balance must be 0 to 10"); return FM_EINVAL; }
        const double h = 0.094 * nt;
        std::vector<double> fixed(b->S), work(b->S);
        for (int32_t i = 0; i < b->S; i++) {
            const HostState* st = b->states[i];
            fixed[i] = (1.5 + 1.5 * asked.balance) * (double)std::max(st->stats.levels_fwd, st->stats.levels_rev);
            work[i] = (double)st->N / h + 8.0 * (double)st->stats.sum_k2 / (35.0 * nt);
        }
        const bool per_level = asked.balance >= 6;
        static const double kMin[11] = {0, 0, 0, 0, 0, 0, 3.0, 3.0, 5.0, 3.0, 4.0};
        static const double kBar[11] = {0, 0, 0, 0, 0, 0, 2.0, 4.0, 2.0, 6.0, 4.0};
        const double t_min = kMin[asked.balance];
        const double t_bar = kBar[asked.balance];
        std::vector<std::vector<double>> lvl_cost;   // [source][p] for p = 0..16
        if (per_level) {
            lvl_cost.assign(b->S, std::vector<double>(17, 0.0));
            for (int32_t i = 0; i < b->S; i++) {
                const Packed& pk = b->states[i]->pk;
                for (int p = 1; p <= 16; p++) {
                    double c = 0.0;
                    for (int32_t n : pk.flvl_nsc) c += std::max((double)((n + p - 1) / p) / h, t_min) + t_bar;
                    lvl_cost[i][p] = c + 8.0 * (double)b->states[i]->stats.sum_k2 / (35.0 * nt) / p;
                }
            }
        }
        auto cost = [&](int32_t i, int p) {
            return per_level ? lvl_cost[i][std::min(std::max(p, 1), 16)] : work[i] / p + fixed[i];
        };
        // deal the sources to the XCDs in snake order of cost at the mean split
        std::vector<int32_t> order(b->S);
        for (int32_t i = 0; i < b->S; i++) order[i] = i;
        const int pm = (int)std::max<int64_t>(2, slots / per8);
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost(x, pm) > cost(y, pm); });
        std::vector<std::vector<int32_t>> on(8);
        for (int32_t r = 0; r < b->S; r++) {
            const int32_t lap = r / 8, pos = r % 8;
            on[lap % 2 == 0 ? pos : 7 - pos].push_back(order[r]);
        }
        src_P.assign(b->S, 0);
        wg_map.assign((size_t)8 * slots, -1);
        for (int x = 0; x < 8; x++) {
            std::vector<int32_t>& v = on[x];
            if (v.empty()) continue;
            const int64_t n = (int64_t)v.size();
            const int pmax = 16;
            for (int32_t i : v) src_P[i] = (int32_t)std::min<int64_t>(pmax, slots / n);
            int64_t used = 0;
            for (int32_t i : v) used += src_P[i];
            // hand out the remaining slots to the slowest sources, then move
            // workgroups from the fastest to the slowest while that helps
            for (;;) {
                int32_t worst = -1;
                for (int32_t i : v)
                    if (src_P[i] < pmax && (worst < 0 || cost(i, src_P[i]) > cost(worst, src_P[worst]))) worst = i;
                if (worst < 0 || used >= slots) break;
                src_P[worst]++;
                used++;
            }
            for (int it = 0; it < 1024; it++) {
                int32_t hi = v[0], lo = -1;
                for (int32_t i : v)
                    if (cost(i, src_P[i]) > cost(hi, src_P[hi])) hi = i;
                for (int32_t i : v)
                    if (i != hi && src_P[i] > 2 && (lo < 0 || cost(i, src_P[i] - 1) < cost(lo, src_P[lo] - 1))) lo = i;
                if (lo < 0 || src_P[hi] >= pmax) break;
                if (std::max(cost(hi, src_P[hi] + 1), cost(lo, src_P[lo] - 1)) >= cost(hi, src_P[hi])) break;
                src_P[hi]++;
                src_P[lo]--;
            }
            int64_t j = 0;
            for (int32_t i : v)
                for (int32_t q = 0; q < src_P[i]; q++, j++) wg_map[(size_t)(x + 8 * j)] = (i << 8) | q;
        }
        int64_t tot = 0;
        for (int32_t i = 0; i < b->S; i++) tot += src_P[i];
        P = (int)((tot + b->S / 2) / b->S);
        b->split_per_xcd = (int32_t)slots;
        b->split_grid = (int32_t)(8 * slots);
        b->split_items = (int32_t)tot;
    } else if (P == 0) {
        P = 1;
        for (int c : {8, 4, 2})
            if (fits(c)) { P = c; break; }
        if (P == 1) { t.split = 1; return FM_OK; }
    } else if (!fits(P)) {
        set_error("split %d needs %lld resident workgroups; the device holds %lld", P, (long long)(8 * per8 * P),
                  (long long)cap);
        return FM_EINVAL;
    }
    int64_t rows = 1;
    for (HostState* st : b->states) {
        int64_t sum = 0;
        for (int32_t i = 0; i < st->pk.nblk; i++) sum += block_stage_rows(st->pk, i);
        rows = std::max(rows, sum);
    }
    t.split = P;
    t.threads = nt;
    t.unroll = u;
    t.balance = asked.balance;
    if (!asked.balance) {
        b->split_per_xcd = (int32_t)(per8 * P);
        b->split_grid = 8 * b->split_per_xcd;
        b->split_items = b->S * P;
    }
    // receiver inputs of the transpose in LDS when they fit in 64 KB (values
    // as FP64, then the int32 positions), the block staging area after them
    size_t n_ent = 0;
    for (HostState* st : b->states) n_ent = std::max(n_ent, st->pk.rcv_node.size());
    const size_t rcv_bytes = n_ent * b->B * sizeof(double) + n_ent * sizeof(int32_t);
    b->split_rcv_lds = n_ent > 0 && rcv_bytes <= 64 * 1024;
    b->split_stage_off = b->split_rcv_lds ? (int32_t)(((rcv_bytes + 255) & ~(size_t)255) / sizeof(double)) : 0;
    const size_t lds_all = std::min<size_t>(lds + (size_t)b->split_stage_off * sizeof(double), (size_t)lds_cap);
    b->split_lds = lds_all;
    t.min_lds_bytes = (int32_t)lds;
    b->split_lds_rows = (int32_t)((lds_all - (size_t)b->split_stage_off * sizeof(double)) / ((size_t)b->B * sizeof(double)));
    for (const void* k : {kf, kr, kq}) {
        int nb = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, nt, lds_all));
        if ((int64_t)nb * cus < b->split_grid) {
            set_error("node split: the workgroups no longer fit with %zu B of LDS", lds_all);
            return FM_EINVAL;
        }
    }
    b->stage_rows = rows;
    if (b->split_lds_rows < 1) { set_error("LDS too small for one staged row"); return FM_EINVAL; }
    const size_t stage_B = ((b->B * sizeof(double) + 127) / 128) * 128 / sizeof(double);   // whole lines per row
    const size_t stage = (size_t)b->S * rows * stage_B * sizeof(double);
    const size_t sync = ((size_t)2 * b->S * kCtrStride + 64) * sizeof(unsigned);
    hipError_t e = hipMalloc(&b->stage, stage);
    if (e == hipSuccess) e = hipMalloc((void**)&b->sync, sync);
    if (e == hipSuccess) e = hipMemset(b->sync, 0, sync);
    if (e == hipSuccess && !wg_map.empty()) {
        wg_map.insert(wg_map.end(), src_P.begin(), src_P.end());
        e = hipMalloc((void**)&b->wg_map, sizeof(int32_t) * wg_map.size());
        if (e == hipSuccess)
            e = hipMemcpy(b->wg_map, wg_map.data(), sizeof(int32_t) * wg_map.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        set_error("node-split buffers (%zu B) failed: %s", stage + sync, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    return FM_OK;
}

void batch_free(fm_batch* b);

// Off-grid sources of a batch: the most seed rows and transpose targets of
// one source (launch sizes), and the union of every source's transpose
// entries grouped by target node for J^T summed over sources (entries of one
// target in ascending source order, each source's in its own order).
static int prepare_point_sources(fm_batch* b) {
    b->max_seed = b->max_tgt = 0;
    struct Ent { int32_t tgt, alpha, idx; uint8_t kind; double w; };
    std::vector<Ent> ents;
    for (int32_t a = 0; a < b->S; a++) {
        const Packed& pk = b->states[a]->pk;
        b->max_seed = std::max(b->max_seed, (int32_t)pk.seed_node.size());
        b->max_tgt = std::max(b->max_tgt, (int32_t)pk.sc_tgt.size());
        for (size_t t = 0; t < pk.sc_tgt.size(); t++)
            for (int32_t i = pk.sc_ptr[t]; i < pk.sc_ptr[t + 1]; i++)
                ents.push_back({pk.sc_tgt[t], a, pk.sc_idx[i], pk.sc_kind[i], pk.sc_w[i]});
    }
    if (ents.empty()) return FM_OK;
    // entries were appended source by source, each source's by target: a
    // stable sort by target keeps sources ascending and each one's order
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) { return x.tgt < y.tgt; });
    std::vector<int32_t> tgt, ptr(1, 0), alpha, idx;
    std::vector<uint8_t> kind;
    std::vector<double> w;
    for (size_t i = 0; i < ents.size(); i++) {
        if (i > 0 && ents[i].tgt != ents[i - 1].tgt) ptr.push_back((int32_t)i);
        if (i == 0 || ents[i].tgt != ents[i - 1].tgt) tgt.push_back(ents[i].tgt);
        alpha.push_back(ents[i].alpha);
        idx.push_back(ents[i].idx);
        kind.push_back(ents[i].kind);
        w.push_back(ents[i].w);
    }
    ptr.push_back((int32_t)ents.size());
    Arena ar;
    const size_t o_t = ar.add<int32_t>(tgt.size()), o_p = ar.add<int32_t>(ptr.size());
    const size_t o_a = ar.add<int32_t>(alpha.size()), o_i = ar.add<int32_t>(idx.size());
    const size_t o_k = ar.add<uint8_t>(kind.size()), o_w = ar.add<double>(w.size());
    const size_t total = ar.add<char>(0) + 256;
    hipError_t e = hipMalloc(&b->union_blob, total);
    if (e != hipSuccess) {
        b->union_blob = nullptr;
        set_error("batch allocation (%zu B source-seed transposes) failed: %s", total, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    char* base = (char*)b->union_blob;
    int rc = put(base, o_t, tgt);
    rc = rc ? rc : put(base, o_p, ptr);
    rc = rc ? rc : put(base, o_a, alpha);
    rc = rc ? rc : put(base, o_i, idx);
    rc = rc ? rc : put(base, o_k, kind);
    rc = rc ? rc : put(base, o_w, w);
    if (rc) return rc;
    b->uni.tgt = (const int32_t*)(base + o_t);
    b->uni.ptr = (const int32_t*)(base + o_p);
    b->uni.alpha = (const int32_t*)(base + o_a);
    b->uni.idx = (const int32_t*)(base + o_i);
    b->uni.kind = (const uint8_t*)(base + o_k);
    b->uni.w = (const double*)(base + o_w);
    b->uni.n = (int32_t)tgt.size();
    return FM_OK;
}

int batch_create(fm_state* const* states, int32_t S, int32_t B, int32_t precision, const fm_tuning* tuning,
                 void* stream, fm_batch** out) {
    if (!out) { set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    if (!states || S < 1) { set_error("need at least one state"); return FM_EINVAL; }
    if (B < 1) { set_error("B must be >= 1"); return FM_EINVAL; }
    if (precision != FM_FP64 && precision != FM_FP32) { set_error("precision must be 64 or 32"); return FM_EINVAL; }
    HostState* s0 = static_cast<HostState*>(states[0]);
    if (!s0) { set_error("null state"); return FM_EINVAL; }
    int32_t R = (int32_t)s0->pk.rcv_ptr.size() - 1;
    int64_t maxk = 0;
    for (int32_t i = 0; i < S; i++) {
        HostState* si = static_cast<HostState*>(states[i]);
        if (!si) { set_error("null state %d", i); return FM_EINVAL; }
        if (!si->same_grid(*s0)) { set_error("state %d has another grid shape or stencil", i); return FM_EINVAL; }
        if ((int32_t)si->pk.rcv_ptr.size() - 1 != R) { set_error("state %d has another receiver count", i); return FM_EINVAL; }
        maxk = std::max<int64_t>(maxk, si->pk.max_blk_rows);
    }
    fm_tuning t{};
    if (tuning) t = *tuning;
    if (t.threads == 0) t.threads = 1024;
    if (t.unroll == 0) t.unroll = 2;
    if (t.rhs_per_group == 0) {
        // up to 4 rhs per group, fewer when the blocks' staged rows would not
        // fit the LDS of the rhs-group kernel
        t.rhs_per_group = 1;
        while (t.rhs_per_group < 16 && B % (t.rhs_per_group * 2) == 0 && t.rhs_per_group * 2 <= 4 &&
               (size_t)maxk * t.rhs_per_group * 2 * sizeof(double) <= kLdsMax)
            t.rhs_per_group *= 2;
    }
    t.xcd_aware = t.xcd_aware < 0 ? 0 : 1;
    if (t.min_lds_bytes == 0) t.min_lds_bytes = 96 * 1024;
    int rg = t.rhs_per_group;
    if (rg != 1 && rg != 2 && rg != 4 && rg != 8 && rg != 16) { set_error("rhs_per_group must be 1,2,4,8 or 16"); return FM_EINVAL; }
    if (B % rg != 0) { set_error("B=%d is not a multiple of rhs_per_group=%d", B, rg); return FM_EINVAL; }
    if (t.threads != 256 && t.threads != 512 && t.threads != 1024) { set_error("threads must be 256, 512 or 1024"); return FM_EINVAL; }
    if (t.unroll < 1 || t.unroll > 6) { set_error("unroll must be 1 to 6"); return FM_EINVAL; }
    size_t need = (size_t)maxk * rg * sizeof(double);
    if (need > kLdsMax) {
        set_error("the SCC blocks need %lld staged rows (%zu B of LDS with %d rhs per group) in the rhs-group "
                  "kernel; use fewer rhs per group", (long long)maxk, need, rg);
        return FM_EINVAL;
    }
    size_t lds = std::max(need, (size_t)std::min<int64_t>(t.min_lds_bytes, (int64_t)kLdsMax));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    for (int32_t i = 0; i < S; i++) {
        int rc = upload_state(static_cast<HostState*>(states[i]));
        if (rc) return rc;
        if (precision == FM_FP32) {
            rc = upload_fp32(static_cast<HostState*>(states[i]));
            if (rc) return rc;
        }
    }
    fm_batch* b = new fm_batch();
    for (int32_t i = 0; i < S; i++) b->states.push_back(static_cast<HostState*>(states[i]));
    b->S = S;
    b->B = B;
    b->prec = precision;
    b->R = R;
    b->tun = t;
    b->stream = (hipStream_t)stream;
    b->N = s0->N;
    b->st1 = s0->stride[1];
    b->st2 = s0->stride[2];
    b->device = dev;
    b->lds_bytes = lds;
    b->items = S * (B / rg);
    b->per_xcd = (b->items + 7) / 8;
    b->grid = t.xcd_aware ? 8 * b->per_xcd : b->items;
    std::vector<SrcDev> h(S);
    for (int32_t i = 0; i < S; i++) {
        HostState* si = static_cast<HostState*>(states[i]);
        h[i] = si->dev->d;
        if (precision == FM_FP32) {
            h[i].fwts = si->dev->fwts32;
            h[i].rwts = si->dev->rwts32;
            h[i].cal_nat = si->dev->cal32;
        }
    }
    size_t vbytes = precision == FM_FP64 ? 8 : 4;
    hipError_t e = hipMalloc(&b->d_src, sizeof(SrcDev) * S + sizeof(void*) * S);
    if (e != hipSuccess) {
        delete b;
        set_error("batch allocation failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    std::vector<const void*> cal(S);
    for (int32_t i = 0; i < S; i++) cal[i] = h[i].cal_nat;
    e = hipMemcpy(b->d_src, h.data(), sizeof(SrcDev) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((char*)b->d_src + sizeof(SrcDev) * S, cal.data(), sizeof(void*) * S, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        set_error("batch upload failed: %s", hipGetErrorString(e));
        return FM_EHIP;
    }
    int rc = prepare_split(b, b->tun, tuning ? *tuning : fm_tuning{});
    if (rc == FM_OK && b->tun.split == 1 && b->tun.unroll != 1 && b->tun.unroll != 2 && b->tun.unroll != 4) {
        set_error("the rhs-group kernel takes unroll 1, 2 or 4");
        rc = FM_EINVAL;
    }
    if (rc) {
        batch_free(b);
        return rc;
    }
    // the node split reads neighbour rows of the scratch through the L1
    // without invalidating it at every level barrier, which needs every
    // node's row to be whole 128-byte lines: rows shorter than that are
    // padded (FP32 with 16 rhs, FP64 with 8)
    b->xB = B;
    if (b->tun.split > 1 && ((size_t)B * vbytes) % 128 != 0)
        b->xB = (int32_t)((((size_t)B * vbytes + 127) / 128) * 128 / vbytes);
    const size_t scratch = (size_t)S * (size_t)b->N * (size_t)b->xB * vbytes;
    e = hipMalloc(&b->scratch, scratch);
    if (e != hipSuccess) {
        b->scratch = nullptr;
        batch_free(b);
        set_error("batch allocation (%zu B scratch) failed: %s", scratch, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
    }
    rc = prepare_point_sources(b);
    if (rc) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return FM_OK;
}

void batch_free(fm_batch* b) {
    if (!b) return;
    if (b->stage) (void)hipFree(b->stage);
    if (b->wg_map) (void)hipFree(b->wg_map);
    if (b->sync) (void)hipFree(b->sync);
    if (b->nat_dev) (void)hipFree(b->nat_dev);
    if (b->cycles_dev) (void)hipFree(b->cycles_dev);
    if (b->d_src) (void)hipFree(b->d_src);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->union_blob) (void)hipFree(b->union_blob);
    delete b;
}

ApplyArgs batch_args(const fm_batch* b);

static ApplyArgs base_args(const fm_batch* b) { return batch_args(b); }

const void* const* batch_calibration(const fm_batch* b) {
    return (const void* const*)((const char*)b->d_src + sizeof(SrcDev) * b->S);
}

ApplyArgs batch_args(const fm_batch* b) {
    ApplyArgs a{};
    a.src = b->d_src;
    a.S = b->S;
    a.B = b->B;
    a.ngroups = b->B / b->tun.rhs_per_group;
    a.items = b->items;
    a.per_xcd = b->per_xcd;
    a.xcd_aware = b->tun.xcd_aware;
    a.N = b->N;
    a.xB = b->B;
    a.st1 = b->st1;
    a.st2 = b->st2;
    a.R = b->R;
    a.cube = b->states[0]->stencil == 26 ? 1 : 0;
    return a;
}

static int check_device(const fm_batch* b) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != b->device) {
        set_error("batch lives on device %d but device %d is current", b->device, dev);
        return FM_ESTATE;
    }
    return FM_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int apply_J(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode) {
    if (!b || !ds || !out) { set_error("null argument"); return FM_EINVAL; }
    if (!aligned16(ds) || !aligned16(out)) { set_error("device buffers must be 16-byte aligned"); return FM_EINVAL; }
    if (ds_mode != FM_DS_PER_PAIR && ds_mode != FM_DS_BROADCAST) { set_error("bad ds_mode %d", ds_mode); return FM_EINVAL; }
    if (out_mode != FM_OUT_NODES && out_mode != FM_OUT_RECEIVERS) { set_error("bad out_mode %d", out_mode); return FM_EINVAL; }
    if (out_mode == FM_OUT_RECEIVERS && b->R == 0) { set_error("the states have no receivers"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    ApplyArgs a = base_args(b);
    a.in = ds;
    a.in_mode = ds_mode;
    a.out_mode = out_mode;
    a.out = out;
    a.work = out_mode == FM_OUT_NODES ? out : b->scratch;
    a.xB = out_mode == FM_OUT_NODES ? b->B : b->xB;
    if (b->max_seed > 0) {
        const int64_t total = (int64_t)b->S * b->max_seed * b->B;
        const int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        if (b->prec == FM_FP64) hipLaunchKernelGGL(k_seed_rows<double>, dim3(grid), dim3(256), 0, b->stream, a, b->max_seed);
        else hipLaunchKernelGGL(k_seed_rows<float>, dim3(grid), dim3(256), 0, b->stream, a, b->max_seed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("seed-row launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    }
    hipError_t e = b->tun.split > 1       ? launch_split(b, true, a)
                   : b->prec == FM_FP64 ? launch_sweep<double>(true, b->tun, a, b->grid, b->lds_bytes, b->stream)
                                        : launch_sweep<float>(true, b->tun, a, b->grid, b->lds_bytes, b->stream);
    if (e != hipSuccess) { set_error("forward launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    if (out_mode == FM_OUT_RECEIVERS) {
        int64_t total = (int64_t)b->S * b->R * b->B;
        int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        if (b->prec == FM_FP64) hipLaunchKernelGGL(k_gather_receivers<double>, dim3(grid), dim3(256), 0, b->stream, a);
        else hipLaunchKernelGGL(k_gather_receivers<float>, dim3(grid), dim3(256), 0, b->stream, a);
        e = hipGetLastError();
        if (e != hipSuccess) { set_error("gather launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    }
    return FM_OK;
}

int apply_JT(fm_batch* b, const void* w, int32_t w_mode, void* out, int32_t out_mode) {
    if (!b || !w || !out) { set_error("null argument"); return FM_EINVAL; }
    if (!aligned16(w) || !aligned16(out)) { set_error("device buffers must be 16-byte aligned"); return FM_EINVAL; }
    if (w_mode != FM_W_NODES && w_mode != FM_W_RECEIVERS) { set_error("bad w_mode %d", w_mode); return FM_EINVAL; }
    if (out_mode != FM_JT_PER_SOURCE && out_mode != FM_JT_SUMMED) { set_error("bad out_mode %d", out_mode); return FM_EINVAL; }
    if (w_mode == FM_W_RECEIVERS && b->R == 0) { set_error("the states have no receivers"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    ApplyArgs a = base_args(b);
    a.in = w;
    a.in_mode = w_mode;
    a.out_mode = out_mode;
    a.out = out;
    a.work = b->scratch;
    a.xB = b->xB;
    hipError_t e = b->tun.split > 1       ? launch_split(b, false, a)
                   : b->prec == FM_FP64 ? launch_sweep<double>(false, b->tun, a, b->grid, b->lds_bytes, b->stream)
                                        : launch_sweep<float>(false, b->tun, a, b->grid, b->lds_bytes, b->stream);
    if (e != hipSuccess) { set_error("reverse launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    if (out_mode == FM_JT_PER_SOURCE && b->max_tgt > 0) {
        const int64_t total = (int64_t)b->S * b->max_tgt * b->B;
        const int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        if (b->prec == FM_FP64) hipLaunchKernelGGL(k_seed_scatter<double>, dim3(grid), dim3(256), 0, b->stream, a, b->max_tgt);
        else hipLaunchKernelGGL(k_seed_scatter<float>, dim3(grid), dim3(256), 0, b->stream, a, b->max_tgt);
        e = hipGetLastError();
        if (e != hipSuccess) { set_error("seed-transpose launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    }
    if (out_mode == FM_JT_SUMMED) {
        int64_t total = b->N * b->B;
        int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
        const void* const* cal = (const void* const*)((char*)b->d_src + sizeof(SrcDev) * b->S);
        const bool pad = a.xB != a.B;
        if (b->prec == FM_FP64) {
            if (pad) hipLaunchKernelGGL((k_sum_sources<double, true>), dim3(grid), dim3(256), 0, b->stream, a, cal);
            else hipLaunchKernelGGL((k_sum_sources<double, false>), dim3(grid), dim3(256), 0, b->stream, a, cal);
        } else {
            if (pad) hipLaunchKernelGGL((k_sum_sources<float, true>), dim3(grid), dim3(256), 0, b->stream, a, cal);
            else hipLaunchKernelGGL((k_sum_sources<float, false>), dim3(grid), dim3(256), 0, b->stream, a, cal);
        }
        e = hipGetLastError();
        if (e != hipSuccess) { set_error("source-sum launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
        if (b->uni.n > 0) {
            const int64_t ut = (int64_t)b->uni.n * b->B;
            const int ug = (int)std::min<int64_t>((ut + 255) / 256, 65535);
            if (b->prec == FM_FP64) hipLaunchKernelGGL(k_union_scatter<double>, dim3(ug), dim3(256), 0, b->stream, a, b->uni);
            else hipLaunchKernelGGL(k_union_scatter<float>, dim3(ug), dim3(256), 0, b->stream, a, b->uni);
            e = hipGetLastError();
            if (e != hipSuccess) { set_error("seed-transpose launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
        }
    }
    return FM_OK;
}

// ---------------------------------------------------------------------------
// directional-sweeping comparison baseline
// ---------------------------------------------------------------------------

static int upload_natural(HostState* st, int prec) {
    DeviceState* ds = st->dev;
    if (st->stencil != 6) {
        set_error("the directional-sweeping baseline takes face-stencil states only");
        return FM_EINVAL;
    }
    if (!ds->blob_nat) {
        std::vector<uint64_t> fm_, rm_;
        std::vector<double> fr, rr;
        pack_natural(st, true, fm_, fr);
        pack_natural(st, false, rm_, rr);
        Arena ar;
        size_t o1 = ar.add<uint64_t>(fm_.size()), o2 = ar.add<double>(fr.size());
        size_t o3 = ar.add<uint64_t>(rm_.size()), o4 = ar.add<double>(rr.size());
        size_t total = ar.add<char>(0) + 256;
        hipError_t e = hipMalloc(&ds->blob_nat, total);
        if (e != hipSuccess) {
            ds->blob_nat = nullptr;
            set_error("hipMalloc(%zu) for baseline records failed: %s", total, hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP;
        }
        char* b = (char*)ds->blob_nat;
        int rc = put(b, o1, fm_);
        rc = rc ? rc : put(b, o2, fr);
        rc = rc ? rc : put(b, o3, rm_);
        rc = rc ? rc : put(b, o4, rr);
        if (rc) return rc;
        ds->nat[0] = b + o1;
        ds->nat[1] = b + o2;
        ds->nat[2] = b + o3;
        ds->nat[3] = b + o4;
        if (prec == FM_FP32) {
            std::vector<float> f32(fr.begin(), fr.end()), r32(rr.begin(), rr.end());
            Arena a2;
            size_t p1 = a2.add<float>(f32.size()), p2 = a2.add<float>(r32.size());
            size_t t2 = a2.add<char>(0) + 256;
            e = hipMalloc(&ds->blob_nat32, t2);
            if (e != hipSuccess) {
                ds->blob_nat32 = nullptr;
                set_error("hipMalloc for FP32 baseline records failed: %s", hipGetErrorString(e));
                return FM_ENOMEM;
            }
            char* c = (char*)ds->blob_nat32;
            rc = put(c, p1, f32);
            rc = rc ? rc : put(c, p2, r32);
            if (rc) return rc;
            ds->nat32[0] = c + p1;
            ds->nat32[1] = c + p2;
        }
    }
    return FM_OK;
}

static int prepare_baseline(fm_batch* b) {
    if (b->max_seed > 0) {
        set_error("the directional-sweeping baseline takes sources on a node only (this batch has off-grid sources)");
        return FM_EINVAL;
    }
    if (b->nat_dev) return FM_OK;
    std::vector<NatDev> h(b->S);
    for (int32_t i = 0; i < b->S; i++) {
        int rc = upload_natural(b->states[i], b->prec);
        if (rc) return rc;
        const DeviceState* ds = b->states[i]->dev;
        h[i].fmeta = (const uint64_t*)ds->nat[0];
        h[i].frec = b->prec == FM_FP64 ? ds->nat[1] : ds->nat32[0];
        h[i].rmeta = (const uint64_t*)ds->nat[2];
        h[i].rrec = b->prec == FM_FP64 ? ds->nat[3] : ds->nat32[1];
    }
    void* nd = nullptr;
    int32_t* cyc = nullptr;
    hipError_t e = hipMalloc(&nd, sizeof(NatDev) * b->S);
    if (e == hipSuccess) e = hipMalloc(&cyc, sizeof(int32_t) * b->items);
    if (e == hipSuccess) e = hipMemcpy(nd, h.data(), sizeof(NatDev) * b->S, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (nd) (void)hipFree(nd);
        if (cyc) (void)hipFree(cyc);
        set_error("baseline setup failed: %s", hipGetErrorString(e));
        return FM_EHIP;
    }
    b->nat_dev = nd;
    b->cycles_dev = cyc;
    return FM_OK;
}

template <int DIR, typename V, int RG, int NT>
static hipError_t launch_gs(const GsArgs& g, int grid, hipStream_t s) {
    constexpr int VW = lane_width<V, RG>();
    hipLaunchKernelGGL((k_gs_sweep<DIR, V, RG, VW, NT>), dim3(grid), dim3(NT), 0, s, g);
    return hipGetLastError();
}

template <int DIR, typename V>
static hipError_t launch_gs_rg(int rg, const GsArgs& g, int grid, hipStream_t s) {
    switch (rg) {
        case 1: return launch_gs<DIR, V, 1, 1024>(g, grid, s);
        case 2: return launch_gs<DIR, V, 2, 1024>(g, grid, s);
        case 4: return launch_gs<DIR, V, 4, 1024>(g, grid, s);
        case 8: return launch_gs<DIR, V, 8, 1024>(g, grid, s);
        case 16: return launch_gs<DIR, V, 16, 1024>(g, grid, s);
    }
    return hipErrorInvalidValue;
}

static int run_gs(fm_batch* b, bool fwd, GsArgs& g, int32_t* cycles_host) {
    const HostState* s0 = b->states[0];
    g.nat = (const NatDev*)b->nat_dev;
    g.cycles = b->cycles_dev;
    g.tol = 1e-15;
    g.dim = s0->dim;
    g.m0 = (int32_t)s0->n[0];
    g.m1 = (int32_t)s0->n[1];
    g.m2 = (int32_t)s0->n[2];
    int rg = b->tun.rhs_per_group;
    hipError_t e;
    if (b->prec == FM_FP64) e = fwd ? launch_gs_rg<kFwd, double>(rg, g, b->grid, b->stream) : launch_gs_rg<kRev, double>(rg, g, b->grid, b->stream);
    else e = fwd ? launch_gs_rg<kFwd, float>(rg, g, b->grid, b->stream) : launch_gs_rg<kRev, float>(rg, g, b->grid, b->stream);
    if (e != hipSuccess) { set_error("sweep launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    if (cycles_host) {
        HIP_TRY(hipMemcpyAsync(cycles_host, b->cycles_dev, sizeof(int32_t) * b->items, hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return FM_OK;
}

int apply_J_sweep(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode, int32_t max_cycles,
                  int32_t* cycles_host) {
    if (!b || !ds || !out) { set_error("null argument"); return FM_EINVAL; }
    if (!aligned16(ds) || !aligned16(out)) { set_error("device buffers must be 16-byte aligned"); return FM_EINVAL; }
    if (ds_mode != FM_DS_PER_PAIR && ds_mode != FM_DS_BROADCAST) { set_error("bad ds_mode %d", ds_mode); return FM_EINVAL; }
    if (out_mode != FM_OUT_NODES && out_mode != FM_OUT_RECEIVERS) { set_error("bad out_mode %d", out_mode); return FM_EINVAL; }
    if (out_mode == FM_OUT_RECEIVERS && b->R == 0) { set_error("the states have no receivers"); return FM_EINVAL; }
    if (max_cycles < 1) { set_error("max_cycles must be >= 1"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    rc = prepare_baseline(b);
    if (rc) return rc;
    GsArgs g{};
    g.a = base_args(b);
    g.a.in = ds;
    g.a.in_mode = ds_mode;
    g.a.out = out;
    g.a.out_mode = out_mode;
    g.a.work = out_mode == FM_OUT_NODES ? out : b->scratch;
    g.max_cycles = max_cycles;
    rc = run_gs(b, true, g, nullptr);
    if (rc) return rc;
    if (out_mode == FM_OUT_RECEIVERS) {
        int64_t total = (int64_t)b->S * b->R * b->B;
        int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
        if (b->prec == FM_FP64) hipLaunchKernelGGL(k_gather_receivers<double>, dim3(grid), dim3(256), 0, b->stream, g.a);
        else hipLaunchKernelGGL(k_gather_receivers<float>, dim3(grid), dim3(256), 0, b->stream, g.a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("gather launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    }
    if (cycles_host) {
        HIP_TRY(hipMemcpyAsync(cycles_host, b->cycles_dev, sizeof(int32_t) * b->items, hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return FM_OK;
}

int apply_JT_sweep(fm_batch* b, const void* w, void* out, int32_t out_mode, int32_t max_cycles, int32_t* cycles_host) {
    if (!b || !w || !out) { set_error("null argument"); return FM_EINVAL; }
    if (!aligned16(w) || !aligned16(out)) { set_error("device buffers must be 16-byte aligned"); return FM_EINVAL; }
    if (out_mode != FM_JT_PER_SOURCE && out_mode != FM_JT_SUMMED) { set_error("bad out_mode %d", out_mode); return FM_EINVAL; }
    if (max_cycles < 1) { set_error("max_cycles must be >= 1"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    rc = prepare_baseline(b);
    if (rc) return rc;
    GsArgs g{};
    g.a = base_args(b);
    g.a.in = w;
    g.a.in_mode = FM_W_NODES;
    g.a.out = out;
    g.a.out_mode = out_mode;
    g.a.work = b->scratch;
    g.max_cycles = max_cycles;
    rc = run_gs(b, false, g, nullptr);
    if (rc) return rc;
    const void* const* cal = (const void* const*)((char*)b->d_src + sizeof(SrcDev) * b->S);
    hipError_t e;
    if (out_mode == FM_JT_SUMMED) {
        int64_t total = b->N * b->B;
        int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
        if (b->prec == FM_FP64) hipLaunchKernelGGL((k_sum_sources<double, false>), dim3(grid), dim3(256), 0, b->stream, g.a, cal);
        else hipLaunchKernelGGL((k_sum_sources<float, false>), dim3(grid), dim3(256), 0, b->stream, g.a, cal);
    } else {
        int64_t total = (int64_t)b->S * b->N * b->B;
        int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
        if (b->prec == FM_FP64) hipLaunchKernelGGL(k_scale_per_source<double>, dim3(grid), dim3(256), 0, b->stream, g.a, cal);
        else hipLaunchKernelGGL(k_scale_per_source<float>, dim3(grid), dim3(256), 0, b->stream, g.a, cal);
    }
    e = hipGetLastError();
    if (e != hipSuccess) { set_error("output launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    if (cycles_host) {
        HIP_TRY(hipMemcpyAsync(cycles_host, b->cycles_dev, sizeof(int32_t) * b->items, hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return FM_OK;
}

int batch_status(fm_batch* b) {
    if (!b) { set_error("null batch"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->sync) {
        unsigned* w = b->sync + (size_t)2 * b->S * kCtrStride + kCtrStride;   // sticky failure word
        unsigned v = 0;
        HIP_TRY(hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost));
        if (v) {
            HIP_TRY(hipMemset(w, 0, sizeof(unsigned)));
            set_error("a level barrier of a node-split apply timed out; the outputs since the last check are invalid");
            return FM_EHIP;
        }
    }
    return FM_OK;
}

int batch_split_info(fm_batch* b, int32_t* xcd_masks) {
    if (!b || !xcd_masks) { set_error("null argument"); return FM_EINVAL; }
    int rc = check_device(b);
    if (rc) return rc;
    if (!b->sync) { set_error("the batch does not use the node split"); return FM_EINVAL; }
    HIP_TRY(hipStreamSynchronize(b->stream));
    std::vector<unsigned> m((size_t)b->S * kCtrStride);
    HIP_TRY(hipMemcpy(m.data(), b->sync + (size_t)b->S * kCtrStride, m.size() * sizeof(unsigned),
                      hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < b->S; i++) xcd_masks[i] = (int32_t)m[(size_t)i * kCtrStride];
    return FM_OK;
}

// ---------------------------------------------------------------------------
// schedule cache: one text line per search, "key|tuning fields|ms"; the key
// names the device (architecture, compute units), the batch (S, B, precision,
// the four modes), a hash of every state's level and block structure, and the
// build of this library, so a stale or foreign entry never matches.
// ---------------------------------------------------------------------------
static uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}

template <class T>
static uint64_t fnv1a_vec(uint64_t h, const std::vector<T>& v) {
    const uint64_t n = v.size();
    h = fnv1a(h, &n, sizeof(n));
    return v.empty() ? h : fnv1a(h, v.data(), v.size() * sizeof(T));
}

static int tune_key(fm_state* const* states, int32_t S, int32_t B, int32_t precision, const int32_t modes[4],
                    std::string& key) {
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint64_t h = 1469598103934665603ull;
    for (int32_t i = 0; i < S; i++) {
        const HostState* st = static_cast<const HostState*>(states[i]);
        if (!st) { set_error("null state %d", i); return FM_EINVAL; }
        const int64_t dims[6] = {st->dim, st->n[0], st->n[1], st->n[2], st->src, st->stencil};
        h = fnv1a(h, dims, sizeof(dims));
        h = fnv1a_vec(h, st->pk.flvl_nsc);
        h = fnv1a_vec(h, st->pk.rlvl_nsc);
        h = fnv1a_vec(h, st->pk.fblk_ptr);
        h = fnv1a_vec(h, st->pk.blk_k);
        h = fnv1a_vec(h, st->pk.rcv_node);
        h = fnv1a_vec(h, st->pk.blk_it);
        h = fnv1a_vec(h, st->pk.seed_node);
        h = fnv1a_vec(h, st->pk.d_col);
    }
    char buf[512];
    snprintf(buf, sizeof(buf), "%s/%d/S%d/B%d/P%d/m%d%d%d%d/%016llx/%s %s", prop.gcnArchName, cus, S, B, precision,
             modes[0], modes[1], modes[2], modes[3], (unsigned long long)h, __DATE__, __TIME__);
    key = buf;
    for (char& c : key)
        if (c == '|' || c == '\n') c = '_';
    return FM_OK;
}

static bool tune_lookup(const char* path, const std::string& key, fm_tuning* t, float* ms) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        const char* bar = strchr(line, '|');
        if (!bar || (size_t)(bar - line) != key.size() || strncmp(line, key.c_str(), key.size()) != 0) continue;
        fm_tuning x{};
        float m = 0.0f;
        if (sscanf(bar + 1, "%d %d %d %d %d %d %d|%f", &x.rhs_per_group, &x.threads, &x.min_lds_bytes, &x.xcd_aware,
                   &x.unroll, &x.split, &x.balance, &m) == 8) {
            *t = x;      // the last matching line wins
            *ms = m;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void tune_store(const char* path, const std::string& key, const fm_tuning& t, float ms) {
    FILE* f = fopen(path, "a");
    if (!f) return;      // the cache is an optimisation: an unwritable path only costs the next search
    fprintf(f, "%s|%d %d %d %d %d %d %d|%.4f\n", key.c_str(), t.rhs_per_group, t.threads, t.min_lds_bytes,
            t.xcd_aware, t.unroll, t.split, t.balance, (double)ms);
    fclose(f);
}

// Schedule search over the built kernels on the caller's own data (the
// level-chunk autotuning of the batching step).
int autotune(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* stream, const void* ds,
             int32_t ds_mode, void* j_out, int32_t out_mode, const void* w, int32_t w_mode, void* jt_out,
             int32_t jt_mode, int32_t reps, const char* cache_path, fm_tuning* best, fm_tuning* cands, float* ms,
             int32_t max_out, int32_t* n_out) {
    if (!best) { set_error("null output pointer"); return FM_EINVAL; }
    if (reps < 1) { set_error("reps must be >= 1"); return FM_EINVAL; }
    if (!states || S < 1) { set_error("need at least one state"); return FM_EINVAL; }
    std::string key;
    if (cache_path && cache_path[0]) {
        const int32_t modes[4] = {ds_mode, out_mode, w_mode, jt_mode};
        int rc = tune_key(states, S, B, precision, modes, key);
        if (rc) return rc;
        float m = 0.0f;
        if (tune_lookup(cache_path, key, best, &m)) {
            if (cands && max_out > 0) cands[0] = *best;
            if (ms && max_out > 0) ms[0] = m;
            if (n_out) *n_out = 0;      // nothing measured: the schedule came from the cache
            clear_error();
            return FM_OK;
        }
    }
    std::vector<fm_tuning> list;
    list.push_back(fm_tuning{0, 0, 0, 0, 0, 1, 0});   // rhs groups, library defaults
    const int vw = precision == FM_FP64 ? 2 : 4;
    const int lpn = B % vw == 0 ? B / vw : 0;
    const bool cube = static_cast<const HostState*>(states[0])->stencil == 26;
#define FM_SPLIT_CAND(L_, N_, U_)                                           \
    if (lpn == L_) {                                                        \
        for (int P : {2, 4, 8, 16}) list.push_back(fm_tuning{0, N_, 0, 0, U_, P, 0}); \
        if (N_ == 256) {                                                    \
            for (int bl : {3, 5, 7, 8, 10}) list.push_back(fm_tuning{0, N_, 0, 0, U_, 0, bl}); \
            /* one workgroup per CU (the LDS request limits occupancy) */   \
            list.push_back(fm_tuning{0, N_, 96 * 1024, 0, U_, 0, 7});       \
        } else {                                                            \
            list.push_back(fm_tuning{0, N_, 0, 0, U_, 0, 7});               \
        }                                                                   \
    }
    if (cube) {
        FM_SPLIT_SHAPES_CUBE(FM_SPLIT_CAND)
    } else {
        FM_SPLIT_SHAPES(FM_SPLIT_CAND)
    }
#undef FM_SPLIT_CAND
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = -1.0f;
    int32_t n = 0;
    int rc = FM_OK;
    for (const fm_tuning& t : list) {
        fm_batch* b = nullptr;
        if (batch_create(states, S, B, precision, &t, stream, &b) != FM_OK) continue;   // does not fit
        if (t.split > 1 && !t.balance && b->tun.split != t.split) { batch_free(b); continue; }
        float m = -1.0f;
        rc = apply_J(b, ds, ds_mode, j_out, out_mode);
        if (rc == FM_OK) rc = apply_JT(b, w, w_mode, jt_out, jt_mode);
        if (rc == FM_OK && hipEventRecord(e0, st) == hipSuccess) {
            for (int r = 0; r < reps && rc == FM_OK; ++r) {
                rc = apply_J(b, ds, ds_mode, j_out, out_mode);
                if (rc == FM_OK) rc = apply_JT(b, w, w_mode, jt_out, jt_mode);
            }
            if (rc == FM_OK && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&m, e0, e1) == hipSuccess)
                m /= (float)reps;
        }
        if (rc == FM_OK) rc = batch_status(b);
        const fm_tuning used = b->tun;
        batch_free(b);
        if (rc != FM_OK) break;
        if (m >= 0.0f) {
            if (cands && n < max_out) cands[n] = used;
            if (ms && n < max_out) ms[n] = m;
            ++n;
            if (best_ms < 0.0f || m < best_ms) { best_ms = m; *best = used; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_out) *n_out = n;
    if (rc != FM_OK) return rc;
    if (best_ms < 0.0f) { set_error("no schedule could be created for these states"); return FM_EINVAL; }
    if (!key.empty()) tune_store(cache_path, key, *best, best_ms);
    clear_error();
    return FM_OK;
}

// ---------------------------------------------------------------------------
// allocation-free primal apply (fm_apply_J_static)
//
// The scratch a batch would allocate - the state table the kernels index by
// source and, for receiver output, the [S][N][B] node values - lives in one
// file-scope device array instead.  Each device holds its own copy of the
// array from module load until the process ends; host code only ever uses
// the address hipGetSymbolAddress returns for the current device (the
// array's name is a host-side stand-in, not a device address).  Every call on
// a device shares that device's array, so calls that overlap on one device
// race.  The rhs-group kernel runs (no cross-workgroup counters, so nothing
// has to start at zero); the table is written by a kernel from its launch
// arguments, so the call also needs no staging copy.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices] = {};

// The current device's address of the array, looked up once per device.
static int static_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d is beyond the %d devices the allocation-free path supports", dev, kMaxDevices);
        return FM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return FM_EHIP;
        }
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return FM_OK;
}

constexpr int kTableChunk = 12;   // SrcDev entries per table-writing launch (kernel arguments stay < 4 KB)
struct TableChunk {
    int32_t first, count;
    SrcDev e[kTableChunk];
};

static_assert(sizeof(TableChunk) < 4096, "kernel arguments must stay below 4 KB");

__global__ void k_put_table(SrcDev* dst, TableChunk c) {
    const int i = (int)threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.e[i];
}

int apply_J_static(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* stream, const void* ds,
                   int32_t ds_mode, void* out, int32_t out_mode) {
    if (!states || S < 1) { set_error("need at least one state"); return FM_EINVAL; }
    if (B < 1) { set_error("B must be >= 1"); return FM_EINVAL; }
    if (precision != FM_FP64 && precision != FM_FP32) { set_error("precision must be 64 or 32"); return FM_EINVAL; }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HostState* s0 = static_cast<HostState*>(states[0]);
    if (!s0) { set_error("null state"); return FM_EINVAL; }
    const int32_t R = (int32_t)s0->pk.rcv_ptr.size() - 1;
    int64_t maxk = 0;
    for (int32_t i = 0; i < S; i++) {
        HostState* si = static_cast<HostState*>(states[i]);
        if (!si) { set_error("null state %d", i); return FM_EINVAL; }
        if (!si->same_grid(*s0)) { set_error("state %d has another grid shape or stencil", i); return FM_EINVAL; }
        if ((int32_t)si->pk.rcv_ptr.size() - 1 != R) { set_error("state %d has another receiver count", i); return FM_EINVAL; }
        if (!si->dev || si->dev->device != dev || (precision == FM_FP32 && !si->dev->blob32)) {
            set_error("state %d is not resident on device %d in FP%d: create a batch over it once first "
                      "(that call uploads the state and allocates)", i, dev, precision);
            return FM_ESTATE;
        }
        maxk = std::max<int64_t>(maxk, si->pk.max_blk_rows);
    }
    // the library's default rhs-group schedule
    fm_tuning t{};
    t.threads = 1024;
    t.unroll = 2;
    t.rhs_per_group = 1;
    while (t.rhs_per_group < 4 && B % (t.rhs_per_group * 2) == 0 &&
           (size_t)maxk * t.rhs_per_group * 2 * sizeof(double) <= kLdsMax)
        t.rhs_per_group *= 2;
    t.xcd_aware = 1;
    t.min_lds_bytes = 96 * 1024;
    t.split = 1;
    const size_t need = (size_t)maxk * t.rhs_per_group * sizeof(double);
    if (need > kLdsMax) {
        set_error("the SCC blocks need %lld staged rows (%zu B of LDS)", (long long)maxk, need);
        return FM_EINVAL;
    }
    const size_t vbytes = precision == FM_FP64 ? 8 : 4;
    const size_t table = ((sizeof(SrcDev) * (size_t)S) + 255) & ~size_t(255);
    const size_t xbytes = out_mode == FM_OUT_RECEIVERS ? (size_t)S * (size_t)s0->N * (size_t)B * vbytes : 0;
    if (table + xbytes > kStaticScratchBytes) {
        set_error("this call needs %zu B of scratch (state table %zu B + node values %zu B); the allocation-free "
                  "path holds at most %zu B", table + xbytes, table, xbytes, kStaticScratchBytes);
        return FM_EINVAL;
    }
    void* base = nullptr;
    int rc = static_scratch(dev, &base);
    if (rc) return rc;
    // a host-side batch object whose device pointers borrow the static array
    fm_batch b;
    for (int32_t i = 0; i < S; i++) b.states.push_back(static_cast<HostState*>(states[i]));
    b.S = S;
    b.B = B;
    b.prec = precision;
    b.R = R;
    b.tun = t;
    b.stream = (hipStream_t)stream;
    b.N = s0->N;
    b.st1 = s0->stride[1];
    b.st2 = s0->stride[2];
    b.device = dev;
    b.lds_bytes = std::max(need, (size_t)t.min_lds_bytes);
    b.items = S * (B / t.rhs_per_group);
    b.per_xcd = (b.items + 7) / 8;
    b.grid = 8 * b.per_xcd;
    b.d_src = (SrcDev*)base;
    b.scratch = xbytes ? (char*)base + table : nullptr;
    b.xB = B;
    for (HostState* si : b.states) b.max_seed = std::max(b.max_seed, (int32_t)si->pk.seed_node.size());
    for (int32_t i0 = 0; i0 < S; i0 += kTableChunk) {
        TableChunk c{};
        c.first = i0;
        c.count = std::min(kTableChunk, S - i0);
        for (int k = 0; k < c.count; k++) {
            const DeviceState* d = b.states[i0 + k]->dev;
            c.e[k] = d->d;
            if (precision == FM_FP32) {
                c.e[k].fwts = d->fwts32;
                c.e[k].rwts = d->rwts32;
                c.e[k].cal_nat = d->cal32;
            }
        }
        hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, b.stream, b.d_src, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("state table launch failed: %s", hipGetErrorString(e)); return FM_EHIP; }
    }
    b.d_src = (SrcDev*)base;
    rc = apply_J(&b, ds, ds_mode, out, out_mode);
    b.d_src = nullptr;   // borrowed: nothing of b is freed
    b.scratch = nullptr;
    return rc;
}

int batch_set_stream(fm_batch* b, void* stream) {
    if (!b) { set_error("null batch"); return FM_EINVAL; }
    b->stream = (hipStream_t)stream;
    return FM_OK;
}

int batch_tuning(const fm_batch* b, fm_tuning* out) {
    if (!b || !out) { set_error("null argument"); return FM_EINVAL; }
    *out = b->tun;
    return FM_OK;
}

}  // namespace fm
