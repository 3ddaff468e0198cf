// Host setup of one frozen source state (Algorithm 1, Phase I).
//
//  1. face-upwind coefficients, row normalisation      Section 3.1, eq. (discrete-row)
//  2. calibration c = (A T) / s                          Section 3.2
//  3. dependency graph j -> i iff w_ij > 0                Section 3.3
//  4. SCCs (iterative Tarjan, linear time) and the        Section 4.1, eq. (block-form)
//     condensation DAG in topological order
//  5. longest-path levels of the condensation DAG, in both directions
//  6. dense LU with partial pivoting of every nontrivial  Section 4.3 (P_C A_C = L_C U_C),
//     SCC block, checked for a vanishing pivot             Section 4.2 (factorisation success)
//  7. packing into the per-direction level-ordered records read by the kernels
//
// Floating-point sums run in a fixed order (axis order for the face
// coefficient, neighbour-slot order for d_p and (W T)_p) and this file is built
// with -ffp-contract=off, so every upwind sign decision is a reproducible FP64
// decision.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>

#include "internal.h"

namespace fm {

static std::atomic<int32_t> g_iterative_min{kIterativeMinDefault};

void set_iterative_min(int32_t k_min) { g_iterative_min.store(k_min == 0 ? kIterativeMinDefault : k_min); }
int32_t iterative_min() { return g_iterative_min.load(); }

namespace {

struct Grid {
    int dim;
    int64_t n[3];
    int64_t stride[3];
    int64_t N;
    const double* G;
    int ncomp_g;   // metric components per node: 3 (2-D) or 6 (3-D)
    int stencil;   // 6 (faces) or 26 (cube)
};

// Full symmetric metric entry (a, b) of node p.
inline double metric(const Grid& g, int64_t p, int a, int b) {
    const double* m = g.G + (size_t)g.ncomp_g * (size_t)p;
    if (g.dim == 2) {
        if (a == b) return m[a];      // Gxx, Gzz
        return m[2];                  // Gxz
    }
    if (a == b) return m[a];          // Gxx, Gyy, Gzz
    int lo = a < b ? a : b, hi = a < b ? b : a;
    if (lo == 0 && hi == 1) return m[3];
    if (lo == 0 && hi == 2) return m[4];
    return m[5];
}

inline int64_t coord(const Grid& g, int64_t p, int axis) {
    return (p / g.stride[axis]) % g.n[axis];
}

// Nodal derivative of T along axis at node p: central inside, one-sided on the
// first and last node of the axis, zero for a single-node axis.
inline double nodal_derivative(const Grid& g, const double* T, int64_t p, int axis) {
    int64_t c = coord(g, p, axis), n = g.n[axis], st = g.stride[axis];
    if (n == 1) return 0.0;
    if (c == 0) return T[p + st] - T[p];
    if (c == n - 1) return T[p] - T[p - st];
    return 0.5 * (T[p + st] - T[p - st]);
}

inline int64_t nbr(const Grid& g, int64_t p, int slot) {
    if (g.stencil == 26) {
        int o[3];
        cube_offset(slot, o);
        return p + o[0] * g.stride[0] + o[1] * g.stride[1] + o[2] * g.stride[2];
    }
    int axis = slot >> 1;
    return (slot & 1) ? p + g.stride[axis] : p - g.stride[axis];
}

inline bool has_nbr(const Grid& g, int64_t p, int slot) {
    int axis = slot >> 1;
    if (axis >= g.dim) return false;
    int64_t c = coord(g, p, axis);
    return (slot & 1) ? (c + 1 < g.n[axis]) : (c > 0);
}

inline int opposite(const Grid& g, int slot) { return g.stencil == 26 ? 25 - slot : slot ^ 1; }

// a failure of the device packer (its message is set)
struct DevicePackError {
    int rc;
};

// Dense LU with partial pivoting (largest magnitude, ties to the lowest row),
// in place on a row-major k x k matrix.  Returns the index of the first pivot
// below tol, or -1.
int lu_factor(int k, double* a, int32_t* piv, double tol) {
    for (int c = 0; c < k; c++) {
        int p = c;
        double best = std::fabs(a[(size_t)c * k + c]);
        for (int r = c + 1; r < k; r++) {
            double v = std::fabs(a[(size_t)r * k + c]);
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (!(best >= tol)) return c;
        if (p != c) {
            double* rc = a + (size_t)c * k;
            double* rp = a + (size_t)p * k;
            for (int j = 0; j < k; j++) std::swap(rc[j], rp[j]);
        }
        const double* rc = a + (size_t)c * k;
        double inv = 1.0 / rc[c];
        for (int r = c + 1; r < k; r++) {
            double* rr = a + (size_t)r * k;
            double l = rr[c] * inv;
            rr[c] = l;
            if (l != 0.0)
                for (int j = c + 1; j < k; j++) rr[j] -= l * rc[j];
        }
    }
    return -1;
}

// X = A^{-1} = U^{-1} L^{-1} P from the factors, row-major into x.
void lu_inverse(int k, const double* lu, const int32_t* piv, double* x) {
    std::vector<int32_t> perm(k);
    for (int i = 0; i < k; i++) perm[i] = i;
    for (int c = 0; c < k; c++) std::swap(perm[c], perm[piv[c]]);
    // P I: row i of P is e_{perm[i]}
    std::fill(x, x + (size_t)k * k, 0.0);
    for (int i = 0; i < k; i++) x[(size_t)i * k + perm[i]] = 1.0;
    // L^{-1} (unit lower), row operations
    for (int i = 0; i < k; i++) {
        double* xi = x + (size_t)i * k;
        const double* li = lu + (size_t)i * k;
        for (int p = 0; p < i; p++) {
            double l = li[p];
            if (l == 0.0) continue;
            const double* xp = x + (size_t)p * k;
            for (int j = 0; j < k; j++) xi[j] -= l * xp[j];
        }
    }
    // U^{-1}
    for (int i = k - 1; i >= 0; i--) {
        double* xi = x + (size_t)i * k;
        const double* ui = lu + (size_t)i * k;
        for (int p = i + 1; p < k; p++) {
            double u = ui[p];
            if (u == 0.0) continue;
            const double* xp = x + (size_t)p * k;
            for (int j = 0; j < k; j++) xi[j] -= u * xp[j];
        }
        double d = 1.0 / ui[i];
        for (int j = 0; j < k; j++) xi[j] *= d;
    }
}

int validate(const fm_grid* g, const double* T, const double* s, int64_t src, const int64_t* rcv,
             const double* rcv_w, int32_t n_rcv, int32_t K, Grid& gr, const PointSource* ps, bool need_T) {
    if (!g || !g->G || (need_T && !T) || !s) { set_error("null argument"); return FM_EINVAL; }
    if (g->dim != 2 && g->dim != 3) { set_error("dim must be 2 or 3, got %d", g->dim); return FM_EINVAL; }
    if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1) { set_error("grid sizes must be >= 1"); return FM_EINVAL; }
    if (g->dim == 2 && g->n2 != 1) { set_error("2-D grids need n2 == 1"); return FM_EINVAL; }
    gr.dim = g->dim;
    gr.n[0] = g->n1;
    if (g->dim == 3) { gr.n[1] = g->n2; gr.n[2] = g->n3; }
    else { gr.n[1] = g->n3; gr.n[2] = 1; }
    gr.stride[0] = 1;
    gr.stride[1] = gr.n[0];
    gr.stride[2] = gr.n[0] * gr.n[1];
    gr.N = gr.n[0] * gr.n[1] * gr.n[2];
    gr.G = g->G;
    gr.ncomp_g = g->dim == 3 ? 6 : 3;
    gr.stencil = g->stencil == 0 ? 6 : g->stencil;
    if (gr.stencil != 6 && gr.stencil != 26) {
        set_error("stencil must be 0 or 6 (faces) or 26 (cube), got %d", g->stencil);
        return FM_EINVAL;
    }
    if (gr.N >= (int64_t)kNodeMask) { set_error("grid too large: %lld nodes", (long long)gr.N); return FM_EINVAL; }
    if (!ps && (src < 0 || src >= gr.N)) { set_error("source node %lld out of range", (long long)src); return FM_EINVAL; }
    if (ps) {
        if (!ps->X) { set_error("an off-grid source needs the node coordinates"); return FM_EINVAL; }
        if (!(ps->rho >= 0.0) || !std::isfinite(ps->rho)) { set_error("seed radius must be finite and >= 0"); return FM_EINVAL; }
        for (int d = 0; d < gr.dim; d++)
            if (!(ps->xi[d] >= 0.0) || !(ps->xi[d] <= (double)(gr.n[d] - 1))) {
                set_error("source coordinate %d (%g) outside the grid [0, %lld]", d, ps->xi[d], (long long)(gr.n[d] - 1));
                return FM_EINVAL;
            }
        for (int64_t i = 0; i < gr.N * gr.dim; i++)
            if (!std::isfinite(ps->X[i])) { set_error("node coordinates are not finite"); return FM_EINVAL; }
    }
    if (n_rcv < 0 || (n_rcv > 0 && !rcv)) { set_error("bad receiver list"); return FM_EINVAL; }
    if (K < 1 || K > 64) { set_error("entries per receiver must be 1 to 64, got %d", K); return FM_EINVAL; }
    for (int64_t e = 0; e < (int64_t)n_rcv * K; e++) {
        if (rcv[e] < 0 || rcv[e] >= gr.N) {
            set_error("receiver %lld entry %lld: node %lld out of range", (long long)(e / K), (long long)(e % K),
                      (long long)rcv[e]);
            return FM_EINVAL;
        }
        if (rcv_w && !std::isfinite(rcv_w[e])) {
            set_error("receiver %lld entry %lld: weight is not finite", (long long)(e / K), (long long)(e % K));
            return FM_EINVAL;
        }
    }
    for (int64_t p = 0; p < gr.N; p++) {
        if (need_T && !std::isfinite(T[p])) { set_error("T[%lld] is not finite", (long long)p); return FM_EINVAL; }
        if (!(s[p] > 0.0) || !std::isfinite(s[p])) { set_error("s[%lld] must be finite and > 0", (long long)p); return FM_EINVAL; }
        const double* m = g->G + (size_t)gr.ncomp_g * p;
        for (int c = 0; c < gr.ncomp_g; c++)
            if (!std::isfinite(m[c])) { set_error("G[%lld] is not finite", (long long)p); return FM_EINVAL; }
        for (int c = 0; c < gr.dim; c++)
            if (!(m[c] > 0.0)) { set_error("G[%lld] has a nonpositive diagonal", (long long)p); return FM_EINVAL; }
    }
    if (need_T && !ps && T[src] != 0.0) { set_error("T at the source node must be 0, got %g", T[src]); return FM_EINVAL; }
    return FM_OK;
}

// The off-grid source's cell: corners (axis 0 fastest in the corner bits)
// and multilinear weights; a coordinate on a cell face gives weight 1 there.
void source_cell(const Grid& gr, const double* xi, int64_t corner[8], double wt[8], int& nc) {
    int64_t base[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int d = 0; d < gr.dim; d++) {
        int64_t b = (int64_t)std::floor(xi[d]);
        b = std::min<int64_t>(std::max<int64_t>(b, 0), std::max<int64_t>(gr.n[d] - 2, 0));
        base[d] = b;
        t[d] = xi[d] - (double)b;
    }
    nc = 1 << gr.dim;
    for (int c = 0; c < nc; c++) {
        double w = 1.0;
        int64_t p = 0;
        for (int d = 0; d < gr.dim; d++) {
            const int up = (c >> d) & 1;
            w *= up ? t[d] : 1.0 - t[d];
            p += (base[d] + (gr.n[d] > 1 ? up : 0)) * gr.stride[d];
        }
        corner[c] = p;
        wt[c] = w;
    }
}

}  // namespace

int build_state(const fm_grid* g, const double* T, const double* s, int64_t src, const int64_t* rcv,
                const double* rcv_w, int32_t n_rcv, int32_t K, fm_state** out, const PointSource* ps,
                const Assembled* pre) {
    auto t0 = std::chrono::steady_clock::now();
    if (!out) { set_error("null output pointer"); return FM_EINVAL; }
    *out = nullptr;
    if (pre && ps) { set_error("precomputed couplings take sources on a node only"); return FM_EINVAL; }
    Grid gr;
    int rc = validate(g, T, s, src, rcv, rcv_w, n_rcv, K, gr, ps, pre == nullptr);
    if (rc != FM_OK) return rc;
    fm_state* st = new (std::nothrow) fm_state();
    if (!st) { set_error("out of host memory"); return FM_ENOMEM; }
    try {
        const int64_t N = gr.N;
        st->dim = gr.dim;
        for (int a = 0; a < 3; a++) { st->n[a] = gr.n[a]; st->stride[a] = gr.stride[a]; }
        st->N = N;
        st->src = src;
        st->stencil = gr.stencil;

        // ---- 0: an off-grid source's seed region (identity rows) ----
        // seed rows take the derivative of the straight-ray seed time
        // T_p = (s_src + s_p)/2 |X_p - x_src| as their right-hand side:
        // q_p = |X_p - x_src|/2 (sum_k phi_k ds_k + ds_p)
        std::vector<uint8_t> ident(N, 0);
        int64_t cell[8];
        double phi[8];
        int ncell = 0;
        double x_src[3] = {0, 0, 0};
        Packed& pk0 = st->pk;
        if (ps) {
            source_cell(gr, ps->xi, cell, phi, ncell);
            for (int c = 0; c < ncell; c++)
                for (int d = 0; d < gr.dim; d++) x_src[d] += phi[c] * ps->X[(size_t)gr.dim * cell[c] + d];
            int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            for (int d = 0; d < gr.dim; d++) {
                lo[d] = std::max<int64_t>(0, (int64_t)std::ceil(ps->xi[d] - ps->rho));
                hi[d] = std::min<int64_t>(gr.n[d] - 1, (int64_t)std::floor(ps->xi[d] + ps->rho));
            }
            pk0.seed_ptr.assign(1, 0);
            for (int64_t k = lo[2]; k <= hi[2]; k++)
                for (int64_t j = lo[1]; j <= hi[1]; j++)
                    for (int64_t i = lo[0]; i <= hi[0]; i++) {
                        const int64_t p = i + gr.stride[1] * j + gr.stride[2] * k;
                        ident[p] = 1;
                        double r2 = 0.0;
                        for (int d = 0; d < gr.dim; d++) {
                            const double dx = ps->X[(size_t)gr.dim * p + d] - x_src[d];
                            r2 += dx * dx;
                        }
                        const double half_r = 0.5 * std::sqrt(r2);
                        pk0.seed_node.push_back((int32_t)p);
                        for (int c = 0; c < ncell; c++) {
                            pk0.seed_col.push_back((int32_t)cell[c]);
                            pk0.seed_w.push_back(half_r * phi[c]);
                        }
                        pk0.seed_col.push_back((int32_t)p);
                        pk0.seed_w.push_back(half_r);
                        pk0.seed_ptr.push_back((int32_t)pk0.seed_col.size());
                    }
            if (pk0.seed_node.empty()) { set_error("the seed region holds no node"); delete st; return FM_EINVAL; }
            src = pk0.seed_node[0];
            st->src = src;
        } else {
            ident[src] = 1;
        }

        // ---- 1-2: couplings, weights, calibration (Sections 3.1-3.2) ----
        const bool cube = gr.stencil == 26;
        if (pre && cube) { set_error("precomputed couplings are face-stencil couplings"); delete st; return FM_EINVAL; }
        st->pmask.assign(N, 0);
        st->wrow.assign((size_t)N * (cube ? 3 : 6), 0.0);
        st->cal.assign(N, 0.0);
        const int nslot = cube ? 26 : 2 * gr.dim;
        int64_t E = 0;
        if (pre) {
            std::copy(pre->pmask, pre->pmask + N, st->pmask.begin());
            std::copy(pre->w6, pre->w6 + (size_t)N * 6, st->wrow.begin());
            std::copy(pre->cal, pre->cal + N, st->cal.begin());
            for (int64_t p = 0; p < N; p++) E += __builtin_popcount(st->pmask[p]);
        }
        // a_f of every face once (Section 3.1): G_f is the mean of the two
        // nodal metrics, the normal derivative the compact difference, each
        // tangential derivative the mean of the two nodal derivatives
        // (computed once per node); the sum runs over d' in axis order.
        // af[p][d] belongs to the face between p and p + e_d.
        std::vector<double> af, nd;
        if (!pre) {
            nd.resize((size_t)N * gr.dim);
            for (int64_t p = 0; p < N; p++)
                for (int d = 0; d < gr.dim; d++) nd[(size_t)p * gr.dim + d] = nodal_derivative(gr, T, p, d);
        }
        if (!pre && !cube) {
            af.assign((size_t)N * gr.dim, 0.0);
            for (int64_t lo = 0; lo < N; lo++)
                for (int d = 0; d < gr.dim; d++) {
                    if (!has_nbr(gr, lo, 2 * d + 1)) continue;
                    const int64_t hi = lo + gr.stride[d];
                    double a = 0.0;
                    for (int dp = 0; dp < gr.dim; dp++) {
                        double gd;
                        if (dp == d) gd = T[hi] - T[lo];
                        else gd = 0.5 * (nd[(size_t)lo * gr.dim + dp] + nd[(size_t)hi * gr.dim + dp]);
                        double Gf = 0.5 * (metric(gr, lo, d, dp) + metric(gr, hi, d, dp));
                        double term = Gf * gd;
                        a = (dp == 0) ? term : a + term;
                    }
                    af[(size_t)lo * gr.dim + d] = a;
                }
        }
        // cube stencil: a = G grad T at the node; the backward characteristic
        // p - a / max|a| leaves the 3x3x3 cube on the dominant axis's face,
        // where the value is interpolated on the Kuhn simplex holding it:
        // axes sorted by r_d = |a_d| / max|a| (descending, ties to the lower
        // axis), vertices the partial sums of the upstream steps, couplings
        // r_(t) - r_(t+1) (the last r_(dim)).  An axis whose upstream
        // neighbour is outside the grid has its component set to 0 first.
        for (int64_t p = 0; p < (pre || !cube ? 0 : N); p++) {
            double a[3] = {0.0, 0.0, 0.0}, r[3] = {0.0, 0.0, 0.0};
            int up[3] = {0, 0, 0};
            double amax = 0.0;
            for (int d = 0; d < gr.dim; d++) {
                double acc = 0.0;
                for (int dp = 0; dp < gr.dim; dp++) {
                    const double term = metric(gr, p, d, dp) * nd[(size_t)p * gr.dim + dp];
                    acc = dp == 0 ? term : acc + term;
                }
                up[d] = acc > 0.0 ? -1 : (acc < 0.0 ? 1 : 0);
                const int64_t c = coord(gr, p, d) + up[d];
                if (c < 0 || c > gr.n[d] - 1) { acc = 0.0; up[d] = 0; }
                a[d] = acc;
                amax = std::max(amax, std::fabs(acc));
            }
            uint32_t mask = 0;
            double acc = 0.0;
            if (!ident[p] && amax > 0.0) {
                int ord[3] = {0, 1, 2};
                for (int d = 0; d < gr.dim; d++) r[d] = std::fabs(a[d]) / amax;
                for (int i = 1; i < gr.dim; i++)
                    for (int j = i; j > 0 && r[ord[j - 1]] < r[ord[j]]; j--) std::swap(ord[j - 1], ord[j]);
                int o[3] = {0, 0, 0}, vs[3];
                double vc[3];
                int nv = 0;
                for (int t = 0; t < gr.dim; t++) {
                    o[ord[t]] += up[ord[t]];
                    const double c = t + 1 < gr.dim ? r[ord[t]] - r[ord[t + 1]] : r[ord[t]];
                    if (!(c > 0.0)) continue;
                    const int b = (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1);
                    vs[nv] = b - (b > 13 ? 1 : 0);
                    vc[nv++] = c;
                }
                for (int i = 1; i < nv; i++)         // ascending slot order
                    for (int j = i; j > 0 && vs[j - 1] > vs[j]; j--) {
                        std::swap(vs[j - 1], vs[j]);
                        std::swap(vc[j - 1], vc[j]);
                    }
                double dsum = 0.0;
                for (int i = 0; i < nv; i++) dsum = dsum + vc[i];
                for (int i = 0; i < nv; i++) {
                    const double w = vc[i] / dsum;
                    st->wrow[(size_t)p * 3 + i] = w;
                    mask |= 1u << vs[i];
                    acc = acc + w * T[nbr(gr, p, vs[i])];
                    E++;
                }
            }
            st->pmask[p] = mask;
            st->cal[p] = (T[p] - acc) / s[p];
        }
        for (int64_t p = 0; p < (pre || cube ? 0 : N); p++) {
            double c6[6] = {0, 0, 0, 0, 0, 0};
            for (int slot = 0; slot < nslot; slot++) {
                if (!has_nbr(gr, p, slot)) continue;
                int d = slot >> 1;
                if (slot & 1) {
                    double a = af[(size_t)p * gr.dim + d];                            // plus face of p
                    c6[slot] = -a > 0.0 ? -a : 0.0;
                } else {
                    double a = af[(size_t)(p - gr.stride[d]) * gr.dim + d];           // minus face of p
                    c6[slot] = a > 0.0 ? a : 0.0;
                }
            }
            double dsum = 0.0;
            for (int slot = 0; slot < nslot; slot++) dsum = dsum + c6[slot];
            double acc = 0.0;
            uint32_t mask = 0;
            if (!ident[p] && dsum > 0.0) {
                for (int slot = 0; slot < nslot; slot++) {
                    if (c6[slot] > 0.0) {
                        double w = c6[slot] / dsum;
                        if (w > 0.0) {
                            st->wrow[(size_t)p * 6 + slot] = w;
                            mask |= 1u << slot;
                            acc = acc + w * T[nbr(gr, p, slot)];
                            E++;
                        }
                    }
                }
            }
            st->pmask[p] = mask;
            double ell = T[p] - acc;
            st->cal[p] = ell / s[p];
        }
        if (ps)
            for (int32_t p : st->pk.seed_node) st->cal[p] = 0.0;   // their right-hand side is the seed row
        st->smask.assign(N, 0);
        for (int64_t p = 0; p < N; p++) {
            uint32_t m = st->pmask[p];
            for (int slot = 0; slot < nslot; slot++)
                if (m & (1u << slot)) st->smask[nbr(gr, p, slot)] |= 1u << opposite(gr, slot);
        }

        // ---- 3-4: SCCs by iterative Tarjan over predecessor edges ----
        // Following predecessors, a component is completed after every
        // component it depends on, so completion order is a topological order
        // of the condensation DAG (Section 4.1).
        std::vector<int32_t> idx(N, -1), low(N, 0);
        std::vector<uint8_t> onstk(N, 0);
        std::vector<int32_t> tstack;
        tstack.reserve(1024);
        std::vector<int32_t> cv;      // call stack: node
        std::vector<int8_t> cs;       // call stack: next slot
        cv.reserve(1024);
        cs.reserve(1024);
        st->comp.assign(N, -1);
        int32_t counter = 0, ncomp = 0;
        // with a trim from the GPU setup pass the search runs on the nodes
        // that neither elimination removed (every cycle lies among them);
        // every other node is its own component
        const uint8_t* trim = pre && pre->levels ? pre->trim : nullptr;
        for (int64_t root = 0; root < N; root++) {
            if (idx[root] >= 0) continue;
            if (trim && (trim[root] & 3)) {
                idx[root] = counter++;
                st->comp[root] = ncomp++;
                continue;
            }
            idx[root] = low[root] = counter++;
            tstack.push_back((int32_t)root);
            onstk[root] = 1;
            cv.push_back((int32_t)root);
            cs.push_back(0);
            while (!cv.empty()) {
                int32_t v = cv.back();
                bool descended = false;
                while (cs.back() < nslot) {
                    int slot = cs.back()++;
                    if (!(st->pmask[v] & (1u << slot))) continue;
                    int32_t u = (int32_t)nbr(gr, v, slot);
                    if (trim && (trim[u] & 3)) continue;
                    if (idx[u] < 0) {
                        idx[u] = low[u] = counter++;
                        tstack.push_back(u);
                        onstk[u] = 1;
                        cv.push_back(u);
                        cs.push_back(0);
                        descended = true;
                        break;
                    } else if (onstk[u]) {
                        low[v] = std::min(low[v], idx[u]);
                    }
                }
                if (descended) continue;
                if (low[v] == idx[v]) {
                    int32_t u;
                    do {
                        u = tstack.back();
                        tstack.pop_back();
                        onstk[u] = 0;
                        st->comp[u] = ncomp;
                    } while (u != v);
                    ncomp++;
                }
                cv.pop_back();
                cs.pop_back();
                if (!cv.empty()) {
                    int32_t p = cv.back();
                    low[p] = std::min(low[p], low[v]);
                }
            }
        }
        st->ncomp = ncomp;
        std::vector<int32_t>().swap(idx);
        std::vector<int32_t>().swap(low);
        std::vector<uint8_t>().swap(onstk);

        // members per component, ascending node id
        st->cptr.assign(ncomp + 1, 0);
        for (int64_t p = 0; p < N; p++) st->cptr[st->comp[p] + 1]++;
        for (int32_t c = 0; c < ncomp; c++) st->cptr[c + 1] += st->cptr[c];
        st->cnodes.assign(N, 0);
        {
            std::vector<int32_t> fill(st->cptr.begin(), st->cptr.end() - 1);
            for (int64_t p = 0; p < N; p++) st->cnodes[fill[st->comp[p]]++] = (int32_t)p;
        }

        // ---- 5: longest-path levels of the condensation DAG ----
        st->clev_f.assign(ncomp, 0);
        st->clev_r.assign(ncomp, 0);
        std::vector<uint8_t> unres(ncomp, 0);   // on or downstream of a cycle (Proposition 2)
        int64_t n_vio = 0;
        if (trim) {
            // levels on the device; the nodes the forward elimination
            // leaves are exactly those on or downstream of a cycle
            int rc = pre->levels(pre->ctx, N, ncomp, st->comp.data(), st->cptr.data(), st->cnodes.data(),
                                 st->pmask.data(), st->smask.data(), st->clev_f.data(), st->clev_r.data());
            if (rc != FM_OK) { delete st; return rc; }
            for (int64_t p = 0; p < N; p++)
                if (!(trim[p] & 1)) unres[st->comp[p]] = 1;
        }
        for (int32_t c = 0; c < (trim ? 0 : ncomp); c++) {
            int32_t lev = 0;
            bool nontrivial = st->cptr[c + 1] - st->cptr[c] > 1;
            uint8_t un = nontrivial ? 1 : 0;
            for (int32_t m = st->cptr[c]; m < st->cptr[c + 1]; m++) {
                int32_t v = st->cnodes[m];
                uint32_t pm = st->pmask[v];
                for (int slot = 0; slot < nslot; slot++) {
                    if (!(pm & (1u << slot))) continue;
                    int32_t u = (int32_t)nbr(gr, v, slot);
                    if (!pre && T[u] > T[v]) n_vio++;
                    int32_t cu = st->comp[u];
                    if (cu == c) continue;
                    lev = std::max(lev, st->clev_f[cu] + 1);
                    un |= unres[cu];
                }
            }
            st->clev_f[c] = lev;
            unres[c] = un;
        }
        for (int32_t c = trim ? -1 : ncomp - 1; c >= 0; c--) {
            int32_t lev = 0;
            for (int32_t m = st->cptr[c]; m < st->cptr[c + 1]; m++) {
                int32_t v = st->cnodes[m];
                uint32_t sm = st->smask[v];
                for (int slot = 0; slot < nslot; slot++) {
                    if (!(sm & (1u << slot))) continue;
                    int32_t cu = st->comp[nbr(gr, v, slot)];
                    if (cu == c) continue;
                    lev = std::max(lev, st->clev_r[cu] + 1);
                }
            }
            st->clev_r[c] = lev;
        }
        if (pre) n_vio = pre->n_vio;
        int32_t L_f = 0, L_r = 0;
        for (int32_t c = 0; c < ncomp; c++) {
            L_f = std::max(L_f, st->clev_f[c] + 1);
            L_r = std::max(L_r, st->clev_r[c] + 1);
        }
        // component ids in ascending forward level, then smallest member
        // (a topological order that does not depend on how the SCCs were
        // found): members, levels and flags follow the new ids
        {
            std::vector<int32_t> start(L_f + 1, 0), newid(ncomp, -1);
            for (int32_t c = 0; c < ncomp; c++) start[st->clev_f[c] + 1]++;
            for (int32_t l = 0; l < L_f; l++) start[l + 1] += start[l];
            for (int64_t p = 0; p < N; p++) {
                const int32_t c = st->comp[p];
                if (newid[c] < 0) newid[c] = start[st->clev_f[c]]++;
            }
            std::vector<int32_t> lf(ncomp), lr(ncomp);
            std::vector<uint8_t> un(ncomp);
            for (int32_t c = 0; c < ncomp; c++) {
                lf[newid[c]] = st->clev_f[c];
                lr[newid[c]] = st->clev_r[c];
                un[newid[c]] = unres[c];
            }
            st->clev_f.swap(lf);
            st->clev_r.swap(lr);
            unres.swap(un);
            for (int64_t p = 0; p < N; p++) st->comp[p] = newid[st->comp[p]];
            std::fill(st->cptr.begin(), st->cptr.end(), 0);
            for (int64_t p = 0; p < N; p++) st->cptr[st->comp[p] + 1]++;
            for (int32_t c = 0; c < ncomp; c++) st->cptr[c + 1] += st->cptr[c];
            std::vector<int32_t> fill(st->cptr.begin(), st->cptr.end() - 1);
            for (int64_t p = 0; p < N; p++) st->cnodes[fill[st->comp[p]]++] = (int32_t)p;
        }

        // ---- 6: factor every nontrivial block, keep A_C^{-1} ----
        // (large blocks: the Neumann series of W_CC instead, see below)
        Packed& pk = st->pk;
        std::vector<int32_t> blk_comp;
        for (int32_t c = 0; c < ncomp; c++)
            if (st->cptr[c + 1] - st->cptr[c] > 1) blk_comp.push_back(c);
        const int32_t nblk = (int32_t)blk_comp.size();
        std::vector<int32_t> comp_blk(ncomp, -1);
        pk.nblk = nblk;
        pk.blk_k.resize(nblk);
        pk.blk_inv.resize(nblk);
        pk.blk_it.assign((size_t)2 * nblk, 0);
        pk.blk_sp.assign(nblk, -1);
        pk.sp_ptr.clear();
        pk.sp_col.clear();
        pk.sp_w.clear();
        pk.spt_ptr.clear();
        pk.spt_col.clear();
        pk.spt_w.clear();
        // A block of k >= the iterative threshold whose series converges is
        // solved as x = sum_{j<=m} W_CC^j b (Theorem 1: rho(W_CC) < 1), with
        // m the least number of terms after which ||W_CC^{m+1}||_inf <= 2^-56
        // relative to x (primal), ||(W_CC^T)^{m+1}||_inf the same (transpose).
        // W_CC >= 0, so these norms are exactly the largest entries of
        // W^{m+1} 1 and (W^T)^{m+1} 1, and a norm below 1 also proves A_C
        // nonsingular.
        const int32_t it_min = iterative_min();
        for (int32_t b = 0; b < nblk; b++) {
            const int32_t c = blk_comp[b];
            const int32_t k = st->cptr[c + 1] - st->cptr[c];
            if (it_min <= 0 || k < it_min) continue;
            const int32_t* mem = st->cnodes.data() + st->cptr[c];
            // in-block couplings, rows in member order, columns ascending
            std::vector<int32_t> rp(1, 0), cl;
            std::vector<double> wv;
            for (int32_t i = 0; i < k; i++) {
                const int32_t v = mem[i];
                const uint32_t pm = st->pmask[v];
                std::vector<std::pair<int32_t, double>> row;
                for (int slot = 0; slot < nslot; slot++) {
                    if (!(pm & (1u << slot))) continue;
                    const int32_t u = (int32_t)nbr(gr, v, slot);
                    if (st->comp[u] != c) continue;
                    row.push_back({(int32_t)(std::lower_bound(mem, mem + k, u) - mem), st->weight(v, slot)});
                }
                std::sort(row.begin(), row.end());
                for (auto& e : row) { cl.push_back(e.first); wv.push_back(e.second); }
                rp.push_back((int32_t)cl.size());
            }
            // the transpose, rows = columns of W_CC, entries in ascending row order
            std::vector<int32_t> tp(k + 1, 0), tc(cl.size());
            std::vector<double> tw(cl.size());
            for (int32_t col : cl) tp[col + 1]++;
            for (int32_t j = 0; j < k; j++) tp[j + 1] += tp[j];
            {
                std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
                for (int32_t i = 0; i < k; i++)
                    for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
                        tc[fill[cl[e]]] = i;
                        tw[fill[cl[e]]++] = wv[e];
                    }
            }
            auto terms = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                             const std::vector<double>& w) {
                std::vector<double> v(k, 1.0), nv(k);
                for (int32_t j = 1; j <= kNeumannMax + 1; j++) {
                    double mx = 0.0;
                    for (int32_t i = 0; i < k; i++) {
                        double a = 0.0;
                        for (int32_t e = ptr[i]; e < ptr[i + 1]; e++) a += w[e] * v[col[e]];
                        nv[i] = a;
                        mx = std::max(mx, a);
                    }
                    v.swap(nv);
                    if (mx <= 0x1p-56) return std::max(j - 1, 1);
                }
                return 0;   // no convergence within the cap: dense
            };
            const int32_t mf = terms(rp, cl, wv);
            const int32_t mr = mf ? terms(tp, tc, tw) : 0;
            if (!mf || !mr) continue;
            pk.blk_it[2 * (size_t)b] = mf;
            pk.blk_it[2 * (size_t)b + 1] = mr;
            const int32_t base = (int32_t)pk.sp_col.size();
            pk.blk_sp[b] = (int64_t)pk.sp_ptr.size();
            for (int32_t i = 0; i <= k; i++) {
                pk.sp_ptr.push_back(base + rp[i]);
                pk.spt_ptr.push_back(base + tp[i]);
            }
            pk.sp_col.insert(pk.sp_col.end(), cl.begin(), cl.end());
            pk.sp_w.insert(pk.sp_w.end(), wv.begin(), wv.end());
            pk.spt_col.insert(pk.spt_col.end(), tc.begin(), tc.end());
            pk.spt_w.insert(pk.spt_w.end(), tw.begin(), tw.end());
        }
        int64_t inv_total = 0, n_cyc = 0, k2_all = 0;
        int32_t largest = 0;
        pk.max_blk_rows = 0;
        for (int32_t b = 0; b < nblk; b++) {
            int32_t c = blk_comp[b];
            comp_blk[c] = b;
            int32_t k = st->cptr[c + 1] - st->cptr[c];
            pk.blk_k[b] = k;
            const bool iter = pk.blk_it[2 * (size_t)b] != 0;
            pk.blk_inv[b] = iter ? -1 : inv_total;
            if (!iter) inv_total += (int64_t)k * k;
            k2_all += (int64_t)k * k;
            n_cyc += k;
            largest = std::max(largest, k);
            pk.max_blk_rows = std::max(pk.max_blk_rows, block_stage_rows(pk, b));
        }
        pk.max_blk_k = largest;
        pk.inv.assign((size_t)inv_total, 0.0);
        pk.invt.assign((size_t)inv_total, 0.0);
        double blk_residual = 0.0;
        {
            std::vector<double> a, x;
            std::vector<int32_t> piv, local(0);
            for (int32_t b = 0; b < nblk; b++) {
                if (pk.blk_it[2 * (size_t)b]) continue;   // iterative: no factors
                int32_t c = blk_comp[b];
                int32_t k = pk.blk_k[b];
                const int32_t* mem = st->cnodes.data() + st->cptr[c];
                a.assign((size_t)k * k, 0.0);
                // A_C = I - W_CC in local member order
                for (int32_t i = 0; i < k; i++) {
                    int32_t v = mem[i];
                    a[(size_t)i * k + i] = 1.0;
                    uint32_t pm = st->pmask[v];
                    for (int slot = 0; slot < nslot; slot++) {
                        if (!(pm & (1u << slot))) continue;
                        int32_t u = (int32_t)nbr(gr, v, slot);
                        if (st->comp[u] != c) continue;
                        int32_t j = (int32_t)(std::lower_bound(mem, mem + k, u) - mem);
                        a[(size_t)i * k + j] -= st->weight(v, slot);
                    }
                }
                double norm = 0.0;
                for (int32_t i = 0; i < k; i++) {
                    double rs = 0.0;
                    for (int32_t j = 0; j < k; j++) rs += std::fabs(a[(size_t)i * k + j]);
                    norm = std::max(norm, rs);
                }
                piv.assign(k, 0);
                int bad = lu_factor(k, a.data(), piv.data(), 1e-14 * norm);
                if (bad >= 0) {
                    set_error("singular SCC block: %d nodes, pivot %d below 1e-14*||A_C||_inf", k, bad);
                    delete st;
                    return FM_ESINGULAR;
                }
                x.assign((size_t)k * k, 0.0);
                lu_inverse(k, a.data(), piv.data(), x.data());
                // accuracy of the stored inverse: ||A_C X e_j - e_j||_inf on
                // four columns, with A_C = I - W_CC from the couplings
                for (int32_t j : {0, k / 3, (2 * k) / 3, k - 1}) {
                    for (int32_t i = 0; i < k; i++) {
                        const int32_t v = mem[i];
                        double r = x[(size_t)i * k + j] - (i == j ? 1.0 : 0.0);
                        const uint32_t pm = st->pmask[v];
                        for (int slot = 0; slot < nslot; slot++) {
                            if (!(pm & (1u << slot))) continue;
                            const int32_t u = (int32_t)nbr(gr, v, slot);
                            if (st->comp[u] != c) continue;
                            const int32_t m = (int32_t)(std::lower_bound(mem, mem + k, u) - mem);
                            r -= st->weight(v, slot) * x[(size_t)m * k + j];
                        }
                        blk_residual = std::max(blk_residual, std::fabs(r));
                    }
                }
                double* dst = pk.inv.data() + pk.blk_inv[b];
                for (int32_t i = 0; i < k; i++)
                    for (int32_t j = 0; j < k; j++) dst[(size_t)j * k + i] = x[(size_t)i * k + j];
                std::copy(x.begin(), x.end(), pk.invt.begin() + pk.blk_inv[b]);
            }
        }

        // ---- 7: level-ordered packing ----
        // receiver nodes (entries of nonzero weight), for records packed on the device
        std::vector<uint8_t> rcvflag;
        if (pre && pre->pack) {
            rcvflag.assign(N, 0);
            for (int64_t e = 0; e < (int64_t)n_rcv * K; e++)
                if (!rcv_w || rcv_w[e] != 0.0) rcvflag[rcv[e]] = 1;
        }
        // order of components inside a level: singletons (see below), then blocks
        auto pack_direction = [&](bool fwd, std::vector<uint64_t>& meta, std::vector<double>& wts,
                                  std::vector<int32_t>& lvl_ptr, std::vector<int32_t>& lvl_nsc,
                                  std::vector<int32_t>& blk_ptr, std::vector<int32_t>& blk_id,
                                  std::vector<int32_t>& blk_pos, std::vector<int32_t>& pos_of, int32_t L,
                                  std::vector<int32_t>& ovf_pos) {
            const std::vector<int32_t>& clev = fwd ? st->clev_f : st->clev_r;
            // an off-grid source's seed nodes take no part in the forward walk
            // (a pass before it writes their values): they get the last
            // positions, after every level
            auto skip = [&](int32_t v) { return fwd && ps && ident[v]; };
            std::vector<int64_t> cnt_sc(L + 1, 0), cnt_bl(L + 1, 0), nb(L + 1, 0);
            for (int32_t c = 0; c < ncomp; c++) {
                int32_t k = st->cptr[c + 1] - st->cptr[c];
                if (k == 1) { if (!skip(st->cnodes[st->cptr[c]])) cnt_sc[clev[c]]++; }
                else { cnt_bl[clev[c]] += k; nb[clev[c]]++; }
            }
            lvl_ptr.assign(L + 1, 0);
            lvl_nsc.assign(L, 0);
            blk_ptr.assign(L + 1, 0);
            for (int32_t l = 0; l < L; l++) {
                lvl_ptr[l + 1] = (int32_t)(lvl_ptr[l] + cnt_sc[l] + cnt_bl[l]);
                lvl_nsc[l] = (int32_t)cnt_sc[l];
                blk_ptr[l + 1] = (int32_t)(blk_ptr[l] + nb[l]);
                pk.max_level_nodes = std::max<int64_t>(pk.max_level_nodes, cnt_sc[l] + cnt_bl[l]);
            }
            std::vector<int32_t> next_sc(L), next_bl(L), next_b(L);
            for (int32_t l = 0; l < L; l++) {
                next_sc[l] = lvl_ptr[l];
                next_bl[l] = lvl_ptr[l] + lvl_nsc[l];
                next_b[l] = blk_ptr[l];
            }
            blk_id.assign(nblk, 0);
            blk_pos.assign(nblk, 0);
            pos_of.assign(N, 0);
            int32_t next_tail = lvl_ptr[L];
            // blocks: in component id order inside a level, members ascending
            for (int32_t c = 0; c < ncomp; c++) {
                const int32_t k = st->cptr[c + 1] - st->cptr[c];
                if (k == 1) continue;
                const int32_t l = clev[c];
                const int32_t b = comp_blk[c];
                blk_id[next_b[l]++] = b;
                blk_pos[b] = next_bl[l];
                for (int32_t m = 0; m < k; m++) pos_of[st->cnodes[st->cptr[c] + m]] = next_bl[l]++;
            }
            // each level's singleton run: nodes with at most three neighbours
            // in ascending node id, then those with more (their further
            // weights are a dependent load, on which a whole wave waits, so
            // they are kept together in the level's last batches); placed by
            // counting, walking the nodes in ascending id
            auto many = [&](int32_t v) { return __builtin_popcount(fwd ? st->pmask[v] : st->smask[v]) > 3; };
            std::vector<int32_t> next_many(L);
            {
                std::vector<int32_t> n_few(L, 0);
                for (int64_t p = 0; p < N; p++) {
                    const int32_t c = st->comp[p];
                    if (st->cptr[c + 1] - st->cptr[c] != 1 || skip((int32_t)p) || many((int32_t)p)) continue;
                    n_few[clev[c]]++;
                }
                for (int32_t l = 0; l < L; l++) next_many[l] = lvl_ptr[l] + n_few[l];
            }
            for (int64_t p = 0; p < N; p++) {
                const int32_t c = st->comp[p];
                if (st->cptr[c + 1] - st->cptr[c] != 1) continue;
                const int32_t v = (int32_t)p;
                const int32_t l = clev[c];
                pos_of[v] = skip(v) ? next_tail++ : many(v) ? next_many[l]++ : next_sc[l]++;
            }
            // records on the device (the GPU setup pass): same format, same bits
            if (pre && pre->pack) {
                meta.clear();
                wts.clear();
                ovf_pos.clear();
                const int rc = pre->pack(pre->ctx, fwd, N, pos_of.data(), st->comp.data(), st->pmask.data(),
                                         st->smask.data(), st->wrow.data(), st->cal.data(), rcvflag.data(), &pk.drec);
                if (rc != FM_OK) throw DevicePackError{rc};
                return;
            }
            // records: a fixed [c, w1, w2, w3] per position, further weights of
            // the rare nodes with more than three neighbours in an overflow area
            // after the N fixed records, in position order.  First the
            // external-neighbour masks in node order (a block member lists
            // only neighbours outside its component) and the overflow counts
            // per position, then the records in position order (sequential
            // writes)
            std::vector<uint32_t> extm((size_t)N);
            std::vector<int64_t> off_at((size_t)N + 1, 0);
            for (int64_t p = 0; p < N; p++) {
                const int32_t v = (int32_t)p, cv_ = st->comp[v];
                uint32_t full = fwd ? st->pmask[v] : st->smask[v], m = 0;
                while (full) {
                    const int slot = __builtin_ctz(full);
                    full &= full - 1u;
                    if (st->comp[(int32_t)nbr(gr, v, slot)] != cv_) m |= 1u << slot;
                }
                extm[v] = m;
                const int t = __builtin_popcount(m);
                off_at[(size_t)pos_of[v] + 1] = t > 3 ? t - 3 : 0;
            }
            for (int64_t q = 0; q < N; q++) off_at[q + 1] += off_at[q];
            if (cube) {
                if (off_at[N] > INT32_MAX) throw std::length_error("record overflow area too large");
                ovf_pos.assign(N, 0);
            } else {
                if (off_at[N] > (int64_t)kOffMask + 1) throw std::length_error("record overflow area too large");
                ovf_pos.clear();
            }
            std::vector<int32_t> node_at((size_t)N);
            for (int64_t p = 0; p < N; p++) node_at[pos_of[p]] = (int32_t)p;
            meta.assign(N, 0);
            wts.assign((size_t)N * 4 + (size_t)off_at[N] + 4, 0.0);
            double* ovf = wts.data() + (size_t)N * 4;
            for (int64_t q = 0; q < N; q++) {
                const int32_t v = node_at[q];
                const uint32_t mask = extm[v];
                double* rec = wts.data() + (size_t)q * 4;
                rec[0] = st->cal[v];
                const int64_t off = off_at[q] < off_at[q + 1] ? off_at[q] : 0;
                uint32_t m = mask;
                for (int t = 0; m; t++) {
                    const int slot = __builtin_ctz(m);
                    m &= m - 1u;
                    // forward: w_{v,u}; reverse: u is a successor, weight w_{u,v}
                    const double w = fwd ? st->weight(v, slot)
                                         : st->weight((int32_t)nbr(gr, v, slot), opposite(gr, slot));
                    if (t < 3) rec[1 + t] = w;
                    else ovf[(size_t)(off + (t - 3))] = w;
                }
                if (cube) {
                    ovf_pos[q] = (int32_t)off;
                    meta[q] = (uint64_t)(uint32_t)v | ((uint64_t)mask << kCubeMaskShift);
                } else {
                    meta[q] = (uint64_t)(uint32_t)v | ((uint64_t)off << kOffShift) | ((uint64_t)mask << kMaskShift);
                }
            }
        };
        std::vector<int32_t> fpos_of, rpos_of;
        pk.L_f = L_f;
        pk.L_r = L_r;
        pack_direction(true, pk.fmeta, pk.fwts, pk.flvl_ptr, pk.flvl_nsc, pk.fblk_ptr, pk.fblk_id,
                       pk.blk_fpos, fpos_of, L_f, pk.fovf);
        pack_direction(false, pk.rmeta, pk.rwts, pk.rlvl_ptr, pk.rlvl_nsc, pk.rblk_ptr, pk.rblk_id,
                       pk.blk_rpos, rpos_of, L_r, pk.rovf);
        pk.cal_nat = st->cal;

        // receivers (P_alpha, Section 4.4): the entries of each receiver in
        // receiver order for the primal gather; for P^T the same entries
        // sorted by reverse position (stable: receiver order within a node),
        // grouped per reverse level
        pk.rcv_ptr.assign((size_t)n_rcv + 1, 0);
        pk.rcv_node.clear();
        pk.rcv_wt.clear();
        std::vector<int32_t> ent_rcv;
        // an off-grid source: a receiver inside the seed region takes the
        // straight-ray time directly, d_r = (s_src + s_r)/2 |x_r - x_src|
        // (s_r, x_r interpolated by its own weights): no P entries, and the
        // row |x_r - x_src|/2 (sum_k phi_k ds_k + sum_e w_e ds_e) of D_alpha
        if (ps) pk.d_ptr.assign((size_t)n_rcv + 1, 0);
        for (int32_t r = 0; r < n_rcv; r++) {
            if (ps) {
                double xr_log[3] = {0, 0, 0}, xr[3] = {0, 0, 0};
                for (int32_t k = 0; k < K; k++) {
                    const int64_t e = (int64_t)r * K + k;
                    const double w = rcv_w ? rcv_w[e] : 1.0;
                    for (int d = 0; d < gr.dim; d++) {
                        xr_log[d] += w * (double)coord(gr, rcv[e], d);
                        xr[d] += w * ps->X[(size_t)gr.dim * rcv[e] + d];
                    }
                }
                bool direct = true;
                for (int d = 0; d < gr.dim; d++)
                    if (!(std::fabs(xr_log[d] - ps->xi[d]) <= ps->rho)) direct = false;
                if (direct) {
                    double r2 = 0.0;
                    for (int d = 0; d < gr.dim; d++) r2 += (xr[d] - x_src[d]) * (xr[d] - x_src[d]);
                    const double half_r = 0.5 * std::sqrt(r2);
                    for (int c = 0; c < ncell; c++) {
                        pk.d_col.push_back((int32_t)cell[c]);
                        pk.d_w.push_back(half_r * phi[c]);
                    }
                    for (int32_t k = 0; k < K; k++) {
                        const int64_t e = (int64_t)r * K + k;
                        const double w = rcv_w ? rcv_w[e] : 1.0;
                        if (w == 0.0) continue;
                        pk.d_col.push_back((int32_t)rcv[e]);
                        pk.d_w.push_back(half_r * w);
                    }
                    pk.d_ptr[r + 1] = (int32_t)pk.d_col.size();
                    pk.rcv_ptr[r + 1] = (int32_t)pk.rcv_node.size();
                    continue;
                }
                pk.d_ptr[r + 1] = (int32_t)pk.d_col.size();
            }
            for (int32_t k = 0; k < K; k++) {
                const int64_t e = (int64_t)r * K + k;
                const double w = rcv_w ? rcv_w[e] : 1.0;
                if (w == 0.0) continue;
                pk.rcv_node.push_back((int32_t)rcv[e]);
                pk.rcv_wt.push_back(w);
                ent_rcv.push_back(r);
            }
            pk.rcv_ptr[r + 1] = (int32_t)pk.rcv_node.size();
        }
        const int32_t n_ent = (int32_t)pk.rcv_node.size();
        std::vector<std::pair<int32_t, int32_t>> ent(n_ent);
        for (int32_t e = 0; e < n_ent; e++) {
            ent[e] = {rpos_of[pk.rcv_node[e]], e};
            if (!pk.rmeta.empty()) pk.rmeta[rpos_of[pk.rcv_node[e]]] |= kRcvFlag;
        }
        std::sort(ent.begin(), ent.end());
        pk.rcv_pos.resize(n_ent);
        pk.rcv_idx.resize(n_ent);
        pk.rcv_ew.resize(n_ent);
        for (int32_t e = 0; e < n_ent; e++) {
            pk.rcv_pos[e] = ent[e].first;
            pk.rcv_idx[e] = ent_rcv[ent[e].second];
            pk.rcv_ew[e] = pk.rcv_wt[ent[e].second];
        }
        pk.rcvlvl_ptr.assign(L_r + 1, 0);
        {
            int32_t e = 0;
            for (int32_t l = 0; l < L_r; l++) {
                while (e < n_ent && pk.rcv_pos[e] < pk.rlvl_ptr[l + 1]) e++;
                pk.rcvlvl_ptr[l + 1] = e;
            }
        }

        // the transposes of the seed rows and of D, grouped by target node
        // (ascending; in a target, seed entries in seed order, then direct
        // entries in receiver order): J^T adds them after the reverse walk
        if (ps) {
            struct Ent { int32_t tgt, order; uint8_t kind; int32_t idx; double w; };
            std::vector<Ent> ents;
            int32_t ord = 0;
            for (size_t e = 0; e + 1 < pk.seed_ptr.size(); e++)
                for (int32_t i = pk.seed_ptr[e]; i < pk.seed_ptr[e + 1]; i++)
                    ents.push_back({pk.seed_col[i], ord++, 0, pk.seed_node[e], pk.seed_w[i]});
            for (int32_t r = 0; r < n_rcv; r++)
                for (int32_t i = pk.d_ptr[r]; i < pk.d_ptr[r + 1]; i++)
                    ents.push_back({pk.d_col[i], ord++, 1, r, pk.d_w[i]});
            std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
                return a.tgt != b.tgt ? a.tgt < b.tgt : a.order < b.order;
            });
            pk.sc_ptr.assign(1, 0);
            for (size_t i = 0; i < ents.size(); i++) {
                if (i == 0 || ents[i].tgt != ents[i - 1].tgt) {
                    if (i > 0) pk.sc_ptr.push_back((int32_t)i);
                    pk.sc_tgt.push_back(ents[i].tgt);
                }
                pk.sc_kind.push_back(ents[i].kind);
                pk.sc_idx.push_back(ents[i].idx);
                pk.sc_w.push_back(ents[i].w);
            }
            if (!ents.empty()) pk.sc_ptr.push_back((int32_t)ents.size());
        }

        // ---- statistics ----
        int64_t n_unr = 0;
        for (int64_t p = 0; p < N; p++) n_unr += unres[st->comp[p]];
        fm_stats& S = st->stats;
        S.N = N;
        S.E = E;
        S.levels_fwd = L_f;
        S.levels_rev = L_r;
        S.n_scc = nblk;
        S.largest_scc = largest;
        S.n_cyc = n_cyc;
        S.sum_k2 = k2_all;
        S.dense_k2 = inv_total;
        S.n_iter_blocks = 0;
        S.max_iter = 0;
        S.iter_nnz = (int64_t)pk.sp_col.size();
        S.block_residual = blk_residual;
        for (int32_t b = 0; b < nblk; b++)
            if (pk.blk_it[2 * (size_t)b]) {
                S.n_iter_blocks++;
                S.max_iter = std::max({S.max_iter, pk.blk_it[2 * (size_t)b], pk.blk_it[2 * (size_t)b + 1]});
            }
        S.n_vio = n_vio;
        S.n_unr = n_unr;
        S.f_vio = E ? (double)n_vio / (double)E : 0.0;
        S.f_cyc = (double)n_cyc / (double)N;
        S.f_unr = (double)n_unr / (double)N;
        const int64_t n_meta = pk.drec.meta[0] ? 2 * N : (int64_t)(pk.fmeta.size() + pk.rmeta.size());
        const int64_t n_wts = pk.drec.meta[0] ? pk.drec.nwts[0] + pk.drec.nwts[1]
                                              : (int64_t)(pk.fwts.size() + pk.rwts.size());
        S.state_bytes = n_meta * 8 + (n_wts + (int64_t)(2 * pk.inv.size() + pk.cal_nat.size())) * 8 +
                        (int64_t)(pk.sp_col.size() + pk.spt_col.size()) * 12 +
                        (int64_t)(pk.sp_ptr.size() + pk.spt_ptr.size()) * 4;
        S.n_seed = (int32_t)pk.seed_node.size();
        S.n_direct = 0;
        for (size_t r = 0; r + 1 < pk.d_ptr.size(); r++) S.n_direct += pk.d_ptr[r + 1] > pk.d_ptr[r];
        S.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } catch (const DevicePackError& e) {
        free_device_state(st);
        delete st;
        return e.rc;   // the packer set the message
    } catch (const std::bad_alloc&) {
        free_device_state(st);
        delete st;
        set_error("out of host memory during setup");
        return FM_ENOMEM;
    } catch (const std::length_error& e) {
        free_device_state(st);
        delete st;
        set_error("state too large for the packed format: %s", e.what());
        return FM_EINVAL;
    }
    *out = st;
    return FM_OK;
}

void pack_natural(const HostState* st, bool fwd, std::vector<uint64_t>& meta, std::vector<double>& rec) {
    const int64_t N = st->N;
    const int nslot = 2 * st->dim;
    meta.assign(N, 0);
    rec.assign((size_t)N * 4, 0.0);
    std::vector<double> ovf;
    for (int64_t v = 0; v < N; v++) {
        uint32_t mask = fwd ? st->pmask[v] : st->smask[v];
        double* r = rec.data() + (size_t)v * 4;
        r[0] = st->cal[v];
        int t = 0;
        int64_t off = 0;
        for (int slot = 0; slot < nslot; slot++) {
            if (!(mask & (1u << slot))) continue;
            int axis = slot >> 1;
            int64_t u = (slot & 1) ? v + st->stride[axis] : v - st->stride[axis];
            double w = fwd ? st->weight(v, slot) : st->weight(u, slot ^ 1);
            if (t < 3) {
                r[1 + t] = w;
            } else {
                if (t == 3) off = (int64_t)ovf.size();
                ovf.push_back(w);
            }
            t++;
        }
        meta[v] = (uint64_t)v | ((uint64_t)off << kOffShift) | ((uint64_t)mask << kMaskShift);
    }
    rec.insert(rec.end(), ovf.begin(), ovf.end());
    rec.resize(rec.size() + 4, 0.0);
}

}  // namespace fm
