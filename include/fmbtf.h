/*
 * fmbtf: frozen full-metric Eikonal tangent transport through its SCC
 * condensation graph (block-triangular form), applied on an MI355X (gfx950).
 *
 * The operation (paper: "Efficient Matrix-Free Gauss-Newton Traveltime
 * Tomography on Full-Metric Deformed Grids"):
 *
 *   A = I - W                    face-upwind frozen transport, Section 3.1,
 *                                eq. (discrete-row) and eq. (transport-system)
 *                                (or the 26-neighbour cube stencil, fm_grid)
 *   C = diag(c), c_i = l_i / s_i with l = A T    Section 3.2
 *   J_alpha   = P_alpha A^{-1} C                 eq. (source-jacobian), M = I, D = 0
 *   J_alpha^T = C A^{-T} P_alpha^T               eq. (source-transpose)
 *   J^T y     = sum_alpha J_alpha^T y_alpha       Section 4.4 (multi-source stacking)
 *
 * A^{-1} and A^{-T} are applied exactly (up to rounding) by traversing the
 * condensation DAG of the dependency graph (edge j -> i iff w_ij > 0,
 * Section 3.3) in topological order: scalar substitution on singleton
 * components and a local block solve on every nontrivial strongly connected
 * component (Section 4.1, Proposition 3; Section 4.3).  The state built once
 * per frozen source (Section 4.3, the setup S_alpha) is reused for every
 * right-hand side in both directions (Algorithm 1, Phases I and III).
 *
 * Conventions shared by every call
 *   node id      n = i + n1*(j + n2*k), i fastest; 2-D grids use (i, k), n2 = 1
 *   metric G     [N][6] = (Gxx,Gyy,Gzz,Gxy,Gxz,Gyz) in 3-D, [N][3] = (Gxx,Gzz,Gxz)
 *                in 2-D, in logical index units (Section 2.2, eq. (metric-eikonal))
 *   batches      vectors are [N][B] with the right-hand-side index fastest;
 *                per-source vectors are [S][N][B]; receiver data [S][R][B]
 *   ownership    every pointer argument is owned by the caller.  Host inputs of
 *                the build calls are copied and may be freed on return.  Device
 *                pointers of the apply calls must stay valid until the work
 *                enqueued on the batch stream has finished.
 *   errors       every int-returning call returns FM_OK (0) or a negative code;
 *                fm_last_error() then describes the failure (thread-local).
 *   threads      states and batches may be used from one thread at a time.
 */
#ifndef FMBTF_H
#define FMBTF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FM_OK 0
#define FM_EINVAL (-1)     /* bad shape, index, non-finite input, s <= 0, T_src != 0, mode */
#define FM_ESINGULAR (-2)  /* an SCC block has a pivot below 1e-14 * ||A_C||_inf (Section 4.2) */
#define FM_ENOMEM (-3)     /* host or device allocation failed */
#define FM_EHIP (-4)       /* a HIP runtime call failed */
#define FM_ESTATE (-5)     /* object used in a state that does not allow the call */

/* precision of a batch (Section 4.3 factors are always formed in FP64) */
#define FM_FP64 64
#define FM_FP32 32

/* input / output layouts of the apply calls */
#define FM_DS_PER_PAIR 0    /* ds [S][N][B]: one slowness perturbation per (source, rhs) */
#define FM_DS_BROADCAST 1   /* ds [N][B]: one model-space vector shared by all sources */
#define FM_OUT_NODES 0      /* J: dT at every node, [S][N][B] */
#define FM_OUT_RECEIVERS 1  /* J: dT sampled at the receivers, [S][R][B] */
#define FM_W_NODES 0        /* J^T input: nodal weights [S][N][B] */
#define FM_W_RECEIVERS 1    /* J^T input: receiver data [S][R][B], scattered by P^T */
#define FM_JT_PER_SOURCE 0  /* J^T output: c_alpha * lambda_alpha per source, [S][N][B] */
#define FM_JT_SUMMED 1      /* J^T output: sum over sources in source order, [N][B] */

typedef struct fm_grid {
    int32_t dim;            /* 2 or 3 */
    int64_t n1, n2, n3;     /* nodes per logical axis; n2 = 1 in 2-D */
    const double* G;        /* host pointer, metric as described above */
    int32_t stencil;        /* dependency stencil of the build calls:
                               0 or 6: the face-based upwinding of Section 3.1
                               (at most six neighbour dependencies per row);
                               26: the cube stencil, a variant the paper does
                               not define: a row interpolates the transport
                               value where the node's backward characteristic
                               (direction -a, a = G grad_xi T at the node)
                               leaves its 3x3x3 cube of nodes, linearly on the
                               Kuhn simplex that holds that point (at most dim
                               dependencies among the 26 neighbours), then is
                               normalised and calibrated as in Sections
                               3.1-3.2; an axis whose upstream neighbour lies
                               outside the grid has its component of a set to
                               0 first.  Any other value: FM_EINVAL.  The GPU
                               setup pass and the sweeping baseline take the
                               face stencil only. */
} fm_grid;

typedef struct fm_state fm_state;   /* one frozen source: W, c, graph, levels, SCC factors */
typedef struct fm_batch fm_batch;   /* S states + preallocated device scratch for B rhs */

typedef struct fm_stats {
    int64_t N;              /* transport unknowns */
    int64_t E;              /* dependency edges (w_ij > 0) */
    int32_t levels_fwd;     /* levels of the condensation DAG (primal traversal) */
    int32_t levels_rev;     /* levels of the reverse traversal (transpose) */
    int32_t n_scc;          /* nontrivial SCCs (size > 1) */
    int32_t largest_scc;
    int64_t n_cyc;          /* nodes in nontrivial SCCs */
    int64_t sum_k2;         /* sum of squared SCC sizes (dense block storage) */
    int64_t n_vio;          /* edges j -> i with T_j > T_i (Section 3.4) */
    int64_t n_unr;          /* nodes left by scalar Kahn elimination (Section 3.5) */
    double f_vio, f_cyc, f_unr;   /* eq. (graph-fractions) */
    double setup_seconds;   /* host time of the build */
    int64_t state_bytes;    /* bytes of the packed per-source state (one precision) */
    int32_t n_seed;         /* seed-region nodes of an off-grid source (0 for a source on a node) */
    int32_t n_direct;       /* receivers an off-grid source reaches through its direct term D */
    int32_t n_iter_blocks;  /* nontrivial SCCs solved iteratively (fm_set_iterative_block_min) */
    int32_t max_iter;       /* most series terms of such a block (either direction) */
    int64_t dense_k2;       /* sum of k^2 over the blocks kept as dense inverses */
    int64_t iter_nnz;       /* in-block couplings stored for the iterative blocks */
    double block_residual;  /* max over the dense blocks of ||A_C X e_j - e_j||_inf on four columns
                               j of the stored inverse X (0 without dense blocks) */
} fm_stats;

/* Launch schedule of a batch; zero fields take the library default. */
typedef struct fm_tuning {
    int32_t rhs_per_group;  /* right-hand sides handled by one workgroup: 1,2,4,8,16 */
    int32_t threads;        /* workgroup size: 256, 512 or 1024 (rhs groups); 256 or 512 (split) */
    int32_t min_lds_bytes;  /* LDS reserved per workgroup (limits workgroups per CU); the split
                               reserves this (default 16 KB) plus the receiver inputs of J^T */
    int32_t xcd_aware;      /* 1 or 0 (default): keep the groups of one source on one XCD; -1: off */
    int32_t unroll;         /* nodes per thread in flight inside a level: 1, 2 or 4 (rhs groups);
                               split, 4 lanes per node (FP64 B=8, FP32 B=16): 2, 3, 4 with
                               512 threads, 4 with 256; 8 lanes per node (FP64 B=16, FP32 B=32):
                               2, 4 with 512 threads, 3, 4 with 256; 16 lanes per node (FP64
                               B=32, FP32 B=64): 2 with 512 threads, 2, 3 with 256 */
    int32_t split;          /* workgroups sharing one source and all B rhs (node split):
                               0 = choose (the rhs-group kernel when no split fits),
                               1 = off (rhs groups), 2, 4, 8, 16 = that many */
    int32_t balance;        /* 1..10: node split with a different number of workgroups per
                               source (2..16), chosen from a cost model of each source (its
                               levels and block work) so that the sources finish together, every
                               resident workgroup slot used (split is then ignored and reports
                               the mean).  1..5: node work / P plus 3, 4.5, 6, 7.5 or 9 us per
                               level; 6..10: level by level, max(share / rate, t_min) plus a
                               barrier, (t_min, barrier) = (3, 2), (3, 4), (5, 2), (3, 6),
                               (4, 4) us.  0: off */
} fm_tuning;

/*
 * Build the frozen state of one source (Algorithm 1, Phase I):
 * face-upwind coefficients and row normalisation (Section 3.1), calibration
 * c = (A T) / s (Section 3.2), dependency graph (Section 3.3), SCCs and a
 * topological level schedule of the condensation DAG (Section 4.1), and a
 * partially pivoted LU of every nontrivial SCC block (Section 4.3).
 *   g         grid and host metric
 *   T, s      host [N] background traveltime (T[src_node] must be 0) and slowness (> 0)
 *   src_node  on-grid source node; its row is an identity row with c = 0
 *   rcv_nodes host [n_rcv] receiver nodes (P_alpha is the selection; duplicates allowed)
 *   out       receives the new state (host-side only until a batch uses it)
 * Errors: FM_EINVAL, FM_ESINGULAR, FM_ENOMEM.
 */
int fm_build_frozen_state(const fm_grid* g, const double* T, const double* s, int64_t src_node,
                          const int64_t* rcv_nodes, int32_t n_rcv, fm_state** out);

/*
 * Build S states at once on up to nthreads host threads (sources are
 * independent, Section 4.4).  T is [S][N], rcv_nodes is [S][n_rcv]; out[S]
 * receives the states.  On error no state is returned (all are freed).
 */
int fm_build_frozen_states(const fm_grid* g, int32_t S, const double* T, const double* s,
                           const int64_t* src_nodes, const int64_t* rcv_nodes, int32_t n_rcv,
                           int32_t nthreads, fm_state** out);

/*
 * The same with interpolating receivers (P_alpha of Section 4.4 samples the
 * transported perturbation at receiver locations between nodes): receiver r
 * of a state samples sum_k w[r][k] x[node[r][k]] over k_per_rcv entries, and
 * P_alpha^T adds w[r][k] y_r at node[r][k].
 *   rcv_nodes    host [n_rcv][k_per_rcv] (per state; [S][n_rcv][k_per_rcv] for the batch builder)
 *   rcv_weights  host, same shape, finite (NULL: every weight 1); entries of
 *                weight 0 are dropped
 *   k_per_rcv    1..64 (1 with NULL weights is the plain selection above)
 * Every state of a batch needs the same n_rcv.  The transpose from receiver
 * data stages the weighted inputs in LDS when a source's entries fit in 64 KB
 * (entries x (8 B + 8 B x B)); otherwise it reads them from global memory.
 * Errors: as fm_build_frozen_state; FM_EINVAL for k_per_rcv out of range or
 * a weight that is not finite.
 */
int fm_build_frozen_state_w(const fm_grid* g, const double* T, const double* s, int64_t src_node,
                            const int64_t* rcv_nodes, const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv,
                            fm_state** out);
int fm_build_frozen_states_w(const fm_grid* g, int32_t S, const double* T, const double* s,
                             const int64_t* src_nodes, const int64_t* rcv_nodes, const double* rcv_weights,
                             int32_t n_rcv, int32_t k_per_rcv, int32_t nthreads, fm_state** out);

/*
 * An off-grid point source (Section 3.1's source-seed rows, Section 3.2's
 * right-hand side from the differentiated source treatment, and the direct
 * term D_alpha of eq. (source-jacobian) / eq. (source-transpose)).  The
 * library's reading, since the paper gives no formula for them:
 *   - the source sits at logical coordinates xi_src (dim values, axis 0
 *     first, each in [0, n_d - 1]); the 2^dim corners k of its cell carry
 *     multilinear weights phi_k, so s_src = sum phi_k s_k and
 *     x_src = sum phi_k X_k;
 *   - the seed region is every node p with max_d |i_d(p) - xi_d| <= seed_radius;
 *     T there must be the straight-ray time (s_src + s_p)/2 |X_p - x_src|
 *     (the caller's first-arrival solver seeds it so); its rows of A are
 *     identity rows with right-hand side
 *     |X_p - x_src|/2 (sum_k phi_k ds_k + ds_p);
 *   - a receiver whose position (its weights applied to its nodes' logical
 *     coordinates) lies in the seed region is direct: it has no row in P,
 *     and its row of D is |x_r - x_src|/2 (sum_k phi_k ds_k + sum_e w_e ds_e)
 *     with x_r interpolated by the receiver's weights;
 *   - J = P A^{-1} C + D, J^T = C^T A^{-T} P^T + D^T; J to nodes is A^{-1} C
 *     (seed rows included), J^T from nodal weights C^T A^{-T} (no D).
 *   X            host [N][dim] physical node coordinates (finite)
 *   xi_src       host [dim] (per state; [S][dim] for the batch builder)
 *   seed_radius  >= 0, logical units; the region must hold at least one node
 * Other arguments as fm_build_frozen_state_w (rcv_weights may be NULL).  Every
 * apply (J, J^T, both modes, both precisions, the allocation-free primal) takes
 * such states, mixed with on-grid ones in one batch; the directional-sweeping
 * baseline refuses them (FM_EINVAL).
 * Errors: as fm_build_frozen_state_w; FM_EINVAL for X NULL or not finite,
 * xi_src outside the grid, seed_radius negative or not finite, or an empty
 * seed region.
 */
int fm_build_frozen_state_pt(const fm_grid* g, const double* X, const double* T, const double* s,
                             const double* xi_src, double seed_radius, const int64_t* rcv_nodes,
                             const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv, fm_state** out);
int fm_build_frozen_states_pt(const fm_grid* g, const double* X, int32_t S, const double* T, const double* s,
                              const double* xi_src, double seed_radius, const int64_t* rcv_nodes,
                              const double* rcv_weights, int32_t n_rcv, int32_t k_per_rcv, int32_t nthreads,
                              fm_state** out);

/*
 * Solver of large SCC blocks (Section 6 leaves sparse or iterative block
 * solvers for large components open; Section 4.3's dense local solve is the
 * default).  Blocks of k >= k_min nodes that the builders create from now on
 * are solved by the Neumann series of W_CC instead of a stored inverse:
 * x_C = sum_{j<=m} W_CC^j b_C (transpose: W_CC^T), m chosen at build time as
 * the least number of terms after which ||W_CC^{m+1}||_inf (||W_CC^{m+1}||_1
 * for the transpose) is at most 2^-56, so the truncation is below FP64
 * rounding; that norm being below 1 also proves A_C nonsingular (Theorem 1
 * gives rho(W_CC) < 1).  A block whose series needs more than 200 terms keeps
 * the dense inverse.  Such a block stores only its couplings (no k x k
 * inverse, no O(k^3) factorisation); applying it costs m sparse products and,
 * in the node split, m - 1 extra barriers between the P workgroups.
 *   k_min  >= 2: that threshold; 0: the default (1024); < 0: never (all dense)
 * Process-wide, read when a state is built; returns FM_OK.
 */
int fm_set_iterative_block_min(int32_t k_min);

/*
 * The GPU setup pass (Algorithm 1, Phase I): the same states as
 * fm_build_frozen_states_w for sources on nodes, with the couplings of every
 * source (face coefficients, upwind weights, identity rows, calibration,
 * Sections 3.1-3.2, and the violating-edge count of eq. (graph-fractions))
 * computed on the device from traveltimes already there, for all sources at
 * once, bit-identical to the host's.  On the device too, one workgroup per
 * source: Kahn's elimination forward and backward (Section 3.5) trims the
 * nodes that lie on no path between cycles, and after the host's SCC search
 * over the remaining core, Kahn's elimination over the components gives the
 * longest-path levels of the condensation DAG in both directions (Section
 * 4.1), and the level-ordered records are written on the device in the
 * host's format.  Host threads place the nodes in level order and factor
 * the blocks, overlapping the device work of the next sources.  The states
 * equal those of fm_build_frozen_states_w (component ids included); their
 * records stay in device memory until a batch first uses them.
 *   T        device [S][N] traveltimes (8-byte aligned), e.g. fm_eikonal_solve's output
 *   s        host [N]; G in g on the host; src_nodes host [S]
 *   receivers as fm_build_frozen_states_w (host, [S][n_rcv][k_per_rcv], weights may be NULL)
 *   nthreads host threads; hip_stream the stream of the device work (NULL: null stream)
 * Device scratch of about min(S, nthreads) x N x 91 bytes (at most ~2.3 GB),
 * pinned host staging of the same chunk x N x 58 bytes, per host thread
 * about 56 x N bytes of device memory and 18 x N bytes of pinned host
 * memory, and a recycled pool of per-source couplings (57 x N bytes each,
 * one per source in flight) are allocated and freed inside the call; each
 * state holds its records
 * (about 80 x N bytes) on the device from the call on.  Face stencil only (fm_grid.stencil
 * 0 or 6, else FM_EINVAL).  Errors: as fm_build_frozen_states_w (a T that is
 * not finite or not 0 at the source gives FM_EINVAL); FM_EHIP for a failed
 * HIP call.
 */
int fm_build_frozen_states_gpu(const fm_grid* g, int32_t S, const double* T, const double* s,
                               const int64_t* src_nodes, const int64_t* rcv_nodes, const double* rcv_weights,
                               int32_t n_rcv, int32_t k_per_rcv, int32_t nthreads, void* hip_stream,
                               fm_state** out);

/* Structural statistics of a state (Section 5.2, eq. (graph-fractions)). */
int fm_state_stats(const fm_state* st, fm_stats* out);

/*
 * Copy the assembled operator out, in natural node order, for host-side
 * checks: rowptr [N+1], col [E] (predecessor j of row i, ascending), w [E],
 * c [N].  Any pointer may be NULL to skip that array.
 */
int fm_state_export_operator(const fm_state* st, int64_t* rowptr, int32_t* col, double* w,
                             double* c);

/*
 * Copy the graph analysis out: comp [N] SCC id (ids number the components in
 * ascending forward level, then by smallest member node: a topological order
 * of the condensation DAG that both setup paths share), level_fwd [N] and
 * level_rev [N]
 * (longest-path level of the node's component from the sources / towards the
 * sinks of the condensation DAG).  Any pointer may be NULL.
 */
int fm_state_export_graph(const fm_state* st, int32_t* comp, int32_t* level_fwd,
                          int32_t* level_rev);

/* Free a state and its device copy.  Free every batch that uses it first. */
void fm_state_free(fm_state* st);

/*
 * Create a batch over S states for B right-hand sides in FM_FP64 or FM_FP32
 * on the current HIP device.  Uploads the states that are not yet on the
 * device and allocates all scratch ([S][N][B] of the batch precision) so that
 * the apply calls allocate nothing.  tuning may be NULL.  hip_stream is a
 * hipStream_t (NULL: the null stream).  All states must share one grid shape.
 * Errors: FM_EINVAL, FM_ENOMEM, FM_EHIP.
 */
int fm_batch_create(fm_state* const* states, int32_t S, int32_t B, int32_t precision,
                    const fm_tuning* tuning, void* hip_stream, fm_batch** out);

/*
 * Schedule search (the autotuned level chunks of the batching step, §4.4):
 * for the rhs-group kernel and every built node-split shape (threads, nodes
 * per thread in flight) with 2, 4, 8 or 16 workgroups per source that fits
 * the device, create a batch of the given states, run fm_apply_J and
 * fm_apply_JT once, then time reps more pairs with HIP events on hip_stream,
 * and free the batch.  *best receives the fastest schedule (pass it to
 * fm_batch_create); candidates / ms (optional, max_out entries) receive
 * every schedule measured and its milliseconds per J + J^T pair, *n_out the
 * count.  ds, j_out, w, jt_out are device buffers laid out per the modes, as
 * for fm_apply_J / fm_apply_JT (j_out and jt_out are overwritten).  Each
 * candidate allocates its own scratch: call it once, before the Krylov loop,
 * not under graph capture.
 *   cache_path  NULL or "": always search.  Otherwise a text file of earlier
 *               results (created if missing, one line appended per search),
 *               keyed by the device (architecture, compute units), S, B,
 *               precision, the four modes, a hash of every state's level and
 *               block structure and the build of this library: on a match
 *               the stored schedule is returned without running anything,
 *               *n_out = 0 and candidates[0] / ms[0] hold the stored entry.
 * Errors: FM_EINVAL, FM_ENOMEM, FM_EHIP.
 */
int fm_autotune(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* hip_stream,
                const void* ds, int32_t ds_mode, void* j_out, int32_t out_mode, const void* w, int32_t w_mode,
                void* jt_out, int32_t jt_mode, int32_t reps, const char* cache_path, fm_tuning* best,
                fm_tuning* candidates, float* ms, int32_t max_out, int32_t* n_out);

/* Change the stream later applies are enqueued on. */
int fm_batch_set_stream(fm_batch* b, void* hip_stream);

/* The schedule the batch resolved (defaults filled in). */
int fm_batch_tuning(const fm_batch* b, fm_tuning* out);

/*
 * Wait for the batch stream and report whether the applies enqueued since
 * the last call completed normally.  With the node split (fm_tuning.split >
 * 1) the workgroups of one source wait on each other at every level; each
 * wait gives up after about 10 s without progress (possible only when the
 * launch cannot keep all its workgroups resident, e.g. beside other work
 * that holds the device), and that launch then runs to its end with invalid
 * outputs.  That case returns FM_EHIP (and clears the flag).  Each launch
 * starts with its own waits armed again, so a failed launch does not shorten
 * the waits of later ones; callers check this status wherever they
 * synchronise (the Python layer does after every solve and benchmark).
 * Errors: FM_EINVAL, FM_ESTATE, FM_EHIP.
 */
int fm_batch_status(fm_batch* b);

/*
 * Diagnostic of the node split: waits for the batch stream, then writes for
 * every source (host xcd_masks [S]) the set of XCDs (bit i = XCD i) its
 * workgroups ran on in the last apply.  One bit per source means the
 * workgroups exchanged values through one L2 (the fast path); more bits mean
 * that launch used device-scope fences at every level.
 * Errors: FM_EINVAL (no node split), FM_ESTATE, FM_EHIP.
 */
int fm_batch_split_info(fm_batch* b, int32_t* xcd_masks);

/*
 * Primal action dT = J ds for every (source, rhs) pair (Algorithm 1,
 * Phase III): q = c * ds, forward traversal of the condensation DAG, then P.
 *   ds   device, layout per ds_mode (FM_DS_PER_PAIR or FM_DS_BROADCAST)
 *   out  device, layout per out_mode (FM_OUT_NODES or FM_OUT_RECEIVERS),
 *        fully overwritten
 * Enqueued on the batch stream; no allocation, no synchronisation, so the
 * call may be captured in a HIP graph.  Errors: FM_EINVAL, FM_EHIP.
 */
int fm_apply_J(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode);

/*
 * Transpose action (Algorithm 1, Phase III): r = w (FM_W_NODES) or P^T w
 * (FM_W_RECEIVERS), reverse traversal solving A^T lambda = r (singletons by
 * transposed substitution, SCC blocks with the transpose of the same
 * factors), then c * lambda per source (FM_JT_PER_SOURCE) or summed over the
 * sources in source order (FM_JT_SUMMED).  Same stream and capture rules as
 * fm_apply_J.  Errors: FM_EINVAL, FM_EHIP.
 */
int fm_apply_JT(fm_batch* b, const void* w, int32_t w_mode, void* out, int32_t out_mode);

/*
 * Allocation-free variant of fm_apply_J, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  It computes what fm_batch_create + fm_apply_J +
 * fm_batch_free would over the same states, without a batch: the scratch a
 * batch allocates (the state table the kernels index and, for receiver
 * output, the [S][N][B] node values) lives in a fixed device array of 64 MiB
 * that the library holds on every device it runs on until the process ends.
 *   states     S states already resident on the current device in this
 *              precision (an earlier fm_batch_create over them uploaded
 *              them); otherwise FM_ESTATE
 *   B, precision, ds, ds_mode, out, out_mode   as for fm_batch_create / fm_apply_J
 *   hip_stream where the work is enqueued (NULL: the null stream)
 * Runs the rhs-group schedule (no node split).  Allocates nothing and does not
 * synchronise.  Calls that overlap on one device share that device's array
 * and race: issue them on one stream or wait between them.
 * Errors: FM_EINVAL (shapes, modes, or more than 64 MiB of scratch needed:
 * sizeof(state table) + S*N*B*(8 or 4) bytes with receiver output),
 * FM_ESTATE, FM_EHIP.
 */
int fm_apply_J_static(fm_state* const* states, int32_t S, int32_t B, int32_t precision, void* hip_stream,
                      const void* ds, int32_t ds_mode, void* out, int32_t out_mode);

/*
 * Comparison baseline, not the method: the same J and J^T computed by
 * directional Gauss-Seidel sweeping (Section 3.6) on the GPU, without the
 * graph analysis.  Every (source, rhs) system is swept over the 2^dim axis
 * orderings (hyperplane by hyperplane, newest values) from zero until a whole
 * cycle changes no entry by more than 1e-15 * max|x| or max_cycles cycles
 * have run.  Layouts as fm_apply_J / fm_apply_JT, except that the transpose
 * takes nodal input only (FM_W_NODES).  The first call on a batch uploads
 * natural-order copies of W and W^T and so allocates device memory.
 * cycles: NULL, or host [S * B / rhs_per_group] receiving the cycles each
 * workgroup used (negative: not converged); non-NULL makes the call wait for
 * the stream.  Errors: FM_EINVAL, FM_ENOMEM, FM_EHIP.
 */
int fm_apply_J_sweep(fm_batch* b, const void* ds, int32_t ds_mode, void* out, int32_t out_mode,
                     int32_t max_cycles, int32_t* cycles);
int fm_apply_JT_sweep(fm_batch* b, const void* w, void* out, int32_t out_mode, int32_t max_cycles,
                      int32_t* cycles);

/*
 * LSQR over the paired actions: the Krylov least-squares inner loop of
 * Algorithm 1 (Section 4.5), which applies J and J^T once per
 * iteration at the same frozen state.  It solves min ||J x - d||_2 for each
 * of the B columns independently: x is a model block [N][B] shared by all
 * sources (FM_DS_BROADCAST), d is stacked receiver data [S][R][B], J^T sums
 * over the sources.  All vectors and per-column scalars live on the device;
 * create allocates them once, the other calls only enqueue kernels on the
 * batch stream (no allocation, no synchronisation, no memset), so
 * fm_lsqr_capture can record n iterations as one HIP graph that
 * fm_lsqr_replay launches again and again.  Free the plan before its batch.
 *   fm_lsqr_start    beta u = d, alpha v = J^T u, w = v, x = 0 (d: device [S][R][B])
 *   fm_lsqr_iterate  enqueue n iterations
 *   fm_lsqr_capture  record n iterations into a graph (needs a non-null stream)
 *   fm_lsqr_replay   launch the recorded graph
 *   fm_lsqr_buffers  device pointers of x [N][B], u [S][R][B], v [N][B] and the
 *                    scalars [8][B] (alpha, beta, rhobar, phibar, rho, phi, theta, 1/norm);
 *                    |phibar| is the current residual norm of each column
 * Errors: FM_EINVAL, FM_ENOMEM, FM_EHIP, FM_ESTATE.
 */
typedef struct fm_lsqr fm_lsqr;
int fm_lsqr_create(fm_batch* b, fm_lsqr** out);
int fm_lsqr_start(fm_lsqr* L, const void* d);
int fm_lsqr_iterate(fm_lsqr* L, int32_t n);
int fm_lsqr_capture(fm_lsqr* L, int32_t n);
int fm_lsqr_replay(fm_lsqr* L);
int fm_lsqr_buffers(const fm_lsqr* L, void** x, void** u, void** v, double** scalars);
void fm_lsqr_free(fm_lsqr* L);

/*
 * CGLS over the paired actions: the inner solve of a Gauss-Newton step
 * (Algorithm 1, Phase III, with CGLS in place of LSMR and no regularisation),
 * min ||J x - d||_2 for each of the B columns independently, J and J^T applied
 * once per iteration at the same frozen state.  Layouts as for LSQR: x and the
 * search direction are model blocks [N][B] (FM_DS_BROADCAST), d and the
 * residual r are stacked receiver data [S][R][B], J^T sums over the sources.
 * Per column: x_0 = 0, r_0 = d, s_0 = J^T d, p_0 = s_0, gamma_0 = ||s_0||^2;
 * then q = J p, alpha = gamma / ||q||^2, x += alpha p, r -= alpha q,
 * s = J^T r, gamma' = ||s||^2, p = s + (gamma'/gamma) p.  A column whose
 * denominators reach zero stops moving.  Same rules as LSQR: everything is on
 * the device, create allocates, the other calls only enqueue kernels on the
 * batch stream, and fm_cgls_capture records n iterations as one HIP graph.
 *   fm_cgls_create   max_iter: rows of the residual history (>= 0)
 *   fm_cgls_buffers  device pointers of x [N][B], r [S][R][B], the scalars
 *                    [6][B] (gamma, ||q||^2, alpha, gamma', beta, ||r||^2)
 *                    and the history [max_iter + 1][B] of ||r||^2: row 0 at
 *                    start, row k after the k-th iteration enqueued since
 *                    start (iterations past max_iter are not recorded; a
 *                    captured graph rewrites the rows it recorded)
 * Errors: FM_EINVAL, FM_ENOMEM, FM_EHIP, FM_ESTATE.
 */
typedef struct fm_cgls fm_cgls;
int fm_cgls_create(fm_batch* b, int32_t max_iter, fm_cgls** out);
int fm_cgls_start(fm_cgls* C, const void* d);
int fm_cgls_iterate(fm_cgls* C, int32_t n);
int fm_cgls_capture(fm_cgls* C, int32_t n);
int fm_cgls_replay(fm_cgls* C);
int fm_cgls_buffers(const fm_cgls* C, void** x, void** r, double** scalars, double** history);
void fm_cgls_free(fm_cgls* C);

/*
 * First-arrival traveltimes on the GPU (the state of Section 2.1: T the
 * viscosity solution of |grad_x T| = s, T = 0 at the source; Algorithm 1,
 * Phase I).  The paper only cites its own solver; the library's
 * discretisation is a monotone semi-Lagrangian update on the
 * boundary-conforming grid: node i takes the least value of
 * T(y) + s_i |x_i - y| over the points y of its stencil's simplices (face
 * neighbours, segments joining neighbours on two different axes, and in 3-D
 * triangles with one neighbour per axis), T linear over each simplex, x the
 * physical positions.  Seeds: nodes within max-norm logical distance
 * seed_radius of the source's logical coordinates keep the straight-ray time
 * (s_src + s_p)/2 |x_p - x_src| (s_src, x_src multilinear over the source's
 * cell; a source on a node is integer coordinates, T = 0 there).  The update
 * is monotone, so every iteration order reaches the same largest fixed point
 * from T = +inf; the solver runs Jacobi iterations (a node is recomputed only
 * when a neighbour changed) until one changes nothing.
 *
 * fm_eikonal_create: X host [N][dim] physical node coordinates (copied);
 *   room for up to max_sources sources per solve (device scratch of
 *   max_sources x N x 10 bytes); work is enqueued on hip_stream (NULL: the
 *   null stream).
 * fm_eikonal_solve: s device [N] slowness (finite, > 0), xi_src host [S][dim]
 *   logical source coordinates in [0, n_d - 1], seed_radius >= 0 logical
 *   units (the region must hold a node), T device [S][N] output, 8-byte
 *   aligned; iterations (may be NULL) receives the number of Jacobi
 *   iterations, the last one changing nothing.  Synchronises the stream.
 *   Errors: FM_EINVAL for bad arguments, FM_ESTATE when no fixed point is
 *   reached within max_iter iterations (T then holds the last iterate) or the
 *   solver lives on another device, FM_EHIP for a failed HIP call.
 */
typedef struct fm_eikonal fm_eikonal;
int fm_eikonal_create(int32_t dim, int64_t n1, int64_t n2, int64_t n3, const double* X, int32_t max_sources,
                      void* hip_stream, fm_eikonal** out);
int fm_eikonal_set_stream(fm_eikonal* e, void* hip_stream);
int fm_eikonal_solve(fm_eikonal* e, const double* s, int32_t S, const double* xi_src, double seed_radius,
                     int32_t max_iter, double* T, int32_t* iterations);
void fm_eikonal_free(fm_eikonal* e);

/*
 * Cell-velocity model map M_alpha (Section 4.4, eq. (source-jacobian)): the
 * model is one velocity per cell of the logical grid (hexahedra between
 * nodes, quadrilaterals in 2-D; cell id ci + (n1-1) (cj + (n2-1) ck), 2-D
 * ci + (n1-1) ck), and a node's slowness is the reciprocal of the mean
 * velocity of the 1, 2, 4 or 8 cells that share it.  The map linearises this
 * at the given velocities:
 *   (M dv)_p  = a_p sum_{cells c of node p} dv_c,   a_p = -1 / (n_p vbar_p^2)
 *   (M^T g)_c = sum_{nodes p of cell c} a_p g_p
 * M is shared by all sources, so J M is fm_apply_J of the broadcast block
 * M dv, and M^T follows fm_apply_JT's summed output.
 *   create     dim, n1, n2, n3 as in fm_grid (every axis of the grid >= 2
 *              nodes); v_cell host [n_cells] finite and > 0 (copied);
 *              hip_stream: where the applies run; uses the current device
 *   sizes      node and cell counts
 *   slowness   host s_out [N]: the background nodal slowness 1 / vbar
 *   apply      device dv [n_cells][B] -> ds [N][B]; apply_T device
 *              g [N][B] -> out [n_cells][B]; FP64 or FP32 (precision as in
 *              fm_batch_create); asynchronous on the map's stream; no
 *              allocation; outputs fully overwritten
 * Errors: FM_EINVAL (shape, velocity not finite or <= 0, null pointer, B < 1),
 * FM_ESTATE (another current device), FM_ENOMEM, FM_EHIP.
 */
typedef struct fm_model_map fm_model_map;
int fm_model_map_create(int32_t dim, int64_t n1, int64_t n2, int64_t n3, const double* v_cell, void* hip_stream,
                        fm_model_map** out);
int fm_model_map_sizes(const fm_model_map* m, int64_t* n_nodes, int64_t* n_cells);
int fm_model_map_slowness(const fm_model_map* m, double* s_out);
int fm_model_map_set_stream(fm_model_map* m, void* hip_stream);
int fm_model_map_apply(fm_model_map* m, int32_t B, int32_t precision, const void* dv, void* ds);
int fm_model_map_apply_T(fm_model_map* m, int32_t B, int32_t precision, const void* g, void* dv_out);
void fm_model_map_free(fm_model_map* m);

/* Free a batch (its scratch); the states stay valid. */
void fm_batch_free(fm_batch* b);

/* Message for the last nonzero return on this thread ("" if none). */
const char* fm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FMBTF_H */
