/*
 * gs.h -- C ABI of the MI355X (gfx950) point-set geodesic shooting library.
 *
 * The library evaluates the right-hand side of the Gaussian-kernel Hamiltonian
 * flow of point-set geodesic shooting and integrates it, exactly (all pairs)
 * or with a Barnes-Hut octree approximation, following Wang, Xie, Yushkevich,
 * Gee, "Barnes-Hut Approximation for Point Set Geodesic Shooting"
 * (arXiv:1907.04834).
 *
 * Mathematical definitions (Sec. 2.1, eq. 1 and eq. 3):
 *   G(r)  = exp(-r^2 / (2 sigma^2))                      (unnormalised, G(0)=1)
 *   v_i   = sum_j G(|q_i - q_j|) p_j                    (self term included)
 *   a_i   = sigma^-2 sum_j G(|q_i - q_j|) (p_i . p_j) (q_i - q_j)
 *   dq/dt = v,  dp/dt = a   (Hamilton's equations for 1/2 <p, K(q) p>)
 *   H     = <p, K(q) p> = sum_i p_i . v_i
 *
 * Common conventions for every entry point
 *   - Point arrays (q, p, dq, dp, q0, p0, q1, p1, target, grad) are DEVICE
 *     pointers to row-major [n][3] arrays (x, y, z of point 0, then point 1,
 *     ...), float32 unless the name ends in _f64.  The caller owns them.
 *   - `ws` is a caller-owned DEVICE workspace of at least gs_workspace_bytes()
 *     bytes (256-byte aligned).  The library allocates no device memory and
 *     keeps no pointer to it after a call returns.  Calls on one point set
 *     take everything they need from their sizes and copy nothing from the
 *     host.  Calls on several sets (the batched calls with nsub > 1) and the
 *     velocity field copy small host-planned tables into the workspace with
 *     one asynchronous copy from pinned staging buffers of the library (per
 *     thread, allocated on first use, kept until the process ends): a call
 *     takes a buffer whose previous copy has completed, the pool grows to at
 *     most 32 buffers, and only a call issued while 32 earlier copies of its
 *     thread are still queued waits on the host for the oldest.  Such a call
 *     must not be captured into a caller's own HIP graph (the captured copy
 *     would read a buffer that later calls reuse); GS_FLAG_GRAPH captures
 *     shootings and gradients safely (their tables are copied by every call,
 *     outside the graph).
 *   - Process-lifetime state of the library, none of it device memory: the
 *     staging buffers above, up to 8 cached work-item plans of batched exact
 *     calls (keyed by the set sizes), and up to 16 graphs of GS_FLAG_GRAPH
 *     calls (keyed by every pointer, size and parameter of the call).
 *   - `stream` is the HIP stream every kernel is enqueued on.  Calls only
 *     enqueue work and return; results are valid once the stream reaches the
 *     point after the call.  The library never synchronises the stream
 *     except in gs_get_status / gs_bh_counters / gs_kernel_timing_read.
 *   - Argument errors are reported before any device work is enqueued:
 *     n < 0, non-finite or non-positive sigma, nt < 1, theta < 0 or NaN,
 *     cutoff_sigmas <= 0 or NaN, leaf_cap outside [1, 64], unknown flags, a
 *     NULL array when n > 0, or a workspace that is too small.  n == 0 is a
 *     no-op (GS_OK).
 *   - Accuracy does not depend on where a point set lies: the FP32 kernels
 *     work on positions relative to an FP64 origin per set (the method
 *     depends only on differences q_i - q_j): the exact all-pairs path uses
 *     the centre of the set's box, the Barnes-Hut path that centre rounded to
 *     a multiple of the smallest power of two not below the box side (0 for
 *     a set around the origin, so that its differences are those of the
 *     inputs).  The Barnes-Hut decisions are taken in FP64 on the positions
 *     as given.
 *   - Outputs must not alias inputs, except q1/p1 which may equal q0/p0.
 *   - gs_last_error() returns a thread-local message for the last failure.
 *   - Calls are reentrant when they use distinct workspaces.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID = -1,     /* bad argument (see conventions above)        */
    GS_ERR_WORKSPACE = -2,   /* workspace pointer NULL or too small         */
    GS_ERR_HIP = -3,         /* a HIP call or kernel launch failed          */
    GS_ERR_NONFINITE = -4,   /* non-finite coordinates met on the tree path */
    GS_ERR_UNSUPPORTED = -5, /* combination of options not implemented      */
    GS_ERR_OVERFLOW = -6     /* a Barnes-Hut traversal stack overflowed      */
} gs_status;

typedef enum {
    GS_EXACT = 0,  /* all N^2 pairs (Sec. 2.1)                              */
    GS_BH = 1      /* Barnes-Hut octree approximation (Sec. 2.2)             */
} gs_method;

/* Operation codes for gs_workspace_bytes. */
typedef enum {
    GS_OP_RHS = 0,      /* gs_rhs_exact / gs_rhs_bh / gs_rhs_exact_f64        */
    GS_OP_SHOOT = 1,    /* gs_shoot / gs_shoot_f64                            */
    GS_OP_ADJOINT = 2,  /* gs_shoot_adjoint                                   */
    GS_OP_FIELD = 3     /* gs_field with n targets and n sources; for other
                           sizes use gs_field_workspace_bytes                 */
} gs_op;

/* flags */
#define GS_FLAG_F64 1u        /* size the workspace for the _f64 entry points */
#define GS_FLAG_GRAPH 4u      /* gs_shoot, gs_shoot_batch, gs_shoot_adjoint,
                                 gs_shoot_adjoint_batch: capture the call's
                                 kernel sequence into a HIP graph on first use
                                 and replay it on later calls with the same
                                 arguments (pointers, sizes, offsets and
                                 parameters; at most 16 graphs are kept, least
                                 recently used dropped).  Cuts the launch
                                 overhead of small problems; results are those
                                 of the call without the flag.               */

typedef struct {
    double sigma;          /* kernel width, > 0                                */
    double cutoff_sigmas;  /* kappa: a node is far when the distance from the
                              target to its tight box is >= kappa * sigma
                              (the paper's 3 sigma rule, Sec. 2.2)           */
    double theta;          /* opening angle >= 0: an approximated node must
                              also satisfy s_k < theta |x - C_k| (s_k: largest
                              side of its tight box).  INFINITY = the paper's
                              rule alone; 0 = exact.                         */
    int32_t leaf_cap;      /* octree leaves hold <= leaf_cap points (1..64);
                              1 = the paper's single-point leaves            */
    int32_t nt;            /* forward-Euler steps over t in [0, 1], >= 1     */
    uint32_t flags;        /* GS_FLAG_*                                       */
    int32_t exact_items;   /* exact FP32 path: work items (one block: 64
                              targets x one source chunk, split among its
                              waves) that a launch aims at; 0 = the library
                              default (24576), else
                              256..4194304.  Changes speed and workspace
                              size, not results beyond the order in which
                              the partial sums are added;
                              gs_autotune_exact picks it.                    */
} gs_params;

/* Library version string (static storage). */
const char *gs_version(void);

/* Message of the last failed call on this thread (static per thread). */
const char *gs_last_error(void);

/* Fills *p with the defaults: sigma 1, cutoff 3, theta 0.5, leaf_cap 1,
 * nt 40, flags 0. */
void gs_params_default(gs_params *p);

/* Workspace bytes needed by `op` for n points with these parameters and
 * method.  Host-only; no device work.  Returns 0 for invalid arguments. */
size_t gs_workspace_bytes(int64_t n, const gs_params *prm, int32_t method, int32_t op);

/* Exact right-hand side (Sec. 2.1, eq. 1 and the pairwise velocity of eq. 3):
 * (dq, dp) = (v, a) as defined above, all N^2 pairs, FP32 pair arithmetic
 * with per-target compensated accumulation.  Uses prm->sigma only. */
gs_status gs_rhs_exact(const float *q, const float *p, int64_t n, const gs_params *prm,
                       float *dq, float *dp, void *ws, size_t ws_bytes, hipStream_t stream);

/* The same in FP64 (q, p, dq, dp are double[n][3]).  The workspace is that
 * of gs_workspace_bytes(n, prm with GS_FLAG_F64, GS_EXACT, GS_OP_RHS) (its
 * header only: the status word). */
gs_status gs_rhs_exact_f64(const double *q, const double *p, int64_t n,
                           const gs_params *prm, double *dq, double *dp, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* Barnes-Hut right-hand side (Sec. 2.2, eq. 4 and the momentum-dot
 * replacement): rebuilds the octree of q (root cube anchored at the per-axis
 * minimum with side equal to the largest extent; octants from 21-bit integer
 * coordinates; a node with more than leaf_cap points below level 21 is split),
 * then for every target x walks it from the root: a node with >= 2 points
 * that is far (kappa sigma) and passes the opening angle contributes as n_k
 * virtual points at its centre C_k with momentum P_k / n_k each; a leaf that
 * is not approximated contributes its exact pairs; other nodes are opened.
 * Non-finite coordinates make gs_get_status report GS_ERR_NONFINITE. */
gs_status gs_rhs_bh(const float *q, const float *p, int64_t n, const gs_params *prm,
                    float *dq, float *dp, void *ws, size_t ws_bytes, hipStream_t stream);

/* Geodesic shooting (Sec. 2.1: the flow of eq. 1 discretised in time):
 * prm->nt forward-Euler steps of size 1/nt from (q0, p0), each step using the
 * right-hand side of `method` evaluated at the state at the start of the
 * step.  Writes q1 = q(1), p1 = p(1).  H (nullable, DEVICE double[nt + 1])
 * receives <p_t, v_t> for t = 0..nt (FP64 reduction; v from `method`).  The
 * state is carried as FP32 (hi, lo) pairs and each step is taken in
 * double-float arithmetic; FP64 serves only the H reduction. */
gs_status gs_shoot(const float *q0, const float *p0, int64_t n, const gs_params *prm,
                   int32_t method, float *q1, float *p1, double *H, void *ws,
                   size_t ws_bytes, hipStream_t stream);

/* Exact shooting in FP64 (arrays are double[n][3]). */
gs_status gs_shoot_f64(const double *q0, const double *p0, int64_t n,
                       const gs_params *prm, double *q1, double *p1, double *H,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* Objective and gradient (Sec. 2.1 eq. 2; backward stage of Sec. 2.2):
 *   E(p0) = (1/n) sum_i |q_i(1) - target_i|^2 + lambda <p0, K(q0) p0>
 * and grad = dE/dp0 by the discrete adjoint of the Euler scheme:
 *   alpha(1) = 2 (q(1) - target) / n, beta(1) = 0;
 *   (alpha, beta)_t = (alpha, beta)_{t+1} + dt J(q_t, p_t)^T (alpha, beta)_{t+1};
 *   grad = beta(0) + 2 lambda K(q0) p0.
 * The forward states are kept (FP64) every `ckpt_every` steps and the steps
 * in between are recomputed during the backward sweep.  With GS_BH the
 * forward steps are Barnes-Hut steps and the backward products use the tree
 * of q_t with node sums of alpha and beta: an approximated node contributes
 * as n_k virtual points carrying the node means of p, alpha and beta (the
 * paper's backward stage).  objective is a DEVICE double[1]; grad_p0 a
 * DEVICE float[n][3]; target a DEVICE float[n][3].  ckpt_every >= 1 (values
 * above nt act as nt); lambda finite.  The workspace comes from
 * gs_adjoint_workspace_bytes (gs_workspace_bytes with GS_OP_ADJOINT assumes
 * ckpt_every = 8). */
size_t gs_adjoint_workspace_bytes(int64_t n, const gs_params *prm, int32_t method,
                                  int32_t ckpt_every);
gs_status gs_shoot_adjoint(const float *q0, const float *p0, const float *target,
                           int64_t n, const gs_params *prm, int32_t method,
                           double lambda, int32_t ckpt_every, double *objective,
                           float *grad_p0, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* Velocity field of eq. (3) at m arbitrary points x (DEVICE float[m][3]):
 * v(x) = sum_j G(|x - q_j|) p_j over the n sources (q, p).  Exact sum, FP32
 * pairs with compensated FP32 accumulation, positions relative to the
 * sources' box centre.  The workspace comes from gs_field_workspace_bytes (0 for invalid
 * arguments). */
size_t gs_field_workspace_bytes(int64_t m, int64_t n, const gs_params *prm);
gs_status gs_field(const float *x, int64_t m, const float *q, const float *p, int64_t n,
                   const gs_params *prm, float *v, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* Batched sets.  Sec. 3.2 registers every subject of a population (665
 * subjects x 2 hemispheres) with its own, independent shooting; the
 * implementation details of Sec. 2.2 run such jobs side by side on a
 * cluster.  Here nsub point sets are stored one after the other: set s is
 * rows [offsets[s], offsets[s+1]) of q / p / q0 / p0 and of the outputs.
 * `offsets` is a HOST array of nsub + 1 int64 values with offsets[0] = 0,
 * non-decreasing (empty sets allowed); 1 <= nsub <= 65536.  Every set is
 * evaluated exactly as the corresponding single-set call would evaluate it
 * alone (its own octree with its own root cube on the Barnes-Hut path; no
 * interaction between sets), in shared launches.  The library copies small
 * tables derived from `offsets` into the workspace with an asynchronous copy
 * from its own pinned staging memory; `offsets` may be freed on return.
 * The workspace comes from gs_batch_workspace_bytes (op GS_OP_RHS,
 * GS_OP_SHOOT or GS_OP_ADJOINT, the last with ckpt_every = 8; 0 for invalid
 * arguments). */
size_t gs_batch_workspace_bytes(const int64_t *offsets, int32_t nsub, const gs_params *prm,
                                int32_t method, int32_t op);

/* Right-hand side of every set (gs_rhs_exact / gs_rhs_bh per set). */
gs_status gs_rhs_batch(const float *q, const float *p, const int64_t *offsets, int32_t nsub,
                       const gs_params *prm, int32_t method, float *dq, float *dp, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* Shooting of every set (gs_shoot per set).  H (nullable) is a DEVICE
 * double[nsub][nt + 1]: row s holds the energies of set s. */
gs_status gs_shoot_batch(const float *q0, const float *p0, const int64_t *offsets,
                         int32_t nsub, const gs_params *prm, int32_t method, float *q1,
                         float *p1, double *H, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* Objective and gradient of every set (gs_shoot_adjoint per set, Sec. 2.1
 * eq. 2 and the backward stage of Sec. 2.2; subjects of a population are
 * registered independently, Sec. 3.2).  Set s has
 *   E_s = (1/n_s) sum_{i in s} |q_i(1) - target_i|^2 + lambda <p0, K(q0) p0>_s
 * with n_s its number of points; grad_p0 rows of set s hold dE_s/dp0.
 * objective is a DEVICE double[nsub] (0 for an empty set); target and grad_p0
 * are DEVICE float[n][3], n = offsets[nsub] (n == 0: no-op).  Checkpoints as
 * in gs_shoot_adjoint.  The workspace comes from
 * gs_adjoint_batch_workspace_bytes (0 for invalid arguments). */
size_t gs_adjoint_batch_workspace_bytes(const int64_t *offsets, int32_t nsub,
                                        const gs_params *prm, int32_t method,
                                        int32_t ckpt_every);
gs_status gs_shoot_adjoint_batch(const float *q0, const float *p0, const float *target,
                                 const int64_t *offsets, int32_t nsub, const gs_params *prm,
                                 int32_t method, double lambda, int32_t ckpt_every,
                                 double *objective, float *grad_p0, void *ws, size_t ws_bytes,
                                 hipStream_t stream);

/* Tuning of the Barnes-Hut leaf capacity for given inputs (one set: offsets
 * {0, n}, nsub 1; or a batch).  Times one right-hand side for each leaf_cap
 * in {8, 16, 32, 48, 64} (after a warm-up run, best of two) on `stream`,
 * waiting for each, and writes the fastest into prm->leaf_cap (other fields
 * unchanged) and its time in milliseconds into *best_ms (nullable).  Larger
 * leaves only turn approximated interactions into exact pairs, so the
 * choice never makes the result less accurate.  dq, dp (DEVICE float[n][3])
 * receive the trial right-hand sides; the workspace is that of
 * gs_batch_workspace_bytes(offsets, nsub, prm, GS_BH, GS_OP_RHS) (it does
 * not depend on leaf_cap).  Synchronous: a set-up call, not a hot-path one. */
gs_status gs_autotune_leaf_cap(const float *q, const float *p, const int64_t *offsets,
                               int32_t nsub, gs_params *prm, float *dq, float *dp, void *ws,
                               size_t ws_bytes, hipStream_t stream, double *best_ms);

/* Tuning of the exact FP32 path (gs_rhs_exact, gs_shoot, gs_shoot_adjoint
 * and the batched calls with GS_EXACT) for given inputs: times one
 * right-hand side for each exact_items in {6144, 12288, 24576, 49152} whose
 * workspace fits ws_bytes (after a warm-up run, best of two) on `stream`,
 * waiting for each, and writes the fastest into prm->exact_items (other
 * fields unchanged) and its time in milliseconds into *best_ms (nullable).
 * offsets / nsub as for the batched calls (one set: {0, n}, 1).  dq, dp
 * (DEVICE float[n][3]) receive the trial right-hand sides.  A workspace of
 * gs_batch_workspace_bytes(offsets, nsub, prm, GS_EXACT, GS_OP_RHS) with
 * prm->exact_items = 49152 fits every candidate.  Synchronous: a set-up
 * call. */
gs_status gs_autotune_exact(const float *q, const float *p, const int64_t *offsets, int32_t nsub,
                            gs_params *prm, float *dq, float *dp, void *ws, size_t ws_bytes,
                            hipStream_t stream, double *best_ms);

/* Diagnostic (for checking the octree against its definition; not a
 * hot-path call): builds the octree of (q, p) exactly as gs_rhs_bh does
 * (Sec. 2.2, octree representation) in `ws` (the workspace of gs_rhs_bh),
 * waits for `stream` and copies it to HOST arrays:
 *   keys[n]   the sorted 63-bit Morton keys (21 bits per axis interleaved,
 *             x highest in each triple of bits);
 *   perm[n]   the input index of each sorted point;
 *   *n_nodes  the number of stored nodes.  The stored tree is the compressed
 *             octree: a chain of single-child cells is stored as its deepest
 *             cell (they hold the same points); node 0 is the root; the
 *             children of a node are contiguous.
 * When *n_nodes <= max_nodes it also writes, per node k: node_start[k] its
 * first sorted point (its points are perm[node_start[k] ..
 * node_start[k] + node_count[k] - 1]), node_count[k], node_first[k] (its
 * first child node; for a leaf, its first sorted point), node_nchild[k] (0
 * for a leaf) and node_stats[13 k ..] = centre C (3, FP64), momentum sum P
 * (3, as stored in FP32), tight box lo (3), hi (3) and the square of its
 * largest side.  Synchronous. */
gs_status gs_tree_export(const float *q, const float *p, int64_t n, const gs_params *prm,
                         void *ws, size_t ws_bytes, hipStream_t stream, int64_t max_nodes,
                         int64_t *n_nodes, uint64_t *keys, uint32_t *perm, int32_t *node_start,
                         int32_t *node_count, int32_t *node_first, int32_t *node_nchild,
                         double *node_stats);

/* Exact right-hand side that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Computes what gs_rhs_exact computes,
 * with its workspace in a static device array of the library of
 * GS_STATIC_SCRATCH_BYTES (64 MiB), which every device the library runs on
 * holds until the process ends; the array's device address is looked up on
 * the first call on each device, with that device current.  n must be at
 * most GS_STATIC_MAX_N (500 000): larger n returns GS_ERR_WORKSPACE before any
 * device work.  The work-item target (prm->exact_items, 0 = the default) is
 * halved, not below 256, until the workspace fits the array, which changes
 * only the order in which partial sums are added.  The call copies nothing from the host and
 * only enqueues kernels on `stream`, so it may be captured into a HIP graph.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (no result depends on them): calls that overlap on one
 * device (other streams, other threads, graph replays still running) race
 * and corrupt each other's results, so the caller must serialise them. */
#define GS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
#define GS_STATIC_MAX_N ((int64_t)500000)
gs_status gs_rhs_exact_static(const float *q, const float *p, int64_t n, const gs_params *prm,
                              float *dq, float *dp, hipStream_t stream);

/* Waits for `stream` and returns the device-side status word of the last
 * Barnes-Hut call that used this workspace: GS_OK; GS_ERR_NONFINITE when a
 * coordinate was NaN or infinite (the results are not meaningful); or
 * GS_ERR_OVERFLOW when a traversal stack overflowed (the results of that call
 * are incomplete; trees of at most 22 levels cannot overflow it). */
gs_status gs_get_status(const void *ws, hipStream_t stream);

/* Waits for `stream` and copies the counters of the last Barnes-Hut call
 * (gs_rhs_bh, gs_shoot or a batched call with GS_BH) that used this
 * workspace, summed over all sets,
 * all targets and all right-hand sides that call evaluated (nt + 1 for a
 * shooting that returns H, nt otherwise): out[0] exact pairs, out[1]
 * monopoles (approximated nodes), out[2] node visits, out[3] octree nodes.
 * Wave-level diagnostics of the GPU traversal: out[4] leaf-point steps
 * executed by waves (each serves up to 64 targets), out[5] node records
 * decided by waves, out[6] the largest out[4] + out[5] of a single wave,
 * out[7] the largest out[5] of a single phase-1 (decision) wave. */
#define GS_BH_COUNTERS 8
gs_status gs_bh_counters(const void *ws, hipStream_t stream, int64_t out[GS_BH_COUNTERS]);

/* Per-launch timing of the dominant kernels.  While enabled, every launch of
 * a timed kernel kind is bracketed by HIP events on its stream.
 * gs_kernel_timing_read waits for the recorded events and returns, per kind
 * k, the number of launches counts[k] and their summed duration ms[k]
 * (milliseconds); reading resets the accumulators.  Kinds: 0 exact
 * all-pairs (v and a), 1 Barnes-Hut traversal (v and a), 2 adjoint pair
 * kernels, 3 octree build (its whole launch sequence), 4 exact all-pairs
 * velocity only, 5 Barnes-Hut traversal velocity only. */
#define GS_TIMING_KINDS 6
gs_status gs_kernel_timing(int32_t enable);
gs_status gs_kernel_timing_read(int64_t counts[GS_TIMING_KINDS], double ms[GS_TIMING_KINDS]);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
