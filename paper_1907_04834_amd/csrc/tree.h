// tree.h -- Barnes-Hut octree: device data layout, workspace and launchers.
//
// The octree is the one of Sec. 2.2 ("Oct-tree Representation of Space"):
// the root cube is anchored at the per-axis minimum with side E = largest
// extent; octants are picked from 21-bit integer coordinates
// c = min(2^21 - 1, floor((q - lo) * 2^21 / E)) (FP64); a cell with more than
// leaf_cap points below level 21 is split; points sharing a level-21 cell
// stay together.  The GPU stores the compressed form of that tree: chains of
// single-child cells (which have the statistics of their only child) are
// represented by their deepest cell, so every stored internal node has >= 2
// children.  Children of a node are stored contiguously.
#pragma once

#include "internal.h"

namespace gs {

constexpr int kLevels = 21;

// The counter copy that block (bx, by) adds into.
__device__ inline unsigned long long *counter_slot(unsigned long long *c, unsigned bx,
                                                   unsigned by = 0) {
    return c + (size_t)((bx + by) % kCounterSlots) * GS_BH_COUNTERS;
}

// One node as the traversal reads it (112 bytes, staged as 7 float4s).  The
// tight box is stored in FP64: it is the exact FP32 box, converted once here
// instead of at every decision.
struct alignas(16) BhNode {
    double cx, cy, cz;  // centre of the member positions (mean, FP64)
    double s2;          // (largest side of the tight box)^2, FP64
    double lo[3];       // tight box (exact: FP64 of the FP32 bounds)
    double hi[3];
    float px, py, pz;   // total momentum (FP32)
    int n;              // number of points
    int first;          // leaf: first sorted point; internal: first child node
    int nchild;         // 0 for a leaf
    int pad0, pad1;
};
static_assert(sizeof(BhNode) == 112, "BhNode layout");
constexpr int kNodeF4 = (int)(sizeof(BhNode) / 16);  // float4s per node record

// Device-side header of the tree of one point set (one per subject when
// several independent point sets are built together as a forest).
struct TreeMeta {
    float lo[3];
    float hi[3];
    double extent;      // E
    double scale;       // 2^21 / E (0 when E == 0)
    double cen[3];      // centre (lo + hi) / 2 of the box (FP64; 0 if not finite)
    int nonfinite;      // a coordinate was NaN or +-inf
    int root_leaf;      // 1 when the root is a leaf
    int root_rank;      // internal rank of the root (if internal)
    int pad;
};

// Totals of a build: internal nodes of all trees, stored nodes (roots
// included).
struct TreeTotals {
    int n_internal;
    int n_nodes;
};

// Targets of one traversal wave: `count` (<= 64) consecutive sorted points
// from `first`, all in the tree whose root is node `root`.
struct GroupDesc {
    int first;
    int count;
    int root;
    int sub;
};

// Forest layout.  Point sets s = 0..nsub-1 occupy the index ranges
// [seg[s], seg[s+1]) of the input; the build sorts every set within its own
// range, so sorted index ranges equal input ranges.  Node s is the root of
// set s.  With seg == nullptr there is one set [0, n).
struct TreeBufs {
    int64_t n;
    int nsub;
    const long long *seg;      // [nsub + 1] device offsets (nullable: one set)
    int64_t groups;            // traversal groups
    const GroupDesc *gtab;     // [groups] (nullable: group g = points [64g, 64g + 64))
    int bbox_blocks;           // per set
    int sort_per;              // radix-sort keys per thread (tiles of 256 x sort_per)
    int sort_tiles;            // radix-sort tiles
    int sort_sbs;              // superblocks of 16 tiles
    int sort_passes;
    int block_sort;            // 1: every set has at most 2048 points, one block sorts each;
                               // 2: one set of at most 32768, sorted in tiles and merged
    TreeMeta *meta;            // [nsub]
    TreeTotals *totals;
    float *bbox_part;          // [nsub][bbox_blocks][6]
    unsigned long long *keyA, *keyB;
    unsigned *valA, *valB;     // ping-pong buffers of the sort
    const unsigned long long *K;  // sorted keys (one of keyA / keyB)
    const unsigned *perm;      // original index of each sorted point
    unsigned *hist;            // [sort_tiles][512] digit counts of each tile
    unsigned *sb;              // [2][sort_sbs][512] digit counts of each superblock
    unsigned *scan_part;       // block sums of the generic scan
    float4 *Qs, *Ps;           // sorted points / momenta (FP32, as given: the decisions)
    float4 *Qc;                // sorted points minus their set's frame origin (FP32, pairs)
    unsigned char *lvl;        // [n-1] split level of each boundary
    unsigned *flag;            // [n] internal-node flag per boundary, then rank
    unsigned *rank;            // [n] exclusive scan of flag
    unsigned *bnd_s, *bnd_e;   // [n] cell range of an internal boundary
    unsigned *rank_bnd;        // [n] boundary of internal rank r
    unsigned *nchild;          // [n] children of internal rank r
    unsigned *cstart;          // [n] exclusive scan of nchild
    unsigned *crun;            // [n][9] child starts of internal rank r, then the cell end
    int *node_start;           // [2n + nsub] first sorted point of each node
    char *chunk0, *chunk1;     // range summaries of 64 and 4096 sorted points
    double *nsum;              // [nodes][6] FP64 sums of q and p per node
    BhNode *nodes;             // [2n + nsub]
    double *adj;               // [nodes][6] per-node sums of alpha, beta (backward stage)
    // traversal work split (see traverse.hip)
    char *list;                // leaf entries of each group, one segment per phase-1 wave
    int *list_n;               // entries used per segment
    double *part;              // [slots][groups * 64][6] partial (v, a) sums: FP64 (backward
                               // stage) or, reinterpreted, float2 hi+lo (forward traversal)
};
// Sizes of the traversal's work-split buffers (defined in traverse.hip).
size_t traverse_list_bytes(int64_t groups);
size_t traverse_count_ints(int64_t groups);
size_t traverse_part_doubles(int64_t groups);
// One tree over n points.
void carve_tree(Arena &a, int64_t n, TreeBufs &t);
// A forest of nsub sets with n points in total and `groups` traversal
// groups; the caller sets t.seg and t.gtab before building.
void carve_forest(Arena &a, int64_t n, int nsub, int64_t groups, int64_t max_set, TreeBufs &t);

// Builds the tree (or forest) of (q, p) (float [n][3]) into t.  `status`
// (nullable) is an int on the device set to 1 when a coordinate is not
// finite.
gs_status build_tree(const float *q, const float *p, int64_t n, int leaf_cap, TreeBufs &t,
                     int *status, hipStream_t s);
// Frame origin of every set of q (FP32 [n][3]; its box centre rounded to a
// multiple of a power of two, see frame_origin) into c0 (FP64 [nsub][3]); uses
// the tree's box buffers and sets `status` for non-finite coordinates.
// c0f (nullable) receives the same origins as double-float.
gs_status tree_set_centres(const float *q, TreeBufs &t, double *c0, float2 *c0f, int *status,
                           hipStream_t s);
// The state of float inputs, FP64 (Sq, Sp) or hi+lo (Fq, Fp; the other pair
// null), and its FP32 copies q32 = q - c0[set], p32 = p; one thread per point.
gs_status launch_state_init(const float *q0, const float *p0, const TreeBufs &t, const double *c0,
                            const float2 *c0f, double *Sq, double *Sp, float2 *Fq, float2 *Fp,
                            float *q32, float *p32, hipStream_t s);
// FP32 copies q32 = Sq - c0[set], p32 = Sp of an FP64 state.
gs_status launch_state_to_f32(const double *Sq, const double *Sp, const TreeBufs &t,
                              const double *c0, float *q32, float *p32, hipStream_t s);

// Traversal parameters (FP64 decision thresholds as in the definition).
struct BhParams {
    float negc;        // -log2(e) / (2 sigma^2)
    float inv_s2f;     // 1 / sigma^2 (FP32)
    double inv_s2;     // 1 / sigma^2
    double cut2;       // (kappa sigma)^2
    double th2;        // theta^2
    int theta_inf;     // theta == +inf
    int pad;
};
BhParams make_bh_params(const gs_params &prm);

// The decision for target x and node nd with n_k >= 2 (FP64, in the order of
// the definition; n_k is the same for every target, so callers test it once):
// approximate when the distance from x to the node's tight box is at least
// kappa sigma and s_k^2 < theta^2 |x - C_k|^2.  d receives x - C_k (FP64).
// The distance to the box adds, per axis in order, the square of
// max(lo - x, x - hi) when it is positive; adding the square of max(that, 0)
// instead gives the same FP64 sum (a skipped term adds an exact zero).
__device__ __forceinline__ bool decide_far(const BhNode &nd, double x, double y, double z,
                                          const BhParams &bp, double *d) {
#pragma clang fp contract(off)
    const double gx = fmax(fmax(nd.lo[0] - x, x - nd.hi[0]), 0.0);
    const double gy = fmax(fmax(nd.lo[1] - y, y - nd.hi[1]), 0.0);
    const double gz = fmax(fmax(nd.lo[2] - z, z - nd.hi[2]), 0.0);
    double dmin2 = gx * gx;
    dmin2 += gy * gy;
    dmin2 += gz * gz;
    d[0] = x - nd.cx;
    d[1] = y - nd.cy;
    d[2] = z - nd.cz;
    double d2 = d[0] * d[0];
    d2 += d[1] * d[1];
    d2 += d[2] * d[2];
    const bool far = dmin2 >= bp.cut2;
    const bool mac = bp.theta_inf || (nd.s2 < bp.th2 * d2);
    return far && mac;
}

// A wave-uniform 64-bit value held in LDS or VGPRs, as scalars.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Forward traversal.  Writes (v, a) for every point in original order: as FP32
// into dq/dp (MODE_RHS), or it advances the state (MODE_SHOOT: q += dt v,
// p += dt a, hi+lo in Fq/Fp when Fq is set, else FP64 in Sq/Sp), refreshes
// the FP32 copies q32/p32 and writes the sum of p . v of every traversal
// group into Hpart[group] (nullable).
// counters (zeroed by the caller) receive exact pairs, monopoles, node
// visits and the wave statistics.
struct TraverseOut {
    float *dq, *dp;                    // RHS mode
    // shooting: hi+lo state [n][3] (hi, lo) pairs, in the order of the points
    // the tree was built from (the previous step's sorted order, or the
    // original order at the first step); the advanced state, q32 and p32 are
    // written in this tree's sorted order into Fq_out / Fp_out, and ord_out
    // receives the original index of each sorted point (ord_in: the same for
    // the build's input order; null: the original order itself)
    const float2 *Fq, *Fp;
    float2 *Fq_out, *Fp_out;
    const unsigned *ord_in;
    unsigned *ord_out;
    double *Sq, *Sp;                   // the backward stage's forward steps: FP64 state
    float *q32, *p32;                  // FP32 copies: q32 = q - c0[set]
    const double *c0;                  // [nsub][3] frame origins of the shooting
    const float2 *c0f;                 // [nsub][3] the same as double-float (hi+lo state)
    double dt;
    double *Hpart;
    double *v64;                       // velocity only (energy pass), nullable
};
gs_status launch_bh_traverse(const TreeBufs &t, const BhParams &bp, bool with_a,
                             const TraverseOut &o, unsigned long long *counters, hipStream_t s);
enum Mode { MODE_RHS = 0, MODE_SHOOT = 1, MODE_ENERGY = 2 };
gs_status launch_bh_traverse(const TreeBufs &t, const BhParams &bp, bool with_a,
                             const TraverseOut &o, unsigned long long *counters, hipStream_t s,
                             int mode, int *status);

// Per-node FP64 sums of two per-point vector fields given in Morton order
// (A, B as float4 [n]); out is [n_nodes][6] (sums of A then B).  Uses the
// same 64 / 4096-point range summaries as the node statistics.
gs_status tree_range_sums(const float4 *A, const float4 *B, TreeBufs &t, double *out,
                          hipStream_t s);

struct ShootBhBufs {
    TreeBufs tree;
    float2 *Fq, *Fp;   // shooting state, FP32 (hi, lo) pairs [n][3]
    float2 *Fq2, *Fp2; // the same, the other buffer (the state moves to each
                       // step's sorted order)
    unsigned *ord, *ord2;  // original index of each point of a sorted state [n]
    double *Sq, *Sp;   // FP64 state [n][3] (the backward stage's forward steps)
    float *q32, *p32;  // FP32 copies [n][3], q32 relative to c0
    double *c0;        // [nsub][3] frame origins of q0, fixed for the call
    float2 *c0f;       // [nsub][3] the same as double-float
    double *Hpart;     // [nt + 1][groups]
    const int *gseg;   // [nsub + 1] group range of each set (nullable: one set)
};
// state: kStateFF (shooting) or kStateF64 (the backward stage's forward steps).
ShootBhBufs layout_shoot_bh(Arena &a, int64_t n, int nt, int state = kStateFF);
// The same for a forest; the caller sets tree.seg, tree.gtab and gseg.
ShootBhBufs layout_shoot_forest(Arena &a, int64_t n, int nsub, int64_t groups, int64_t max_set,
                                int nt, int state = kStateFF);

gs_status rhs_bh(const float *q, const float *p, int64_t n, const gs_params &prm, float *dq,
                 float *dp, TreeBufs &t, char *ws, hipStream_t s);
// Shooting of one set, or of every set of a forest (H then holds nsub rows of
// nt + 1 energies).
gs_status shoot_bh(const float *q0, const float *p0, int64_t n, const gs_params &prm, float *q1,
                   float *p1, double *H, ShootBhBufs &b, char *ws, hipStream_t s);

}  // namespace gs
