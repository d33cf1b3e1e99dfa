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

// One node as the traversal reads it (80 bytes; wave-uniform loads).
struct alignas(16) BhNode {
    double cx, cy, cz;  // centre of the member positions (mean, FP64)
    double s2;          // (largest side of the tight box)^2, FP64
    float lox, loy, loz, hix;
    float hiy, hiz, px, py;  // tight box (exact), total momentum (FP32)
    float pz;
    int n;       // number of points
    int first;   // leaf: first sorted point; internal: first child node
    int nchild;  // 0 for a leaf
};
static_assert(sizeof(BhNode) == 80, "BhNode layout");

// Small device-side header of one tree build.
struct TreeMeta {
    float lo[3];
    float hi[3];
    double extent;      // E
    double scale;       // 2^21 / E (0 when E == 0)
    int nonfinite;      // a coordinate was NaN or +-inf
    int root_leaf;      // 1 when the root is a leaf
    int n_internal;     // compressed internal nodes (excluding a leaf root)
    int n_nodes;        // stored nodes
    int root_rank;      // internal rank of the root (if internal)
    int pad;
};

struct TreeBufs {
    int64_t n;
    int bbox_blocks;
    int sort_blocks;
    TreeMeta *meta;
    float *bbox_part;          // [bbox_blocks][6]
    unsigned long long *keyA, *keyB;
    unsigned *valA, *valB;     // permutation (original index of sorted point)
    unsigned *hist;            // [256][sort_blocks]
    unsigned *scan_part;       // block sums of the generic scan
    float4 *Qs, *Ps;           // sorted points / momenta (FP32)
    unsigned char *lvl;        // [n-1] split level of each boundary
    unsigned *flag;            // [n] internal-node flag per boundary, then rank
    unsigned *rank;            // [n] exclusive scan of flag
    unsigned *bnd_s, *bnd_e;   // [n] cell range of an internal boundary
    unsigned *rank_bnd;        // [n] boundary of internal rank r
    unsigned *nchild;          // [n] children of internal rank r
    unsigned *cstart;          // [n] exclusive scan of nchild
    int *node_of;              // [n] node id of internal rank r
    int *parent_rank;          // [2n] internal rank of a node's parent (-1 root)
    unsigned *counter;         // [2n] bottom-up arrival counters (adjoint sums)
    int *node_start;           // [2n] first sorted point of each node
    char *chunk0, *chunk1;     // range summaries of 64 and 4096 sorted points
    double *nsum;              // [2n][6] FP64 sums of q and p per node
    BhNode *nodes;             // [2n]
    double *adj;               // [2n][6] per-node sums of alpha, beta (backward stage)
    // traversal work split (see traverse.hip)
    char *list;                // [groups][kListCap] leaf entries of each group
    int *list_n;               // [groups] entries used
    double *part;              // [1 + chunks][groups * 64][6] partial (v, a) sums
};
// Sizes of the traversal's work-split buffers (defined in traverse.hip).
size_t traverse_list_bytes(int64_t n);
size_t traverse_part_doubles(int64_t n);
void carve_tree(Arena &a, int64_t n, TreeBufs &t);

// Builds the tree of (q, p) (float [n][3]) into t.  `status` (nullable) is an
// int on the device set to 1 when a coordinate is not finite.
gs_status build_tree(const float *q, const float *p, int64_t n, int leaf_cap, TreeBufs &t,
                     int *status, hipStream_t s);

// Adds FP64 node sums of per-point vectors (alpha, beta; [n][3] each, original
// order) into t.adj, bottom-up over the built tree.
gs_status tree_adjoint_sums(const double *alpha, const double *beta, TreeBufs &t, hipStream_t s);

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

// The decision for target x and node nd (FP64, in the order of the
// definition): approximate when the node holds >= 2 points, the distance from
// x to its tight box is at least kappa sigma, and s_k^2 < theta^2 |x - C_k|^2.
__device__ __forceinline__ bool decide(const BhNode &nd, double x, double y, double z,
                              const BhParams &bp) {
#pragma clang fp contract(off)
    double dmin2 = 0.0;
    {
        const double below = (double)nd.lox - x, above = x - (double)nd.hix;
        const double g = below > above ? below : above;
        if (g > 0.0) dmin2 += g * g;
    }
    {
        const double below = (double)nd.loy - y, above = y - (double)nd.hiy;
        const double g = below > above ? below : above;
        if (g > 0.0) dmin2 += g * g;
    }
    {
        const double below = (double)nd.loz - z, above = z - (double)nd.hiz;
        const double g = below > above ? below : above;
        if (g > 0.0) dmin2 += g * g;
    }
    const bool far = dmin2 >= bp.cut2;
    const double dx = x - nd.cx, dy = y - nd.cy, dz = z - nd.cz;
    double d2 = dx * dx;
    d2 += dy * dy;
    d2 += dz * dz;
    const bool mac = bp.theta_inf || (nd.s2 < bp.th2 * d2);
    return nd.n >= 2 && far && mac;
}



// Forward traversal.  Writes (v, a) for every point in original order: as FP32
// into dq/dp when they are non-null, else it advances the FP64 state
// (Sq += dt v, Sp += dt a), refreshes the FP32 copies q32/p32 and adds
// p . v per block into Hpart (nullable).  counters (4 x u64, zeroed by the
// build) receive exact pairs, monopoles and node visits.
struct TraverseOut {
    float *dq, *dp;                    // RHS mode
    double *Sq, *Sp;                   // shooting mode
    float *q32, *p32;
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
int traverse_blocks(int64_t n);

struct ShootBhBufs {
    TreeBufs tree;
    double *Sq, *Sp;   // FP64 state [n][3]
    float *q32, *p32;  // FP32 copies [n][3]
    double *Hpart;
};
ShootBhBufs layout_shoot_bh(Arena &a, int64_t n, int nt);

gs_status rhs_bh(const float *q, const float *p, int64_t n, const gs_params &prm, float *dq,
                 float *dp, TreeBufs &t, char *ws, hipStream_t s);
gs_status shoot_bh(const float *q0, const float *p0, int64_t n, const gs_params &prm, float *q1,
                   float *p1, double *H, ShootBhBufs &b, char *ws, hipStream_t s);

}  // namespace gs
