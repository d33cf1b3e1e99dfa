// adjoint.h -- backward stage (discrete adjoint of the Euler flow) of one
// point set or of a batch of independent sets stored one after the other
// (set s = points [offsets[s], offsets[s+1])); one set is a batch of one.
#pragma once

#include "internal.h"
#include "tree.h"

namespace gs {

// Buffers of the Barnes-Hut backward products.
struct BhAdjBufs {
    float4 *ALs, *BEs;  // alpha, beta in Morton order (FP32)
};
BhAdjBufs layout_bh_adjoint(Arena &a, int64_t n);

struct AdjointBufs {
    int64_t n;                // points of all sets
    int nsub, nt, ckpt, nck;
    bool bh;
    // exact path: the work-item plan, its packed state and partial sums
    const ExactBatchPlan *xp;
    ExactBatchBufs ex;
    float4 *AL, *BE;          // [npad] packed adjoint variables (alpha / k, beta)
    // Barnes-Hut path: the forest, its FP32 copies and traversal buffers
    ShootBhBufs sh;
    BhAdjBufs bhadj;
    // both paths
    double *Sq, *Sp;          // FP64 state [n][3] (ex.Sq / sh.Sq)
    double *al, *be;          // FP64 adjoint variables [n][3]
    double *v0;               // velocity at t = 0 [n][3]
    double *ckq, *ckp;        // checkpoints [nck][n][3]
    double *segq, *segp;      // states of one segment [ckpt][n][3]
    double *hpart;            // energy partials of step 0 (exact: row blocks, BH: groups)
    int nh;
    const int *hseg;          // [nsub + 1] partial range of each set
    double *dpart;            // data-term partials, one per unit
    int nunits;
    const int4 *units;        // [nunits] (first point, count <= 256, set, -); null: the
    RowGeom urows;            // row blocks of one set (urows)
    const int *useg;          // [nsub + 1] unit range of each set
    const double *setn;       // [nsub] points of each set (null: one set of n points)
    double *dsum, *hsum;      // [nsub] data term and energy of each set
};
// Carves the buffers that both paths add to their forward buffers; the
// caller fills the path-specific members and the tables.
void carve_adjoint_common(Arena &a, int64_t n, int nsub, int nt, int ckpt, int nunits,
                          AdjointBufs &b);

// objective: DEVICE double[nsub]; grad: float [n][3].
gs_status shoot_adjoint(const float *q0, const float *p0, const float *y, const gs_params &prm,
                        double lambda, double *objective, float *grad, AdjointBufs &b, char *ws,
                        hipStream_t s);

// Barnes-Hut hooks (bh_adjoint.hip).
gs_status bh_adjoint_begin(const float *q0, AdjointBufs &b, char *ws, hipStream_t s);
gs_status bh_adjoint_forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                                  char *ws, hipStream_t s);
gs_status bh_adjoint_step(AdjointBufs &b, const gs_params &prm, double dt, const double *sq,
                          const double *sp, char *ws, hipStream_t s);

}  // namespace gs
