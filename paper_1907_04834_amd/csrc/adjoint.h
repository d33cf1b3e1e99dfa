// adjoint.h -- backward stage (discrete adjoint of the Euler flow).
#pragma once

#include "internal.h"
#include "tree.h"

namespace gs {

// Buffers of the Barnes-Hut backward stage.
struct BhAdjBufs {
    float4 *ALs, *BEs;  // alpha, beta in Morton order (FP32)
    double *gq, *gp;    // per-target products J^T (alpha, beta) (original order)
};
BhAdjBufs layout_bh_adjoint(Arena &a, int64_t n);

struct AdjointBufs {
    int64_t n;
    int nt, ckpt, nck, nblk;  // nblk: data-term partials (blocks of 256 points)
    int nh;                   // energy partials (blocks, or tree groups on the tree path)
    bool bh;
    ExactPlan pl;
    ExactBufs ex;             // packed state and partial sums of the exact kernels
    float4 *AL, *BE;          // packed adjoint variables (exact path)
    double *Sq, *Sp;          // FP64 state
    double *al, *be;          // FP64 adjoint variables
    double *v0;               // velocity at t = 0
    double *ckq, *ckp;        // checkpoints [nck][n][3]
    double *segq, *segp;      // states of one segment [ckpt][n][3]
    double *hpart, *dpart;    // energy and data-term block partials
    ShootBhBufs sh;           // Barnes-Hut forward buffers (tree, FP32 copies)
    BhAdjBufs bhadj;
};
AdjointBufs layout_adjoint(Arena &a, int64_t n, int nt, int ckpt, int method);

gs_status shoot_adjoint(const float *q0, const float *p0, const float *y, const gs_params &prm,
                        double lambda, double *objective, float *grad, AdjointBufs &b, char *ws,
                        hipStream_t s);

// Barnes-Hut hooks (bh_adjoint.hip).
gs_status bh_adjoint_begin(AdjointBufs &b, char *ws, hipStream_t s);
gs_status bh_adjoint_forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                                  char *ws, hipStream_t s);
gs_status bh_adjoint_step(AdjointBufs &b, const gs_params &prm, double dt, const double *sq,
                          const double *sp, char *ws, hipStream_t s);

}  // namespace gs
