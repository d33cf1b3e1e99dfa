// adjoint.hip -- backward stage (Sec. 2.1 eq. 2 objective; Sec. 2.2 backward
// stage): discrete adjoint of the forward-Euler flow, exact all-pairs form,
// and the checkpointed forward / backward sweep of both methods.
//
// For Phi = sum_k alpha_k . v_k + beta_k . a_k the vector-Jacobian product of
// the right-hand side is, with d = q_k - q_j, G = G(|d|), s = p_k . p_j and
// db = beta_k - beta_j:
//   g_q,k = sigma^-2 sum_j G { -d [ p_j . alpha_k + p_k . alpha_j ]
//                               + s [ db - d (d . db) / sigma^2 ] }
//   g_p,k = sum_j G alpha_j + sigma^-2 sum_j G p_j (d . db)
// and one backward Euler step is (alpha, beta)_t = (alpha, beta)_{t+1} +
// dt (g_q, g_p) evaluated at (q_t, p_t) with (alpha, beta)_{t+1}.
//
// The exact products use the forward work items (a block of 256 targets
// against a source chunk of its own set) on positions stored as q' = k q,
// k = sqrt(log2(e) / (2 sigma^2)), so that G = exp2(-|q'_k - q'_j|^2).  The
// adjoint variables are stored as alpha' = alpha / k and beta' = beta / (k^2
// sigma^2).  With d' = k d, db' = beta'_k - beta'_j and c = d' . db' (which
// equals (d . db) / (k sigma^2)):
//   sum G { -d' [ s c + p_j . alpha'_k + p_k . alpha'_j ] }
//     + k^2 sigma^2 sum G s db'                         = sigma^2 g_q,k
//   sum G alpha'_j + sum G c p_j                        = g_p,k / k
// so a pair costs 38 VALU operations and one exp2.
#include <hip/hip_runtime.h>

#include "adjoint.h"

namespace gs {

namespace {

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__device__ inline double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) s += lds[k];
    return s;
}

// FP64 state from float [n][3] inputs.
__global__ void k_state64(const float *__restrict__ q, const float *__restrict__ p, int64_t n3,
                          double *__restrict__ Sq, double *__restrict__ Sp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    Sq[i] = q[i];
    Sp[i] = p[i];
}

// Terminal adjoint of unit u (points of one set): alpha = 2 (q - y) / n_s,
// beta = 0, and the unit's sum of |q - y|^2.
__global__ __launch_bounds__(256) void k_terminal_units(const double *__restrict__ q,
                                                        const float *__restrict__ y,
                                                        const int4 *__restrict__ units, RowGeom rg,
                                                        const double *__restrict__ setn,
                                                        double n1, double *__restrict__ al,
                                                        double *__restrict__ be,
                                                        double *__restrict__ part) {
    __shared__ double lds[8];
    const int4 d = row_block(units, rg, blockIdx.x);
    double e = 0.0;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        const double ns = setn ? setn[d.z] : n1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double r = q[3 * i + c] - (double)y[3 * i + c];
            e += r * r;
            al[3 * i + c] = 2.0 * r / ns;
            be[3 * i + c] = 0.0;
        }
    }
    const double s = block_sum(e, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// objective[s] = data[s] / n_s + lambda H[s] (0 for an empty set).
__global__ void k_objective_sets(const double *__restrict__ dsum,
                                 const double *__restrict__ hsum,
                                 const double *__restrict__ setn, double n1, int nsub,
                                 double lambda, double *__restrict__ obj) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsub) return;
    const double ns = setn ? setn[s] : n1;
    obj[s] = ns > 0.0 ? dsum[s] / ns + lambda * hsum[s] : 0.0;
}

// Work item b = (first target row, source rows [j0, j1) of the same set,
// partial slot; slot -1: padding item), with the layout of the forward pair
// kernel: wave (group g, split w) takes targets it.x + 64 g + lane and the
// w-th share (whole tiles) of the chunk; the waves of a group add their
// sums in LDS in split order.  FP32 pairs summed per tile of kTile sources
// and accumulated in FP64.  Padding rows hold zero p, alpha', beta' and add
// exactly zero.  bscale = k^2 sigma^2.  The source loop is not unrolled:
// measured at 50k points, 2.01 ms per launch against 2.39 ms unrolled by 4
// (76 VGPRs, 6 waves per SIMD) and 2.45 ms with the source tile staged in
// LDS.
__global__ __launch_bounds__(kItemThreads) void k_adj_items(
    const float4 *__restrict__ Q, const float4 *__restrict__ P, const float4 *__restrict__ AL,
    const float4 *__restrict__ BE, int64_t npad, const int4 *__restrict__ items, ItemGeom geom,
    double bscale, double *__restrict__ part) {
    __shared__ double red[kItemSplit > 1 ? kItemSplit - 1 : 1][6][kItemRows];
    const int4 it = work_item(items, geom, blockIdx.x);
    if (it.w < 0) return;  // padding item: the whole block leaves before any barrier
    const int wv = wave_in_block();
    const int grp = wv % kItemGroups, w = wv / kItemGroups;
    const int r = grp * 64 + (threadIdx.x & 63);
    const int64_t i = (int64_t)it.x + r;
    const float4 qa = Q[i], pa4 = P[i], aa = AL[i], ba = BE[i];
    const float x = qa.x, y = qa.y, z = qa.z;
    const float px = pa4.x, py = pa4.y, pz = pa4.z;
    const float ax = aa.x, ay = aa.y, az = aa.z;
    const float bx = ba.x, by = ba.y, bz = ba.z;
    double sq[3] = {0, 0, 0}, spp[3] = {0, 0, 0};
    const int ntile = (it.z - it.y) / kTile;
    const int per = (ntile + kItemSplit - 1) / kItemSplit;
    const int j0 = it.y + min(w * per, ntile) * kTile;
    const int j1 = it.y + min((w + 1) * per, ntile) * kTile;
    for (int jt = j0; jt < j1; jt += kTile) {  // 32-bit: scalar-unit compares
        float tq[3] = {0.f, 0.f, 0.f}, tb[3] = {0.f, 0.f, 0.f}, tp[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
        for (int u = 0; u < kTile; ++u) {
            const float4 qj = Q[jt + u], pj = P[jt + u], aj = AL[jt + u], bj = BE[jt + u];
            const float dx = x - qj.x, dy = y - qj.y, dz = z - qj.z;
            const float g = __builtin_amdgcn_exp2f(-(dx * dx + dy * dy + dz * dz));
            const float s = px * pj.x + py * pj.y + pz * pj.z;
            const float pa = pj.x * ax + pj.y * ay + pj.z * az;
            const float ap = px * aj.x + py * aj.y + pz * aj.z;
            const float dbx = bx - bj.x, dby = by - bj.y, dbz = bz - bj.z;
            const float c2 = dx * dbx + dy * dby + dz * dbz;
            const float w1 = -g * fmaf(s, c2, pa + ap);
            const float w2 = g * s;
            const float w3 = g * c2;
            tq[0] = fmaf(w1, dx, tq[0]);
            tq[1] = fmaf(w1, dy, tq[1]);
            tq[2] = fmaf(w1, dz, tq[2]);
            tb[0] = fmaf(w2, dbx, tb[0]);
            tb[1] = fmaf(w2, dby, tb[1]);
            tb[2] = fmaf(w2, dbz, tb[2]);
            tp[0] = fmaf(g, aj.x, tp[0]);
            tp[1] = fmaf(g, aj.y, tp[1]);
            tp[2] = fmaf(g, aj.z, tp[2]);
            tp[0] = fmaf(w3, pj.x, tp[0]);
            tp[1] = fmaf(w3, pj.y, tp[1]);
            tp[2] = fmaf(w3, pj.z, tp[2]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sq[c] += (double)tq[c] + (double)tb[c] * bscale;
            spp[c] += (double)tp[c];
        }
    }
    if (kItemSplit > 1) {
        if (w > 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[w - 1][c][r] = sq[c];
                red[w - 1][3 + c][r] = spp[c];
            }
        __syncthreads();
        if (w == 0)
            for (int k = 0; k < kItemSplit - 1; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sq[c] += red[k][c][r];
                    spp[c] += red[k][3 + c][r];
                }
    }
    if (w != 0) return;
    double *dst = part + (int64_t)it.w * 6 * npad;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dst[c * npad + i] = sq[c];
        dst[(3 + c) * npad + i] = spp[c];
    }
}

// (alpha, beta) += dt (sigma^-2 S_q, k S_p) from the partial slots of each row.
__global__ __launch_bounds__(256) void k_adj_update_rows(const double *__restrict__ part,
                                                         int64_t npad,
                                                         const int4 *__restrict__ blk, RowGeom rg,
                                                         double inv_s2, double ks, double dt,
                                                         double *__restrict__ al,
                                                         double *__restrict__ be) {
    const int4 d = row_block(blk, rg, blockIdx.x);
    if ((int)threadIdx.x >= d.y) return;
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = (int64_t)d.x + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < d.w; ++s)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += part[((int64_t)s * 6 + c) * npad + row];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        al[3 * i + c] += dt * (acc[c] * inv_s2);
        be[3 * i + c] += dt * (acc[3 + c] * ks);
    }
}

// grad = beta_0 + 2 lambda v_0
__global__ void k_grad(const double *__restrict__ be, const double *__restrict__ v0,
                       int64_t n3, double lambda, float *__restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) grad[i] = (float)(be[i] + 2.0 * lambda * v0[i]);
}

}  // namespace

// ---------------------------------------------------------------- host side
void carve_adjoint_common(Arena &a, int64_t n, int nsub, int nt, int ckpt, int nunits,
                          AdjointBufs &b) {
    b.n = n;
    b.nsub = nsub;
    b.nt = nt;
    b.ckpt = ckpt;
    b.nck = (nt + ckpt - 1) / ckpt;
    const int64_t m = n > 0 ? n : 1;
    b.al = a.take<double>(3 * m);
    b.be = a.take<double>(3 * m);
    b.v0 = a.take<double>(3 * m);
    b.ckq = a.take<double>((size_t)b.nck * 3 * m);
    b.ckp = a.take<double>((size_t)b.nck * 3 * m);
    b.segq = a.take<double>((size_t)ckpt * 3 * m);
    b.segp = a.take<double>((size_t)ckpt * 3 * m);
    b.nunits = nunits;
    b.dpart = a.take<double>(nunits > 0 ? nunits : 1);
    b.dsum = a.take<double>(nsub);
    b.hsum = a.take<double>(nsub);
}

// Restores the packed FP32 rows of the exact path from the FP64 state.
static gs_status exact_repack(AdjointBufs &b, const gs_params &prm, hipStream_t s) {
    return launch_pack_rows64(*b.xp, b.ex, b.Sq, b.Sp, position_scale(prm.sigma), b.ex.Q, b.ex.P,
                              s, 1.0, true);
}

// One forward Euler step of the chosen method from the FP64 state (b.Sq,
// b.Sp) and its FP32 copies.  With v0 non-null, also stores the step's
// velocity there and its energy partials in b.hpart.
static gs_status forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                              char *ws, hipStream_t s) {
    if (b.bh) return bh_adjoint_forward_step(b, prm, dt, v0, ws, s);
    GS_TRY(launch_exact_items(*b.xp, b.ex, true, s));
    return launch_combine_rows(*b.xp, b.ex, prm.sigma, 1, nullptr, nullptr, dt,
                               v0 ? b.hpart : nullptr, s, v0);
}

// One backward step at state (q_t, p_t) = (sq, sp): (al, be) += dt J^T (al, be).
static gs_status adjoint_step(AdjointBufs &b, const gs_params &prm, double dt, const double *sq,
                              const double *sp, char *ws, hipStream_t s) {
    if (b.bh) return bh_adjoint_step(b, prm, dt, sq, sp, ws, s);
    const ExactBatchPlan &pl = *b.xp;
    const int64_t ni = plan_item_count(pl);
    if (ni == 0) return GS_OK;
    const double ks = position_scale(prm.sigma);
    GS_TRY(launch_pack_rows64(pl, b.ex, sq, sp, ks, b.ex.Q, b.ex.P, s, 1.0, true));
    const double bscale = ks * ks * prm.sigma * prm.sigma;
    GS_TRY(launch_pack_rows64(pl, b.ex, b.al, b.be, 1.0 / ks, b.AL, b.BE, s, 1.0 / bscale,
                              false));
    // the backward products keep FP64 partial sums (in the forward partials'
    // memory: 8 bytes a value either way)
    double *part = reinterpret_cast<double *>(b.ex.part);
    timing_begin(KIND_ADJOINT, s);
    hipLaunchKernelGGL(k_adj_items, dim3((unsigned)ni), dim3(kItemThreads), 0, s, b.ex.Q, b.ex.P,
                       b.AL, b.BE, pl.npad, pl.single ? nullptr : b.ex.items, pl.geom, bscale,
                       part);
    timing_end(KIND_ADJOINT, s);
    GS_LAUNCH_CHECK("adj_items");
    hipLaunchKernelGGL(k_adj_update_rows, dim3((unsigned)plan_block_count(pl)), dim3(256), 0, s,
                       part, pl.npad, b.ex.blk, pl.rows, 1.0 / (prm.sigma * prm.sigma), ks,
                       dt, b.al, b.be);
    GS_LAUNCH_CHECK("adj_update_rows");
    return GS_OK;
}

gs_status shoot_adjoint(const float *q0, const float *p0, const float *y, const gs_params &prm,
                        double lambda, double *objective, float *grad, AdjointBufs &b, char *ws,
                        hipStream_t s) {
    const int64_t n = b.n, n3 = 3 * n;
    const double dt = 1.0 / prm.nt;
    if (n3 > 0) {
        if (b.bh) {
            GS_TRY(bh_adjoint_begin(q0, b, ws, s));
            hipLaunchKernelGGL(k_state64, dim3(nblk(n3)), dim3(kBlock), 0, s, q0, p0, n3, b.Sq,
                               b.Sp);
            GS_LAUNCH_CHECK("state64");
        } else {
            GS_TRY(launch_pack_state_rows(*b.xp, b.ex, q0, p0, prm.sigma, s));
        }
        // forward sweep with checkpoints every b.ckpt steps
        for (int t = 0; t < prm.nt; ++t) {
            if (t % b.ckpt == 0) {
                const int c = t / b.ckpt;
                GS_TRY(launch_copy_f64(b.Sq, b.ckq + (size_t)c * n3, n3, s));
                GS_TRY(launch_copy_f64(b.Sp, b.ckp + (size_t)c * n3, n3, s));
            }
            GS_TRY(forward_step(b, prm, dt, t == 0 ? b.v0 : nullptr, ws, s));
        }
        // terminal adjoint and the per-set data term
        if (b.nunits > 0) {
            hipLaunchKernelGGL(k_terminal_units, dim3((unsigned)b.nunits), dim3(256), 0, s, b.Sq,
                               y, b.units, b.urows, b.setn, (double)b.n, b.al, b.be, b.dpart);
            GS_LAUNCH_CHECK("terminal");
        }
    }
    GS_TRY(launch_reduce_h_seg(b.dpart, b.nunits, b.useg, b.nsub, 1, b.dsum, s));
    GS_TRY(launch_reduce_h_seg(b.hpart, b.nh, b.hseg, b.nsub, 1, b.hsum, s));
    hipLaunchKernelGGL(k_objective_sets, dim3(nblk(b.nsub)), dim3(kBlock), 0, s, b.dsum, b.hsum,
                       b.setn, (double)b.n, b.nsub, lambda, objective);
    GS_LAUNCH_CHECK("objective");
    if (n3 == 0) return GS_OK;
    // backward sweep, one checkpoint segment at a time
    for (int c = b.nck - 1; c >= 0; --c) {
        const int t0 = c * b.ckpt;
        const int t1 = t0 + b.ckpt < prm.nt ? t0 + b.ckpt : prm.nt;
        GS_TRY(launch_copy_f64(b.ckq + (size_t)c * n3, b.Sq, n3, s));
        GS_TRY(launch_copy_f64(b.ckp + (size_t)c * n3, b.Sp, n3, s));
        if (!b.bh && t1 - t0 > 1) GS_TRY(exact_repack(b, prm, s));
        for (int t = t0; t < t1; ++t) {
            GS_TRY(launch_copy_f64(b.Sq, b.segq + (size_t)(t - t0) * n3, n3, s));
            GS_TRY(launch_copy_f64(b.Sp, b.segp + (size_t)(t - t0) * n3, n3, s));
            if (t + 1 < t1) GS_TRY(forward_step(b, prm, dt, nullptr, ws, s));
        }
        for (int t = t1 - 1; t >= t0; --t)
            GS_TRY(adjoint_step(b, prm, dt, b.segq + (size_t)(t - t0) * n3,
                                b.segp + (size_t)(t - t0) * n3, ws, s));
    }
    hipLaunchKernelGGL(k_grad, dim3(nblk(n3)), dim3(kBlock), 0, s, b.be, b.v0, n3, lambda, grad);
    GS_LAUNCH_CHECK("grad");
    return GS_OK;
}

}  // namespace gs
