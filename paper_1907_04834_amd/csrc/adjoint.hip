// adjoint.hip -- backward stage (Sec. 2.1 eq. 2 objective; Sec. 2.2 backward
// stage): discrete adjoint of the forward-Euler flow, exact all-pairs form.
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
// k_adj_pairs has the layout of the forward all-pairs kernel: one target per
// lane, wave-uniform (scalar-load) sources q, p, alpha, beta, FP32 pair
// arithmetic, tiles of kTile sources summed in FP32 and accumulated in FP64,
// source splits (split-fastest block order), FP64 partial sums combined in a
// fixed order.
#include <hip/hip_runtime.h>

#include "adjoint.h"

namespace gs {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

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

// FP64 [n][3] pair of arrays -> zero-padded FP32 float4 copies.
__global__ void k_pack2(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                        int64_t npad, float4 *__restrict__ A, float4 *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i < n) {
        A[i] = make_float4((float)a[3 * i], (float)a[3 * i + 1], (float)a[3 * i + 2], 0.f);
        B[i] = make_float4((float)b[3 * i], (float)b[3 * i + 1], (float)b[3 * i + 2], 0.f);
    } else {
        A[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        B[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__global__ void k_copy(const double *__restrict__ s, double *__restrict__ d, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) d[i] = s[i];
}

// Terminal adjoint: alpha = 2 (q - y) / n, beta = 0; block partial sums of
// |q - y|^2 (the data term).
__global__ __launch_bounds__(256) void k_terminal(const double *__restrict__ q,
                                                  const float *__restrict__ y, int64_t n,
                                                  double *__restrict__ al,
                                                  double *__restrict__ be,
                                                  double *__restrict__ part) {
    __shared__ double lds[8];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = q[3 * i + c] - (double)y[3 * i + c];
            e += d * d;
            al[3 * i + c] = 2.0 * d / (double)n;
            be[3 * i + c] = 0.0;
        }
    }
    const double s = block_sum(e, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// objective = (sum of data partials) / n + lambda * (sum of energy partials)
__global__ __launch_bounds__(256) void k_objective(const double *__restrict__ dpart, int nb,
                                                   const double *__restrict__ hpart, int nh,
                                                   int64_t n, double lambda,
                                                   double *__restrict__ obj) {
    __shared__ double lds[8];
    double d = 0.0, h = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) d += dpart[b];
    for (int b = threadIdx.x; b < nh; b += blockDim.x) h += hpart[b];
    d = block_sum(d, lds);
    __syncthreads();
    h = block_sum(h, lds);
    if (threadIdx.x == 0) *obj = d / (double)n + lambda * h;
}

template <int T>
__global__ __launch_bounds__(256) void k_adj_pairs(
    const float4 *__restrict__ Q, const float4 *__restrict__ P, const float4 *__restrict__ AL,
    const float4 *__restrict__ BE, int64_t ntgt, int64_t chunk, int64_t nsrc, int splits,
    float negc, float inv_s2, double *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    // block b: target block b / splits, source split b % splits (as the
    // forward pair kernel)
    const int64_t split = blockIdx.x % splits, tb = blockIdx.x / splits;
    const int64_t wave = tb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t t0 = wave * (64 * T) + lane;
    float x[T], y[T], z[T], px[T], py[T], pz[T], ax[T], ay[T], az[T], bx[T], by[T], bz[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t i = t0 + 64 * k;
        const float4 a = Q[i], b = P[i], c = AL[i], d = BE[i];
        x[k] = a.x, y[k] = a.y, z[k] = a.z;
        px[k] = b.x, py[k] = b.y, pz[k] = b.z;
        ax[k] = c.x, ay[k] = c.y, az[k] = c.z;
        bx[k] = d.x, by[k] = d.y, bz[k] = d.z;
    }
    double sq[T][3], spp[T][3];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sq[k][c] = spp[k][c] = 0.0;
    const int64_t j0 = split * chunk;
    const int64_t j1 = j0 + chunk < nsrc ? j0 + chunk : nsrc;
    for (int64_t jt = j0; jt < j1; jt += kTile) {
        float tq[T][3], tp[T][3];
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) tq[k][c] = tp[k][c] = 0.f;
#pragma unroll 4
        for (int u = 0; u < kTile; ++u) {
            const float4 qj = Q[jt + u], pj = P[jt + u], aj = AL[jt + u], bj = BE[jt + u];
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const float dx = x[k] - qj.x, dy = y[k] - qj.y, dz = z[k] - qj.z;
                const float g = __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * negc);
                const float s = px[k] * pj.x + py[k] * pj.y + pz[k] * pj.z;
                const float pa = pj.x * ax[k] + pj.y * ay[k] + pj.z * az[k];
                const float ap = px[k] * aj.x + py[k] * aj.y + pz[k] * aj.z;
                const float dbx = bx[k] - bj.x, dby = by[k] - bj.y, dbz = bz[k] - bj.z;
                const float c2 = (dx * dbx + dy * dby + dz * dbz) * inv_s2;
                // w1 = -G ((p_j . alpha_k) + (p_k . alpha_j) + s (d . dbeta) / sigma^2)
                const float w1 = -g * fmaf(s, c2, pa + ap);
                const float w2 = g * s;
                const float w3 = g * c2;
                // each sum as two chained FMAs (written as one expression the
                // products would be added first and cost an extra add)
                tq[k][0] = fmaf(w1, dx, tq[k][0]);
                tq[k][1] = fmaf(w1, dy, tq[k][1]);
                tq[k][2] = fmaf(w1, dz, tq[k][2]);
                tq[k][0] = fmaf(w2, dbx, tq[k][0]);
                tq[k][1] = fmaf(w2, dby, tq[k][1]);
                tq[k][2] = fmaf(w2, dbz, tq[k][2]);
                tp[k][0] = fmaf(g, aj.x, tp[k][0]);
                tp[k][1] = fmaf(g, aj.y, tp[k][1]);
                tp[k][2] = fmaf(g, aj.z, tp[k][2]);
                tp[k][0] = fmaf(w3, pj.x, tp[k][0]);
                tp[k][1] = fmaf(w3, pj.y, tp[k][1]);
                tp[k][2] = fmaf(w3, pj.z, tp[k][2]);
            }
        }
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sq[k][c] += (double)tq[k][c];
                spp[k][c] += (double)tp[k][c];
            }
    }
    double *dst = part + split * 6 * ntgt;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t i = t0 + 64 * k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dst[c * ntgt + i] = sq[k][c];
            dst[(3 + c) * ntgt + i] = spp[k][c];
        }
    }
}

// (alpha, beta) += dt (sigma^-2 S_q, S_p) from the split partials.
__global__ __launch_bounds__(256) void k_adj_update(const double *__restrict__ part, int splits,
                                                    int64_t ntgt, int64_t n, double inv_s2,
                                                    double dt, double *__restrict__ al,
                                                    double *__restrict__ be) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < splits; ++s)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += part[((int64_t)s * 6 + c) * ntgt + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        al[3 * i + c] += dt * (acc[c] * inv_s2);
        be[3 * i + c] += dt * acc[3 + c];
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
AdjointBufs layout_adjoint(Arena &a, int64_t n, int nt, int ckpt, int method) {
    AdjointBufs b{};
    b.n = n;
    b.nt = nt;
    b.ckpt = ckpt;
    b.nck = (nt + ckpt - 1) / ckpt;
    b.pl = plan_exact(n, n);
    carve_exact(a, b.pl, b.ex);
    const int64_t npad = b.pl.nsrc > b.pl.ntgt ? b.pl.nsrc : b.pl.ntgt;
    b.AL = a.take<float4>(npad);
    b.BE = a.take<float4>(npad);
    b.Sq = a.take<double>(3 * n);
    b.Sp = a.take<double>(3 * n);
    b.al = a.take<double>(3 * n);
    b.be = a.take<double>(3 * n);
    b.v0 = a.take<double>(3 * n);
    b.ckq = a.take<double>((size_t)b.nck * 3 * n);
    b.ckp = a.take<double>((size_t)b.nck * 3 * n);
    b.segq = a.take<double>((size_t)ckpt * 3 * n);
    b.segp = a.take<double>((size_t)ckpt * 3 * n);
    b.nblk = combine_blocks(n);
    b.nh = b.nblk;
    if (method == GS_BH) {
        b.bh = true;
        b.sh = layout_shoot_bh(a, n, 1);
        b.bhadj = layout_bh_adjoint(a, n);
        b.nh = (int)b.sh.tree.groups;
    }
    b.hpart = a.take<double>(b.nh > b.nblk ? b.nh : b.nblk);
    b.dpart = a.take<double>(b.nblk);
    return b;
}

gs_status launch_pack2(const double *a, const double *b, int64_t n, int64_t npad, float4 *A,
                       float4 *B, hipStream_t s) {
    hipLaunchKernelGGL(k_pack2, dim3(nblk(npad)), dim3(kBlock), 0, s, a, b, n, npad, A, B);
    GS_LAUNCH_CHECK("pack2");
    return GS_OK;
}

gs_status launch_copy(const double *src, double *dst, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(nblk(count)), dim3(kBlock), 0, s, src, dst, count);
    GS_LAUNCH_CHECK("copy");
    return GS_OK;
}

// One forward Euler step of the exact flow from the FP64 state (b.Sq, b.Sp):
// refreshes the packed copies, evaluates the RHS and updates the state.
// With v0 non-null, also stores the step's velocity there and its energy
// partials in b.hpart.
static gs_status exact_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                            hipStream_t s) {
    const int64_t npad = b.pl.nsrc > b.pl.ntgt ? b.pl.nsrc : b.pl.ntgt;
    GS_TRY(launch_pack2(b.Sq, b.Sp, b.n, npad, b.ex.Q, b.ex.P, s));
    GS_TRY(launch_exact_pairs(b.pl, b.ex.Q, b.ex.P, b.ex.Q, b.ex.P, prm.sigma, true, b.ex.part,
                              s));
    return launch_combine_euler_v(b.pl, b.ex.part, prm.sigma, dt, b.Sq, b.Sp, b.ex.Q, b.ex.P,
                                  v0 ? b.hpart : nullptr, v0, s);
}

// One forward step of the chosen method from (b.Sq, b.Sp).
static gs_status forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                              char *ws, hipStream_t s) {
    if (!b.bh) return exact_step(b, prm, dt, v0, s);
    return bh_adjoint_forward_step(b, prm, dt, v0, ws, s);
}

// One backward step at state (q_t, p_t) = (sq, sp): (al, be) += dt J^T (al, be).
static gs_status adjoint_step(AdjointBufs &b, const gs_params &prm, double dt, const double *sq,
                              const double *sp, char *ws, hipStream_t s) {
    if (b.bh) return bh_adjoint_step(b, prm, dt, sq, sp, ws, s);
    const int64_t npad = b.pl.nsrc > b.pl.ntgt ? b.pl.nsrc : b.pl.ntgt;
    GS_TRY(launch_pack2(sq, sp, b.n, npad, b.ex.Q, b.ex.P, s));
    GS_TRY(launch_pack2(b.al, b.be, b.n, npad, b.AL, b.BE, s));
    const double c = kLog2e / (2.0 * prm.sigma * prm.sigma);
    const ExactPlan &pl = b.pl;
    dim3 grid((unsigned)(pl.ntgt / (64 * 4) * pl.splits));
    timing_begin(KIND_ADJOINT, s);
    hipLaunchKernelGGL(k_adj_pairs<1>, grid, dim3(256), 0, s, b.ex.Q, b.ex.P, b.AL, b.BE, pl.ntgt,
                       pl.chunk, pl.nsrc, pl.splits, (float)(-c),
                       (float)(1.0 / (prm.sigma * prm.sigma)), b.ex.part);
    timing_end(KIND_ADJOINT, s);
    GS_LAUNCH_CHECK("adj_pairs");
    hipLaunchKernelGGL(k_adj_update, dim3(nblk(b.n)), dim3(kBlock), 0, s, b.ex.part, pl.splits,
                       pl.ntgt, b.n, 1.0 / (prm.sigma * prm.sigma), dt, b.al, b.be);
    GS_LAUNCH_CHECK("adj_update");
    return GS_OK;
}

gs_status shoot_adjoint(const float *q0, const float *p0, const float *y, const gs_params &prm,
                        double lambda, double *objective, float *grad, AdjointBufs &b, char *ws,
                        hipStream_t s) {
    const int64_t n = b.n, n3 = 3 * n;
    const double dt = 1.0 / prm.nt;
    const int64_t npad = b.pl.nsrc > b.pl.ntgt ? b.pl.nsrc : b.pl.ntgt;
    if (b.bh) GS_TRY(bh_adjoint_begin(b, ws, s));
    // forward sweep with checkpoints every b.ckpt steps
    GS_TRY(launch_pack_state(q0, p0, n, npad, b.Sq, b.Sp, b.ex.Q, b.ex.P, s));
    for (int t = 0; t < prm.nt; ++t) {
        if (t % b.ckpt == 0) {
            const int c = t / b.ckpt;
            GS_TRY(launch_copy(b.Sq, b.ckq + (size_t)c * n3, n3, s));
            GS_TRY(launch_copy(b.Sp, b.ckp + (size_t)c * n3, n3, s));
        }
        GS_TRY(forward_step(b, prm, dt, t == 0 ? b.v0 : nullptr, ws, s));
    }
    // objective and terminal adjoint
    hipLaunchKernelGGL(k_terminal, dim3(nblk(n)), dim3(kBlock), 0, s, b.Sq, y, n, b.al, b.be,
                       b.dpart);
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(kBlock), 0, s, b.dpart, b.nblk, b.hpart, b.nh, n,
                       lambda, objective);
    GS_LAUNCH_CHECK("objective");
    // backward sweep, one checkpoint segment at a time
    for (int c = b.nck - 1; c >= 0; --c) {
        const int t0 = c * b.ckpt;
        const int t1 = t0 + b.ckpt < prm.nt ? t0 + b.ckpt : prm.nt;
        GS_TRY(launch_copy(b.ckq + (size_t)c * n3, b.Sq, n3, s));
        GS_TRY(launch_copy(b.ckp + (size_t)c * n3, b.Sp, n3, s));
        for (int t = t0; t < t1; ++t) {
            GS_TRY(launch_copy(b.Sq, b.segq + (size_t)(t - t0) * n3, n3, s));
            GS_TRY(launch_copy(b.Sp, b.segp + (size_t)(t - t0) * n3, n3, s));
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
