// exact.hip -- exact all-pairs right-hand side (Sec. 2.1, eq. 1 and eq. 3),
// the Euler step with the FP64 energy reduction, the velocity field of eq. 3
// at arbitrary points, and the FP64 variants.
//
// FP32 all-pairs kernel (k_exact_items):
//   * a work item is one block: kItemGroups groups of 64 consecutive target
//     rows (one target per lane) against one chunk of source rows of the same
//     point set; the chunk is split among kItemSplit waves per target group,
//     whose double-float sums are added in LDS in a fixed order and written as one
//     partial per (target, chunk); the combine kernel adds a target's
//     partials in chunk order (bitwise deterministic);
//   * sources are read with wave-uniform addresses, so they arrive through
//     the scalar data cache straight into SGPRs; the next group of 4 is
//     loaded while the current one is evaluated;
//   * positions are stored as k (q - c) with k = sqrt(log2(e) / (2 sigma^2))
//     and c the FP64 centre of the point set's box: G = exp2(-|d'|^2) needs
//     no scaling multiply, and the FP32 rounding of a stored position is
//     relative to the set's extent, not to its distance from the origin, so
//     the accuracy does not depend on where the set lies (the method depends
//     only on differences q_i - q_j);
//   * per pair 16 VALU operations and one v_exp_f32; each tile of kTile
//     sources is summed in FP32 and the tile sums are accumulated with
//     Kahan's compensation in FP32, and the partials and their sum are kept
//     as double-float (hi, lo) pairs, so a target's rounding error grows with
//     the tile length, not with N; FP64 serves only the energy reduction (and
//     the backward stage's own state).
//   * a shooting keeps its state as FP32 hi+lo pairs and takes the Euler step
//     in double-float arithmetic.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace gs {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

__device__ inline double block_sum_f64(double v, double *lds) {
    // Fixed reduction tree: wave shuffle, then the per-wave sums in order.
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

// ---------------------------------------------------------------- set centres
// Box of the points of row block b (min / max of its finite coordinates).
__global__ __launch_bounds__(256) void k_box_rows(const float *__restrict__ q,
                                                  const int4 *__restrict__ blk, RowGeom rg,
                                                  float *__restrict__ bpart) {
    __shared__ float red[6][256];
    const int4 d = row_block(blk, rg, blockIdx.x);
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = q[3 * i + c];
            if (isfinite(x)) {
                lo[c] = x;
                hi[c] = x;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = lo[c];
        red[3 + c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fminf(red[c][threadIdx.x], red[c][threadIdx.x + s]);
                red[3 + c][threadIdx.x] =
                    fmaxf(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) bpart[(int64_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Centre (lo + hi) / 2 in FP64 of every set from its row blocks' boxes; one
// wave per set; 0 for a set without finite points.
__global__ __launch_bounds__(64) void k_box_sets(const float *__restrict__ bpart,
                                                 const int *__restrict__ bseg, int nblk,
                                                 double *__restrict__ cen,
                                                 float2 *__restrict__ cenf) {
    const int lane = threadIdx.x, set = blockIdx.x;
    const int b0 = bseg ? bseg[set] : 0, b1 = bseg ? bseg[set + 1] : nblk;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = b0 + lane; b < b1; b += 64)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], bpart[6 * (int64_t)b + c]);
            hi[c] = fmaxf(hi[c], bpart[6 * (int64_t)b + 3 + c]);
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], off, 64));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], off, 64));
        }
    if (lane < 3) {
        const float l = lane == 0 ? lo[0] : (lane == 1 ? lo[1] : lo[2]);
        const float h = lane == 0 ? hi[0] : (lane == 1 ? hi[1] : hi[2]);
        const double c = l <= h ? 0.5 * ((double)l + (double)h) : 0.0;
        cen[3 * set + lane] = c;
        const float ch = (float)c;
        cenf[3 * set + lane] = make_float2(ch, (float)(c - (double)ch));  // exact split
    }
}

// ---------------------------------------------------------------- packing
// Row block b of the rows is row_block(b) = (first real point, real rows in
// it, set, partial slots of the set); real point i of the block sits at row
// 256 b + (i - first).  Padding rows get zero position and momentum, so a
// padded source adds exactly zero and a padded target is never read back.

// FP32 source (and target) rows k (q - c_set), p; with Sq non-null also the
// FP64 state copy of (q, p).
// With Fq non-null also the hi+lo state ((hi, lo) = (the input, 0)).
__global__ __launch_bounds__(256) void k_pack_state_rows(const float *__restrict__ q,
                                                         const float *__restrict__ p,
                                                         const int4 *__restrict__ blk, RowGeom rg,
                                                         double ks, const double *__restrict__ cen,
                                                         double *__restrict__ Sq,
                                                         double *__restrict__ Sp,
                                                         float2 *__restrict__ Fq,
                                                         float2 *__restrict__ Fp,
                                                         float4 *__restrict__ Q,
                                                         float4 *__restrict__ P) {
    const int4 d = row_block(blk, rg, blockIdx.x);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        const double *c = cen + 3 * d.z;
        const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
        const float u = p[3 * i], v = p[3 * i + 1], w = p[3 * i + 2];
        if (Fq) {
            const float qs[3] = {x, y, z}, ps[3] = {u, v, w};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Fq[3 * i + k] = make_float2(qs[k], 0.f);
                Fp[3 * i + k] = make_float2(ps[k], 0.f);
            }
        }
        if (Sq) {
            Sq[3 * i] = x;
            Sq[3 * i + 1] = y;
            Sq[3 * i + 2] = z;
            Sp[3 * i] = u;
            Sp[3 * i + 1] = v;
            Sp[3 * i + 2] = w;
        }
        Q[row] = make_float4((float)(ks * ((double)x - c[0])), (float)(ks * ((double)y - c[1])),
                             (float)(ks * ((double)z - c[2])), 0.f);
        P[row] = make_float4(u, v, w, 0.f);
    } else {
        Q[row] = make_float4(0.f, 0.f, 0.f, 0.f);
        P[row] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// FP32 target rows k (x - c) of the velocity field (positions only).
__global__ __launch_bounds__(256) void k_pack_pos_rows(const float *__restrict__ x,
                                                       const int4 *__restrict__ blk, RowGeom rg,
                                                       double ks, const double *__restrict__ cen,
                                                       float4 *__restrict__ X) {
    const int4 d = row_block(blk, rg, blockIdx.x);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        X[row] = make_float4((float)(ks * ((double)x[3 * i] - cen[0])),
                             (float)(ks * ((double)x[3 * i + 1] - cen[1])),
                             (float)(ks * ((double)x[3 * i + 2] - cen[2])), 0.f);
    } else {
        X[row] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// FP64 [n][3] pair (a, b) -> packed FP32 rows (sa (a - c_set), sb b); the
// centre is subtracted only when cen is non-null (positions).
__global__ __launch_bounds__(256) void k_pack_rows64(const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     const int4 *__restrict__ blk, RowGeom rg,
                                                     double sa, double sb,
                                                     const double *__restrict__ cen,
                                                     float4 *__restrict__ A,
                                                     float4 *__restrict__ B) {
    const int4 d = row_block(blk, rg, blockIdx.x);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        const double c0 = cen ? cen[3 * d.z] : 0.0, c1 = cen ? cen[3 * d.z + 1] : 0.0,
                     c2 = cen ? cen[3 * d.z + 2] : 0.0;
        A[row] = make_float4((float)(sa * (a[3 * i] - c0)), (float)(sa * (a[3 * i + 1] - c1)),
                             (float)(sa * (a[3 * i + 2] - c2)), 0.f);
        B[row] = make_float4((float)(sb * b[3 * i]), (float)(sb * b[3 * i + 1]),
                             (float)(sb * b[3 * i + 2]), 0.f);
    } else {
        A[row] = make_float4(0.f, 0.f, 0.f, 0.f);
        B[row] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// q = hi + lo of the hi+lo state, rounded to FP32.
__global__ void k_unpack_state(const float2 *__restrict__ Fq, const float2 *__restrict__ Fp,
                               int64_t n, float *__restrict__ q, float *__restrict__ p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    q[i] = Fq[i].x + Fq[i].y;
    p[i] = Fp[i].x + Fp[i].y;
}

// ---------------------------------------------------------------- pair kernel
// Work item b = (first target row, source rows [j0, j1) of the same set,
// partial slot).  Wave (group g, split w) takes targets it.x + 64 g + lane and
// the w-th share (whole tiles) of the chunk.  Qt holds the target rows (the
// source rows themselves for a right-hand side), Q / P the source rows.
//
// The sources of the next group of four are loaded while the current four
// are evaluated (software pipelining through SGPRs): without it every group
// waits for its own loads.  With at most 64 VGPRs (8 waves per SIMD) the loop
// measured 13.3 ms per 200k right-hand side, against 14.4 ms for groups of
// eight loaded and then evaluated (7 waves per SIMD).
template <bool WITH_A>
__global__ __launch_bounds__(kItemThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_exact_items(const float4 *__restrict__ Qt, const float4 *__restrict__ Q,
              const float4 *__restrict__ P, int64_t npad, const int4 *__restrict__ items,
              ItemGeom geom, float2 *__restrict__ part) {
    constexpr int B = 4;  // sources per pipeline stage (kTile is a multiple)
    constexpr int NV = WITH_A ? 6 : 3;
    __shared__ float2 red[kItemSplit > 1 ? kItemSplit - 1 : 1][NV][kItemRows];
    const int4 it = work_item(items, geom, blockIdx.x);
    if (it.w < 0) return;  // padding item: the whole block leaves before any barrier
    const int wv = wave_in_block();
    const int grp = wv % kItemGroups, w = wv / kItemGroups;
    const int r = grp * 64 + (threadIdx.x & 63);
    const int64_t t0 = (int64_t)it.x + r;
    const float4 a = Qt[t0];
    const float x = a.x, y = a.y, z = a.z;
    float px = 0.f, py = 0.f, pz = 0.f;
    if (WITH_A) {
        const float4 b = P[t0];
        px = b.x;
        py = b.y;
        pz = b.z;
    }
    // compensated sums of the tile sums: value = s - c
    float sv[3] = {0.f, 0.f, 0.f}, cv[3] = {0.f, 0.f, 0.f};
    float sa[3] = {0.f, 0.f, 0.f}, ca[3] = {0.f, 0.f, 0.f};
    // this wave's share of the chunk in whole tiles; 32-bit source indices, so
    // the loop and prefetch-clamp compares run on the scalar unit
    const int ntile = (it.z - it.y) / kTile;
    const int per = (ntile + kItemSplit - 1) / kItemSplit;
    const int j0 = it.y + min(w * per, ntile) * kTile;
    const int j1 = it.y + min((w + 1) * per, ntile) * kTile;
    if (j0 < j1) {
        float4 qn[B], pn[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            qn[b] = Q[j0 + b];
            pn[b] = P[j0 + b];
        }
        for (int jt = j0; jt < j1; jt += kTile) {
            float tv[3] = {0.f, 0.f, 0.f}, ta[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
            for (int u = 0; u < kTile; u += B) {
                float4 qj[B], pj[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    qj[b] = qn[b];
                    pj[b] = pn[b];
                }
                // next group (the last group reloads itself: j1 - j0 >= kTile >= B)
                int jn = jt + u + B;
                jn = jn < j1 - B ? jn : j1 - B;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    qn[b] = Q[jn + b];
                    pn[b] = P[jn + b];
                }
                float dx[B], dy[B], dz[B], g[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    dx[b] = x - qj[b].x;
                    dy[b] = y - qj[b].y;
                    dz[b] = z - qj[b].z;
                }
#pragma unroll
                for (int b = 0; b < B; ++b)
                    g[b] =
                        __builtin_amdgcn_exp2f(-(dx[b] * dx[b] + dy[b] * dy[b] + dz[b] * dz[b]));
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    tv[0] += g[b] * pj[b].x;
                    tv[1] += g[b] * pj[b].y;
                    tv[2] += g[b] * pj[b].z;
                    if (WITH_A) {
                        const float wgt = g[b] * (px * pj[b].x + py * pj[b].y + pz * pj[b].z);
                        ta[0] += wgt * dx[b];
                        ta[1] += wgt * dy[b];
                        ta[2] += wgt * dz[b];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                kahan_add(sv[c], cv[c], tv[c]);
                if (WITH_A) kahan_add(sa[c], ca[c], ta[c]);
            }
        }
    }
    // as double-float values; the waves of a target group add theirs in
    // split order
    ff xv[3], xa[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xv[c] = ff_fast_two_sum(sv[c], -cv[c]);
        xa[c] = ff_fast_two_sum(sa[c], -ca[c]);
    }
    if (kItemSplit > 1) {
        if (w > 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[w - 1][c][r] = make_float2(xv[c].h, xv[c].l);
                if (WITH_A) red[w - 1][3 + c][r] = make_float2(xa[c].h, xa[c].l);
            }
        __syncthreads();
        if (w == 0)
            for (int k = 0; k < kItemSplit - 1; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 u = red[k][c][r];
                    xv[c] = ff_add(xv[c], ff{u.x, u.y});
                    if (WITH_A) {
                        const float2 e = red[k][3 + c][r];
                        xa[c] = ff_add(xa[c], ff{e.x, e.y});
                    }
                }
    }
    if (w != 0) return;
    float2 *dst = part + (int64_t)it.w * 6 * npad;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dst[c * npad + t0] = make_float2(xv[c].h, xv[c].l);
        if (WITH_A) dst[(3 + c) * npad + t0] = make_float2(xa[c].h, xa[c].l);
    }
}

// Constants of the combine kernel: 1 / (k sigma^2) (the a-sums were taken on
// scaled positions), k and dt, in FP64 for the FP64 state and as
// double-float for the hi+lo state.
struct CombineConst {
    double inv_s2, ks, dt;
    ff inv_s2f, ksf, dtf;
};

// Sums the partial slots of each row (double-float, in slot order).  mode 0:
// (dq, dp) = (v, a) (dp nullable: velocity field).  mode 1: energy partial of
// the block into Hpart (nullable; FP64, the energy reduction), the velocity
// into vout (FP64 [n][3], nullable) and, if dt > 0, the Euler step of the
// state and its packed copies: the hi+lo state (Fq, Fp) in double-float
// arithmetic when Fq is non-null, else the FP64 state (Sq, Sp) of the
// backward stage.  A slot's components are loaded together before they are
// added (the loop bounds are fixed, so acc stays in registers).
__global__ __launch_bounds__(256) void k_combine_rows(
    const float2 *__restrict__ part, int64_t npad, const int4 *__restrict__ blk, RowGeom rg,
    CombineConst k, int mode, float *__restrict__ dq, float *__restrict__ dp,
    double *__restrict__ Sq, double *__restrict__ Sp, float2 *__restrict__ Fq,
    float2 *__restrict__ Fp, float4 *__restrict__ Q, float4 *__restrict__ P,
    const double *__restrict__ cen, const float2 *__restrict__ cenf, double *__restrict__ Hpart,
    double *__restrict__ vout) {
    __shared__ double lds[8];
    const int4 d = row_block(blk, rg, blockIdx.x);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        ff acc[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] = ff{0.f, 0.f};
        const bool with_a = !(mode == 0 && !dp);
        for (int s = 0; s < d.w; ++s) {
            float2 u[6];
#pragma unroll
            for (int c = 0; c < 6; ++c)
                u[c] = (c < 3 || with_a) ? part[((int64_t)s * 6 + c) * npad + row]
                                         : make_float2(0.f, 0.f);
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] = ff_add(acc[c], ff{u[c].x, u[c].y});
        }
        if (mode == 0) {  // right-hand side or velocity field
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dq[3 * i + c] = acc[c].h + acc[c].l;
                if (dp) {
                    const ff a = ff_mul(acc[3 + c], k.inv_s2f);
                    dp[3 * i + c] = a.h + a.l;
                }
            }
        } else if (Fq) {  // shooting: hi+lo state
            ff q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float2 fq = Fq[3 * i + c], fp = Fp[3 * i + c];
                q[c] = ff{fq.x, fq.y};
                p[c] = ff{fp.x, fp.y};
                e += ((double)p[c].h + (double)p[c].l) * ((double)acc[c].h + (double)acc[c].l);
                if (vout) vout[3 * i + c] = (double)acc[c].h + (double)acc[c].l;
            }
            if (k.dt > 0.0) {
                const float2 *c0 = cenf + 3 * d.z;
                float xq[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] = ff_add(q[c], ff_mul(k.dtf, acc[c]));
                    p[c] = ff_add(p[c], ff_mul(k.dtf, ff_mul(acc[3 + c], k.inv_s2f)));
                    Fq[3 * i + c] = make_float2(q[c].h, q[c].l);
                    Fp[3 * i + c] = make_float2(p[c].h, p[c].l);
                    const ff r = ff_mul(k.ksf, ff_add(q[c], ff{-c0[c].x, -c0[c].y}));
                    xq[c] = r.h + r.l;
                }
                Q[row] = make_float4(xq[0], xq[1], xq[2], 0.f);
                P[row] = make_float4(p[0].h + p[0].l, p[1].h + p[1].l, p[2].h + p[2].l, 0.f);
            }
        } else {  // the backward stage's forward steps: FP64 state
            double v[3], a[3], q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c] = (double)acc[c].h + (double)acc[c].l;
                a[c] = ((double)acc[3 + c].h + (double)acc[3 + c].l) * k.inv_s2;
                q[c] = Sq[3 * i + c];
                p[c] = Sp[3 * i + c];
            }
            e = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
            if (vout)
#pragma unroll
                for (int c = 0; c < 3; ++c) vout[3 * i + c] = v[c];
            if (k.dt > 0.0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] += k.dt * v[c];
                    p[c] += k.dt * a[c];
                    Sq[3 * i + c] = q[c];
                    Sp[3 * i + c] = p[c];
                }
                const double *c0 = cen + 3 * d.z;
                Q[row] = make_float4((float)(k.ks * (q[0] - c0[0])), (float)(k.ks * (q[1] - c0[1])),
                                     (float)(k.ks * (q[2] - c0[2])), 0.f);
                P[row] = make_float4((float)p[0], (float)p[1], (float)p[2], 0.f);
            }
        }
    }
    if (Hpart) {
        const double s = block_sum_f64(e, lds);
        if (threadIdx.x == 0) Hpart[blockIdx.x] = s;
    }
}

// H[set * count + t] = sum of Hpart[t * stride + b] over the partials b of
// the set (seg[set] <= b < seg[set + 1]; all of [0, stride) when seg is
// null).  grid (count, sets).
__global__ __launch_bounds__(256) void k_reduce_h(const double *__restrict__ Hpart,
                                                  int64_t stride, const int *__restrict__ seg,
                                                  int count, double *__restrict__ H) {
    __shared__ double lds[8];
    const int t = blockIdx.x, set = blockIdx.y;
    const int64_t lo = seg ? seg[set] : 0, hi = seg ? seg[set + 1] : stride;
    double s = 0.0;
    for (int64_t b = lo + threadIdx.x; b < hi; b += blockDim.x) s += Hpart[(int64_t)t * stride + b];
    s = block_sum_f64(s, lds);
    if (threadIdx.x == 0) H[(int64_t)set * count + t] = s;
}

// ---------------------------------------------------------------- FP64 path
// Differences of FP64 positions lose nothing that matters at any offset of
// the set (2^-53 relative), so this path works on the inputs as they are.
template <bool WITH_A>
__global__ __launch_bounds__(256) void k_exact_f64(const double *__restrict__ q,
                                                   const double *__restrict__ p, int64_t n,
                                                   double sigma, double *__restrict__ v,
                                                   double *__restrict__ a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    const int64_t ii = live ? i : 0;
    const double xi = q[3 * ii], yi = q[3 * ii + 1], zi = q[3 * ii + 2];
    const double pxi = p[3 * ii], pyi = p[3 * ii + 1], pzi = p[3 * ii + 2];
    const double m = -1.0 / (2.0 * sigma * sigma);
    double vx = 0, vy = 0, vz = 0, ax = 0, ay = 0, az = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double dx = xi - q[3 * j], dy = yi - q[3 * j + 1], dz = zi - q[3 * j + 2];
        const double g = exp((dx * dx + dy * dy + dz * dz) * m);
        const double pjx = p[3 * j], pjy = p[3 * j + 1], pjz = p[3 * j + 2];
        vx += g * pjx;
        vy += g * pjy;
        vz += g * pjz;
        if (WITH_A) {
            const double w = g * (pxi * pjx + pyi * pjy + pzi * pjz);
            ax += w * dx;
            ay += w * dy;
            az += w * dz;
        }
    }
    if (!live) return;
    v[3 * i] = vx;
    v[3 * i + 1] = vy;
    v[3 * i + 2] = vz;
    if (WITH_A) {
        const double inv = 1.0 / (sigma * sigma);
        a[3 * i] = ax * inv;
        a[3 * i + 1] = ay * inv;
        a[3 * i + 2] = az * inv;
    }
}

__global__ __launch_bounds__(256) void k_euler_f64(double *__restrict__ q, double *__restrict__ p,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ a, int64_t n,
                                                   double dt, double *__restrict__ Hpart) {
    __shared__ double lds[8];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        e = p[3 * i] * v[3 * i] + p[3 * i + 1] * v[3 * i + 1] + p[3 * i + 2] * v[3 * i + 2];
        if (dt > 0.0)
            for (int c = 0; c < 3; ++c) {
                q[3 * i + c] += dt * v[3 * i + c];
                p[3 * i + c] += dt * a[3 * i + c];
            }
    }
    if (Hpart) {
        double s = block_sum_f64(e, lds);
        if (threadIdx.x == 0) Hpart[blockIdx.x] = s;
    }
}

__global__ void k_copy_f64(const double *__restrict__ s, double *__restrict__ d, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) d[i] = s[i];
}

inline unsigned nblocks(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- planning
// Chunk length of a launch: about `items` work items of kItemRows targets
// (kItemsDefault unless the caller chose), never below kMinWaveSources
// sources per wave nor, for the default target, above kMaxChunk sources (4 MB
// of packed rows, one XCD's L2: 400k / 500k points in 2 chunks of 200k / 250k
// took 52.8 / 83.8 ms per RHS against 51.8 / 81.4 ms in 4).  A caller's
// target is followed as given (the static-workspace entry lowers it until
// the partial sums fit its array).  Small sets need short chunks to fill the GPU: one RHS of
// 5000 / 20 000 points took 0.119 / 0.308 ms with chunks of at least 2048
// sources, 0.025 / 0.152 ms with at least 256.
constexpr int64_t kMaxChunk = 131072;

static int64_t chunk_for(int64_t work_rows_x_sources, int64_t items, bool *at_min = nullptr) {
    const int64_t target = items > 0 ? items : kItemsDefault;
    int64_t chunk = round_up((work_rows_x_sources + kItemRows * target - 1) / (kItemRows * target),
                             kTile);
    const int64_t minc = (int64_t)kMinWaveSources * kItemSplit;
    if (at_min) *at_min = chunk <= minc;
    if (items <= 0 && chunk > kMaxChunk) chunk = kMaxChunk;
    return chunk < minc ? minc : chunk;
}

// XCDs sharing each of nch < kXcds chunks, and nch rounded up to a power of
// two: chunk c's homes are c + pw r, r < rep (all XCDs busy for 1, 2, 4
// chunks).
static void chunk_homes(int nch, int &pw, int &rep) {
    pw = 1;
    while (pw < nch) pw *= 2;
    rep = nch >= kXcds ? 1 : kXcds / pw;
}

ItemGeom item_geom(int64_t n, int64_t items) {
    ItemGeom g{};
    g.n = (int)n;
    g.ng = (int)((n + kItemRows - 1) / kItemRows);
    g.sp = (int)round_up(n > 0 ? n : 1, kTile);
    bool at_min = false;
    const int64_t chunk = chunk_for((int64_t)g.ng * kItemRows * g.sp, items, &at_min);
    int nch = (int)((g.sp + chunk - 1) / chunk);
    // fewer chunks than XCDs: a power of two of them, each shared by
    // kXcds / nch XCDs (400k / 500k points: 51.6 / 80.9 ms per RHS against
    // 101.8 / 159.6 ms with 4 chunks on 4 XCDs), unless the chunks are at
    // their minimum length (small sets: more chunks mean more items)
    if (nch < kXcds && !at_min) {
        int p2 = 1;
        while (p2 * 2 <= nch) p2 *= 2;
        nch = items > 0 || (g.sp + p2 - 1) / p2 <= kMaxChunk ? p2 : 2 * p2;
    }
    g.csz = (int)round_up((g.sp + nch - 1) / nch, kTile);
    g.nch = (g.sp + g.csz - 1) / g.csz;
    chunk_homes(g.nch, g.pw, g.rep);
    g.gpp = (g.ng + g.rep - 1) / g.rep;
    g.qlen = g.rep > 1 ? g.gpp : ((g.nch + kXcds - 1) / kXcds) * g.ng;  // XCD 0's queue is the longest
    return g;
}

RowGeom row_geom(int64_t n, int slots) {
    RowGeom r{};
    r.n = (int)n;
    r.slots = slots;
    return r;
}

// Work items of point sets (targets and sources of set s: rows
// [tbase_s, tbase_s + tn_s) of the target rows and [sbase_s, sbase_s + sn_s)
// of the source rows).  Every source chunk gets a home XCD (the largest
// chunks first, each to the least loaded XCD), so that an XCD streams only
// its own chunks and they stay in its L2; with fewer chunks than XCDs a
// chunk's target groups are shared out among several homes.  Workgroups are dealt to the 8
// XCDs in turn, so item i of the launch runs on XCD i % 8: the launch
// interleaves the 8 queues, largest items first in each, and pads a short
// queue with empty items (slot -1) to keep the interleave aligned.
static void plan_items(const std::vector<int64_t> &tn, const std::vector<int64_t> &sn,
                       const std::vector<int64_t> &tbase, const std::vector<int64_t> &sbase,
                       int64_t items, std::vector<int> &nch_out, ExactBatchPlan &pl) {
    const size_t ns = tn.size();
    int64_t work = 0;
    for (size_t s = 0; s < ns; ++s)
        if (tn[s] > 0 && sn[s] > 0)
            work += round_up(tn[s], kItemRows) * round_up(sn[s], kTile);
    const int64_t chunk = chunk_for(work, items);
    struct Chunk {
        int set, c;
        int64_t j0, j1, work;
    };
    std::vector<Chunk> chunks;
    nch_out.assign(ns, 0);
    pl.max_chunks = 1;
    for (size_t s = 0; s < ns; ++s) {
        if (tn[s] == 0 || sn[s] == 0) continue;
        const int64_t sp = round_up(sn[s], kTile);
        int nch = (int)((sp + chunk - 1) / chunk);
        const int64_t csz = round_up((sp + nch - 1) / nch, kTile);
        nch = (int)((sp + csz - 1) / csz);
        nch_out[s] = nch;
        if (nch > pl.max_chunks) pl.max_chunks = nch;
        const int64_t tr = round_up(tn[s], kItemRows);
        for (int c = 0; c < nch; ++c) {
            const int64_t j0 = sbase[s] + c * csz;
            const int64_t j1 = std::min(j0 + csz, sbase[s] + sp);
            chunks.push_back({(int)s, c, j0, j1, tr * (j1 - j0)});
        }
    }
    // fewer chunks than XCDs: each chunk's target groups are split into
    // pieces for several XCDs, so that every XCD has work
    int pw = 1, rep = 1;
    if (!chunks.empty()) chunk_homes((int)chunks.size(), pw, rep);
    struct Piece {
        int chunk;
        int64_t g0, g1, work;
    };
    std::vector<Piece> pieces;
    for (size_t k = 0; k < chunks.size(); ++k) {
        const Chunk &ch = chunks[k];
        const int64_t groups = (tn[ch.set] + kItemRows - 1) / kItemRows;
        const int64_t per = (groups + rep - 1) / rep;
        for (int64_t g0 = 0; g0 < groups; g0 += per) {
            const int64_t g1 = std::min(groups, g0 + per);
            pieces.push_back({(int)k, g0, g1, (g1 - g0) * kItemRows * (ch.j1 - ch.j0)});
        }
    }
    std::vector<int> order(pieces.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pieces[a].work > pieces[b].work; });
    int64_t load[kXcds] = {};
    struct Item {
        int64_t cost;
        int4 it;
    };
    std::vector<Item> queue[kXcds];
    for (int k : order) {
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
            if (load[y] < load[x]) x = y;
        const Piece &pc = pieces[k];
        const Chunk &ch = chunks[pc.chunk];
        load[x] += pc.work;
        for (int64_t g = pc.g0; g < pc.g1; ++g)
            queue[x].push_back({ch.j1 - ch.j0, make_int4((int)(tbase[ch.set] + kItemRows * g),
                                                         (int)ch.j0, (int)ch.j1, ch.c)});
    }
    size_t longest = 0;
    for (int x = 0; x < kXcds; ++x) {
        std::stable_sort(queue[x].begin(), queue[x].end(),
                         [](const Item &a, const Item &b) { return a.cost > b.cost; });
        longest = std::max(longest, queue[x].size());
    }
    pl.items.clear();
    pl.items.reserve(longest * kXcds);
    for (size_t i = 0; i < longest; ++i)
        for (int x = 0; x < kXcds; ++x)
            pl.items.push_back(i < queue[x].size() ? queue[x][i].it : make_int4(0, 0, 0, -1));
    while (!pl.items.empty() && pl.items.back().w < 0) pl.items.pop_back();
}

ExactBatchPlan plan_exact_batch(const int64_t *offsets, int nsub, int64_t items) {
    ExactBatchPlan pl{};
    pl.nsub = nsub;
    pl.ntot = offsets[nsub];
    pl.nsrc = pl.ntot;
    std::vector<int64_t> tn(nsub), base(nsub);
    int64_t rows = 0;
    for (int s = 0; s < nsub; ++s) {
        tn[s] = offsets[s + 1] - offsets[s];
        base[s] = rows;
        rows += round_up(tn[s], 256);
    }
    pl.npad = rows > 0 ? rows : 256;
    pl.spad = pl.npad;
    std::vector<int> nch;
    plan_items(tn, tn, base, base, items, nch, pl);
    pl.bseg.resize(nsub + 1);
    for (int s = 0; s < nsub; ++s) {
        pl.bseg[s] = (int)pl.blocks.size();
        for (int64_t b = 0; b * 256 < tn[s]; ++b)
            pl.blocks.push_back(make_int4((int)(offsets[s] + 256 * b),
                                          (int)std::min<int64_t>(256, tn[s] - 256 * b), s,
                                          std::max(nch[s], 1)));
    }
    pl.bseg[nsub] = (int)pl.blocks.size();
    return pl;
}

void carve_exact_batch(Arena &a, const ExactBatchPlan &pl, int nt, int state,
                       ExactBatchBufs &b) {
    b.Q = a.take<float4>(pl.spad);
    b.P = a.take<float4>(pl.spad);
    b.X = b.Q;
    b.part = a.take<float2>((size_t)pl.max_chunks * 6 * pl.npad);
    const int64_t n = pl.ntot > 0 ? pl.ntot : 1;
    b.Fq = b.Fp = nullptr;
    b.Sq = b.Sp = nullptr;
    if (state == kStateFF) {
        b.Fq = a.take<float2>(3 * n);
        b.Fp = a.take<float2>(3 * n);
    } else if (state == kStateF64) {
        b.Sq = a.take<double>(3 * n);
        b.Sp = a.take<double>(3 * n);
    }
    const size_t nb = (size_t)std::max<int64_t>(plan_block_count(pl), 1);
    b.Hpart = a.take<double>((size_t)(nt + 1) * nb);
    b.bpart = a.take<float>(6 * nb);
    b.cen = a.take<double>(3 * (size_t)std::max(pl.nsub, 1));
    b.cenf = a.take<float2>(3 * (size_t)std::max(pl.nsub, 1));
}

// One set without tables: the same items, row blocks and centres as
// plan_exact_batch of {0, n} gives, computed from the geometry in the kernels.
ExactBatchPlan plan_exact_single(int64_t n, int64_t items) {
    ExactBatchPlan pl{};
    pl.nsub = 1;
    pl.ntot = n;
    pl.nsrc = n;
    pl.npad = round_up(n > 0 ? n : 1, 256);
    pl.spad = pl.npad;
    pl.single = true;
    pl.geom = item_geom(n, items);
    pl.rows = row_geom(n, pl.geom.nch);
    pl.max_chunks = pl.geom.nch;
    pl.nitems = (int64_t)kXcds * pl.geom.qlen;
    pl.nblocks = (n + 255) / 256;
    return pl;
}

// Velocity field: m targets against n sources (one set each side).
ExactBatchPlan plan_exact_field(int64_t m, int64_t n, int64_t items) {
    ExactBatchPlan pl{};
    pl.nsub = 1;
    pl.ntot = m;
    pl.nsrc = n;
    pl.npad = round_up(m > 0 ? m : 1, 256);
    pl.spad = round_up(n > 0 ? n : 1, 256);
    pl.field = true;
    std::vector<int64_t> tn{m}, sn{n}, zero{0};
    std::vector<int> nch;
    plan_items(tn, sn, zero, zero, items, nch, pl);
    const int slots = std::max(nch[0], 1);
    for (int64_t b = 0; b * 256 < m; ++b)
        pl.blocks.push_back(make_int4((int)(256 * b), (int)std::min<int64_t>(256, m - 256 * b), 0,
                                      slots));
    pl.bseg = {0, (int)pl.blocks.size()};
    for (int64_t b = 0; b * 256 < n; ++b)
        pl.sblocks.push_back(
            make_int4((int)(256 * b), (int)std::min<int64_t>(256, n - 256 * b), 0, 0));
    pl.sbseg = {0, (int)pl.sblocks.size()};
    return pl;
}

void carve_exact_field(Arena &a, const ExactBatchPlan &pl, ExactBatchBufs &b) {
    b.Q = a.take<float4>(pl.spad);
    b.P = a.take<float4>(pl.spad);
    b.X = a.take<float4>(pl.npad);
    b.part = a.take<float2>((size_t)pl.max_chunks * 6 * pl.npad);
    b.Sq = b.Sp = nullptr;
    b.Fq = b.Fp = nullptr;
    b.Hpart = nullptr;
    b.bpart = a.take<float>(6 * std::max<size_t>(pl.sblocks.size(), 1));
    b.cen = a.take<double>(3);
    b.cenf = a.take<float2>(3);
}

// k = sqrt(log2(e) / (2 sigma^2)): the items kernel works on k (q - c).
double position_scale(double sigma) { return sqrt(kLog2e / (2.0 * sigma * sigma)); }

int64_t plan_item_count(const ExactBatchPlan &pl) {
    return pl.single ? pl.nitems : (int64_t)pl.items.size();
}
int64_t plan_block_count(const ExactBatchPlan &pl) {
    return pl.single ? pl.nblocks : (int64_t)pl.blocks.size();
}

// ---------------------------------------------------------------- launchers
gs_status launch_set_centres(const ExactBatchPlan &pl, const ExactBatchBufs &b, const float *q,
                             hipStream_t s) {
    // the source rows' boxes: row blocks of the sets (sblocks for the field)
    const bool fld = pl.field;
    const int64_t nb = fld ? (int64_t)pl.sblocks.size() : plan_block_count(pl);
    if (nb == 0) return GS_OK;
    const int4 *blk = fld ? b.sblk : b.blk;
    const int *bseg = fld ? b.sbseg : b.bseg;
    hipLaunchKernelGGL(k_box_rows, dim3((unsigned)nb), dim3(256), 0, s, q, blk, pl.rows, b.bpart);
    hipLaunchKernelGGL(k_box_sets, dim3((unsigned)pl.nsub), dim3(64), 0, s, b.bpart, bseg, (int)nb,
                       b.cen, b.cenf);
    GS_LAUNCH_CHECK("set_centres");
    return GS_OK;
}

gs_status launch_pack_rows64(const ExactBatchPlan &pl, const ExactBatchBufs &b, const double *a,
                             const double *bb, double sa, float4 *A, float4 *B, hipStream_t s,
                             double sb, bool centre) {
    const int64_t nb = plan_block_count(pl);
    if (nb == 0) return GS_OK;
    hipLaunchKernelGGL(k_pack_rows64, dim3((unsigned)nb), dim3(256), 0, s, a, bb, b.blk, pl.rows,
                       sa, sb, centre ? b.cen : nullptr, A, B);
    GS_LAUNCH_CHECK("pack_rows64");
    return GS_OK;
}

gs_status launch_pack_state_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b,
                                 const float *q, const float *p, double sigma, hipStream_t s) {
    const int64_t nb = plan_block_count(pl);
    if (nb == 0) return GS_OK;
    GS_TRY(launch_set_centres(pl, b, q, s));
    hipLaunchKernelGGL(k_pack_state_rows, dim3((unsigned)nb), dim3(256), 0, s, q, p, b.blk,
                       pl.rows, position_scale(sigma), b.cen, b.Sq, b.Sp, b.Fq, b.Fp, b.Q, b.P);
    GS_LAUNCH_CHECK("pack_state_rows");
    return GS_OK;
}

gs_status launch_pack_field(const ExactBatchPlan &pl, const ExactBatchBufs &b, const float *x,
                            const float *q, const float *p, double sigma, hipStream_t s) {
    GS_TRY(launch_set_centres(pl, b, q, s));
    const double ks = position_scale(sigma);
    const RowGeom none{};
    hipLaunchKernelGGL(k_pack_state_rows, dim3((unsigned)pl.sblocks.size()), dim3(256), 0, s, q,
                       p, b.sblk, none, ks, b.cen, nullptr, nullptr, nullptr, nullptr, b.Q, b.P);
    hipLaunchKernelGGL(k_pack_pos_rows, dim3((unsigned)pl.blocks.size()), dim3(256), 0, s, x,
                       b.blk, none, ks, b.cen, b.X);
    GS_LAUNCH_CHECK("pack_field");
    return GS_OK;
}

gs_status launch_exact_items(const ExactBatchPlan &pl, const ExactBatchBufs &b, bool with_a,
                             hipStream_t s) {
    const int64_t ni = plan_item_count(pl);
    if (ni == 0) return GS_OK;
    const int kind = with_a ? KIND_EXACT : KIND_EXACT_V;
    const int4 *items = pl.single ? nullptr : b.items;
    timing_begin(kind, s);
    if (with_a)
        hipLaunchKernelGGL(k_exact_items<true>, dim3((unsigned)ni), dim3(kItemThreads), 0, s, b.X,
                           b.Q, b.P, pl.npad, items, pl.geom, b.part);
    else
        hipLaunchKernelGGL(k_exact_items<false>, dim3((unsigned)ni), dim3(kItemThreads), 0, s,
                           b.X, b.Q, b.P, pl.npad, items, pl.geom, b.part);
    timing_end(kind, s);
    GS_LAUNCH_CHECK("exact_items");
    return GS_OK;
}

gs_status launch_combine_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                              int mode, float *dq, float *dp, double dt, double *Hpart,
                              hipStream_t s, double *vout) {
    const int64_t nb = plan_block_count(pl);
    if (nb == 0) return GS_OK;
    CombineConst k{};
    k.ks = position_scale(sigma);
    k.inv_s2 = 1.0 / (k.ks * sigma * sigma);
    k.dt = dt;
    k.ksf = ff_from_double(k.ks);
    k.inv_s2f = ff_from_double(k.inv_s2);
    k.dtf = ff_from_double(dt);
    hipLaunchKernelGGL(k_combine_rows, dim3((unsigned)nb), dim3(256), 0, s, b.part, pl.npad, b.blk,
                       pl.rows, k, mode, dq, dp, b.Sq, b.Sp, b.Fq, b.Fp, b.Q,
                       b.P, b.cen, b.cenf, Hpart, vout);
    GS_LAUNCH_CHECK("combine_rows");
    return GS_OK;
}

gs_status launch_unpack_state(const float2 *Fq, const float2 *Fp, int64_t n, float *q, float *p,
                              hipStream_t s) {
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(k_unpack_state, dim3(nblocks(3 * n)), dim3(kBlock), 0, s, Fq, Fp, n, q,
                       p);
    GS_LAUNCH_CHECK("unpack_state");
    return GS_OK;
}

int combine_blocks(int64_t n) { return (int)nblocks(n > 0 ? n : 1); }

gs_status launch_reduce_h(const double *Hpart, int nblk, int count, double *H, hipStream_t s) {
    return launch_reduce_h_seg(Hpart, nblk, nullptr, 1, count, H, s);
}

gs_status launch_reduce_h_seg(const double *Hpart, int64_t stride, const int *seg, int nsub,
                              int count, double *H, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_h, dim3((unsigned)count, (unsigned)nsub), dim3(kBlock), 0, s,
                       Hpart, stride, seg, count, H);
    GS_LAUNCH_CHECK("reduce_h");
    return GS_OK;
}

gs_status launch_exact_f64(const double *q, const double *p, int64_t n, double sigma,
                           bool with_a, double *v, double *a, hipStream_t s) {
    if (with_a)
        hipLaunchKernelGGL(k_exact_f64<true>, dim3(nblocks(n)), dim3(kBlock), 0, s, q, p, n,
                           sigma, v, a);
    else
        hipLaunchKernelGGL(k_exact_f64<false>, dim3(nblocks(n)), dim3(kBlock), 0, s, q, p, n,
                           sigma, v, a);
    GS_LAUNCH_CHECK("exact_f64");
    return GS_OK;
}

gs_status launch_euler_f64(double *q, double *p, const double *v, const double *a, int64_t n,
                           double dt, double *Hpart, hipStream_t s) {
    hipLaunchKernelGGL(k_euler_f64, dim3(nblocks(n)), dim3(kBlock), 0, s, q, p, v, a, n, dt,
                       Hpart);
    GS_LAUNCH_CHECK("euler_f64");
    return GS_OK;
}

gs_status launch_copy_f64(const double *src, double *dst, int64_t count, hipStream_t s) {
    if (count == 0) return GS_OK;
    hipLaunchKernelGGL(k_copy_f64, dim3(nblocks(count)), dim3(kBlock), 0, s, src, dst, count);
    GS_LAUNCH_CHECK("copy_f64");
    return GS_OK;
}

}  // namespace gs
