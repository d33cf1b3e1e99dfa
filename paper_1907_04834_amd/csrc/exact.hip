// exact.hip -- exact all-pairs right-hand side (Sec. 2.1, eq. 1 and eq. 3),
// the Euler step with the FP64 energy reduction, and the FP64 variants.
//
// FP32 all-pairs kernel (k_exact_pairs):
//   * one lane owns T targets (held in registers); a wave owns 64*T
//     consecutive targets; the source range [0, N) is split into S chunks
//     (grid.y) so that a launch has tens of waves per SIMD;
//   * sources are read with wave-uniform addresses, so they arrive through
//     the scalar data cache straight into SGPRs and every pair is pure VALU
//     work with no LDS or VGPR staging of source data;
//   * per pair: d = q_i - q_j (exact for near pairs), r2, G = exp2(-c r2)
//     with c = log2(e) / (2 sigma^2) on the hardware v_exp_f32, v += G p_j,
//     w = G (p_i . p_j), a += w d;
//   * compensation: each tile of kTile sources is summed in FP32 and the
//     tile sums are added into FP64 accumulators, so the rounding error of a
//     target's sum grows with the tile length, not with N;
//   * each (split, target) writes its six FP64 partial sums; a second kernel
//     adds the S partials in a fixed order (bitwise deterministic).
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "internal.h"

namespace gs {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

__global__ void k_pack(const float *__restrict__ q, const float *__restrict__ p, int64_t n,
                       int64_t npad, float4 *__restrict__ Q, float4 *__restrict__ P) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i < n) {
        Q[i] = make_float4(q[3 * i], q[3 * i + 1], q[3 * i + 2], 0.f);
        P[i] = make_float4(p[3 * i], p[3 * i + 1], p[3 * i + 2], 0.f);
    } else {
        // padding: zero momentum, so a padded source adds exactly zero
        Q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        P[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Shooting state: positions and momenta are carried in FP64 between Euler
// steps (rounding the state to FP32 every step would perturb near-pair
// distances by ~1e-7 / sigma per step and the flow amplifies that drift);
// each step hands FP32 copies to the pair kernel.
__global__ void k_pack_state(const float *__restrict__ q, const float *__restrict__ p, int64_t n,
                             int64_t npad, double *__restrict__ Sq, double *__restrict__ Sp,
                             float4 *__restrict__ Q, float4 *__restrict__ P) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i < n) {
        const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
        const float u = p[3 * i], v = p[3 * i + 1], w = p[3 * i + 2];
        Sq[3 * i] = x;
        Sq[3 * i + 1] = y;
        Sq[3 * i + 2] = z;
        Sp[3 * i] = u;
        Sp[3 * i + 1] = v;
        Sp[3 * i + 2] = w;
        Q[i] = make_float4(x, y, z, 0.f);
        P[i] = make_float4(u, v, w, 0.f);
    } else {
        Q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        P[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__global__ void k_unpack_state(const double *__restrict__ Sq, const double *__restrict__ Sp,
                               int64_t n, float *__restrict__ q, float *__restrict__ p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    q[i] = (float)Sq[i];
    p[i] = (float)Sp[i];
}

// Positions only (targets of the velocity field), zero-padded.
__global__ void k_pack_pos(const float *__restrict__ x, int64_t m, int64_t npad,
                           float4 *__restrict__ X) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    X[i] = i < m ? make_float4(x[3 * i], x[3 * i + 1], x[3 * i + 2], 0.f)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Sums of targets t0 + 64 k (k < T, one lane each) over sources [j0, j1)
// (a multiple of kTile), written as six FP64 rows of dst (row stride ntgt).
template <int T, bool WITH_A>
__device__ __forceinline__ void pair_sums(const float4 *__restrict__ Qt,
                                          const float4 *__restrict__ Pt, int64_t ntgt,
                                          const float4 *__restrict__ Qs,
                                          const float4 *__restrict__ Ps, int64_t t0, int64_t j0,
                                          int64_t j1, float negc, double *__restrict__ dst) {
    // B sources are processed stage by stage (differences, r^2, exp2, sums)
    // so that every wave has B independent dependency chains in flight.
    constexpr int B = T == 1 ? 4 : 2;
    float x[T], y[T], z[T], px[T], py[T], pz[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const float4 a = Qt[t0 + 64 * k];
        x[k] = a.x;
        y[k] = a.y;
        z[k] = a.z;
        if (WITH_A) {
            const float4 b = Pt[t0 + 64 * k];
            px[k] = b.x;
            py[k] = b.y;
            pz[k] = b.z;
        }
    }
    double sv[T][3], sa[T][3];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[k][c] = sa[k][c] = 0.0;

    for (int64_t jt = j0; jt < j1; jt += kTile) {
        float tv[T][3], ta[T][3];
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) tv[k][c] = ta[k][c] = 0.f;
#pragma unroll 2
        for (int u = 0; u < kTile; u += B) {
            float4 qj[B], pj[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                qj[b] = Qs[jt + u + b];
                pj[b] = Ps[jt + u + b];
            }
#pragma unroll
            for (int k = 0; k < T; ++k) {
                float dx[B], dy[B], dz[B], g[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    dx[b] = x[k] - qj[b].x;
                    dy[b] = y[k] - qj[b].y;
                    dz[b] = z[k] - qj[b].z;
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const float r2 = dx[b] * dx[b] + dy[b] * dy[b] + dz[b] * dz[b];
                    g[b] = __builtin_amdgcn_exp2f(r2 * negc);
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    tv[k][0] += g[b] * pj[b].x;
                    tv[k][1] += g[b] * pj[b].y;
                    tv[k][2] += g[b] * pj[b].z;
                    if (WITH_A) {
                        const float w =
                            g[b] * (px[k] * pj[b].x + py[k] * pj[b].y + pz[k] * pj[b].z);
                        ta[k][0] += w * dx[b];
                        ta[k][1] += w * dy[b];
                        ta[k][2] += w * dz[b];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sv[k][c] += (double)tv[k][c];
                if (WITH_A) sa[k][c] += (double)ta[k][c];
            }
    }
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t i = t0 + 64 * k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dst[c * ntgt + i] = sv[k][c];
            if (WITH_A) dst[(3 + c) * ntgt + i] = sa[k][c];
        }
    }
}

// Block b of a launch takes target block b / splits against source split
// b % splits: consecutive blocks share their targets and stream different
// source ranges.
//
// Occupancy hint: allowing at most 7 waves per SIMD
// lets the compiler keep the scalar loads of 8 sources in flight (66 VGPRs);
// aiming at 8 waves it splits each batch of 8 sources into two halves with a
// full wait each, measured 16.4 vs 14.7 ms per 200k right-hand side.
template <int T, bool WITH_A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 7))) void k_exact_pairs(
    const float4 *__restrict__ Qt, const float4 *__restrict__ Pt, int64_t ntgt,
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, int64_t chunk, int64_t nsrc,
    int splits, float negc, double *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t split = blockIdx.x % splits, tb = blockIdx.x / splits;
    const int64_t wave = tb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t t0 = wave * (64 * T) + lane;
    const int64_t j0 = split * chunk;
    const int64_t j1 = j0 + chunk < nsrc ? j0 + chunk : nsrc;
    pair_sums<T, WITH_A>(Qt, Pt, ntgt, Qs, Ps, t0, j0, j1, negc, part + split * 6 * ntgt);
}

// Batched sets: block b takes work item b = (first padded target row of 256,
// source rows [j0, j1) of the same set, partial slot).  Positions are stored
// scaled by k = sqrt(log2(e) / (2 sigma^2)), so that G = exp2(-|q'_i -
// q'_j|^2) needs no scaling multiply and the a-sums come out multiplied by
// k.  One target per lane; the sources are wave-uniform (scalar loads), FP32
// pair terms are summed per tile of kTile sources and the tile sums
// accumulated in FP64.
//
// The sources of the next group of four are loaded while the current four
// are evaluated (software pipelining through SGPRs): without it every group
// waits for its own loads.  With at most 64 VGPRs (8 waves per SIMD) this
// measured 13.3 ms per 200k right-hand side, against 14.4 ms for groups of
// eight loaded and then evaluated (7 waves per SIMD) and 13.4 ms for the
// pipelined loop at 7 waves.
template <bool WITH_A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exact_items(
    const float4 *__restrict__ Q, const float4 *__restrict__ P, int64_t npad,
    const int4 *__restrict__ items, double *__restrict__ part) {
    constexpr int B = 4;  // sources per pipeline stage (kTile is a multiple)
    const int4 it = items[blockIdx.x];
    if (it.w < 0) return;  // padding item (keeps the XCD interleave aligned)
    const int64_t t0 = (int64_t)it.x + (threadIdx.x >> 6) * 64 + (threadIdx.x & 63);
    const float4 a = Q[t0];
    const float x = a.x, y = a.y, z = a.z;
    float px = 0.f, py = 0.f, pz = 0.f;
    if (WITH_A) {
        const float4 b = P[t0];
        px = b.x;
        py = b.y;
        pz = b.z;
    }
    double sv[3] = {0, 0, 0}, sa[3] = {0, 0, 0};
    // 32-bit source indices: the loop and prefetch-clamp compares then run on
    // the scalar unit (there is no 64-bit scalar less-than)
    const int j0 = it.y, j1 = it.z;
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
                g[b] = __builtin_amdgcn_exp2f(-(dx[b] * dx[b] + dy[b] * dy[b] + dz[b] * dz[b]));
#pragma unroll
            for (int b = 0; b < B; ++b) {
                tv[0] += g[b] * pj[b].x;
                tv[1] += g[b] * pj[b].y;
                tv[2] += g[b] * pj[b].z;
                if (WITH_A) {
                    const float w = g[b] * (px * pj[b].x + py * pj[b].y + pz * pj[b].z);
                    ta[0] += w * dx[b];
                    ta[1] += w * dy[b];
                    ta[2] += w * dz[b];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sv[c] += (double)tv[c];
            if (WITH_A) sa[c] += (double)ta[c];
        }
    }
    double *dst = part + (int64_t)it.w * 6 * npad;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dst[c * npad + t0] = sv[c];
        if (WITH_A) dst[(3 + c) * npad + t0] = sa[c];
    }
}

// Same sums with the source tile staged in LDS: every wave reads each source
// with one wave-uniform (broadcast) LDS load into VGPRs, so the pair
// arithmetic has only VGPR operands (VALU instructions that read an SGPR
// operand issue measurably slower on gfx950).
constexpr int kLdsTile = 256;  // sources per LDS tile (one per thread)

template <int T, bool WITH_A>
__global__ __launch_bounds__(256) void k_exact_pairs_lds(
    const float4 *__restrict__ Qt, const float4 *__restrict__ Pt, int64_t ntgt,
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, int64_t chunk, int64_t nsrc,
    int splits, float negc, double *__restrict__ part) {
    __shared__ float4 sq[kLdsTile];
    __shared__ float4 sp[kLdsTile];
    constexpr int B = 4;
    const int lane = threadIdx.x & 63;
    const int64_t split = blockIdx.x % splits, tb = blockIdx.x / splits;
    const int64_t wave = tb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t t0 = wave * (64 * T) + lane;

    float x[T], y[T], z[T], px[T], py[T], pz[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const float4 a = Qt[t0 + 64 * k];
        x[k] = a.x;
        y[k] = a.y;
        z[k] = a.z;
        if (WITH_A) {
            const float4 b = Pt[t0 + 64 * k];
            px[k] = b.x;
            py[k] = b.y;
            pz[k] = b.z;
        }
    }
    double sv[T][3], sa[T][3];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[k][c] = sa[k][c] = 0.0;

    const int64_t j0 = split * chunk;
    const int64_t j1 = j0 + chunk < nsrc ? j0 + chunk : nsrc;
    for (int64_t jt = j0; jt < j1; jt += kLdsTile) {
        __syncthreads();
        sq[threadIdx.x] = Qs[jt + threadIdx.x];
        sp[threadIdx.x] = Ps[jt + threadIdx.x];
        __syncthreads();
        for (int u0 = 0; u0 < kLdsTile; u0 += kTile) {
            float tv[T][3], ta[T][3];
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) tv[k][c] = ta[k][c] = 0.f;
#pragma unroll 2
            for (int u = u0; u < u0 + kTile; u += B) {
                float4 qj[B], pj[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    qj[b] = sq[u + b];
                    pj[b] = sp[u + b];
                }
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    float dx[B], dy[B], dz[B], g[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        dx[b] = x[k] - qj[b].x;
                        dy[b] = y[k] - qj[b].y;
                        dz[b] = z[k] - qj[b].z;
                    }
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        g[b] = __builtin_amdgcn_exp2f(
                            (dx[b] * dx[b] + dy[b] * dy[b] + dz[b] * dz[b]) * negc);
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        tv[k][0] += g[b] * pj[b].x;
                        tv[k][1] += g[b] * pj[b].y;
                        tv[k][2] += g[b] * pj[b].z;
                        if (WITH_A) {
                            const float w =
                                g[b] * (px[k] * pj[b].x + py[k] * pj[b].y + pz[k] * pj[b].z);
                            ta[k][0] += w * dx[b];
                            ta[k][1] += w * dy[b];
                            ta[k][2] += w * dz[b];
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sv[k][c] += (double)tv[k][c];
                    if (WITH_A) sa[k][c] += (double)ta[k][c];
                }
        }
    }
    double *dst = part + split * 6 * ntgt;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t i = t0 + 64 * k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dst[c * ntgt + i] = sv[k][c];
            if (WITH_A) dst[(3 + c) * ntgt + i] = sa[k][c];
        }
    }
}

// ---------------------------------------------------------------- MFMA kernel
// Matrix-core formulation of the same sums.  With c = log2(e) / (2 sigma^2),
// k = sqrt(c), a per-wave origin o and scaled, centred coordinates
// t_i = k (q_i - o), s_j = k (q_j - o):
//   G_ij = exp2(-|t_i - s_j|^2)
//   v_i  = sum_j G_ij p_j
//   a_i  = sigma^-2 / k * sum_c p_ic (t_i M_ic - Q_ic)   with
//   M_ic = sum_j G_ij p_jc,  Q_icd = sum_j G_ij p_jc s_jd.
// The 3 + 9 = 12 source features (p_c, p_c s_d) form a 16 x 4 operand (rows
// 12..15 are zero) and G for 16 targets x 4 sources the 4 x 16 operand of
// v_mfma_f32_16x16x4_f32; only G itself (6 VALU + exp2 per pair) stays on
// the vector ALU.  The centring keeps the cancellation in t M - Q small for
// the near pairs that matter.  Each lane: source s = lane / 16 of the
// current group of 4, feature / target row r = lane % 16.  Accumulators are
// flushed to FP64 every kFlush sources.  The partial (v, a k sigma^2 ... )
// sums are written in the layout of k_exact_pairs.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kMTile = 256;   // sources staged in LDS per block step
constexpr int kFlush = 64;    // sources summed in FP32 before the FP64 flush

template <int T>
__global__ __launch_bounds__(256) void k_exact_mfma(
    const float4 *__restrict__ Qt, const float4 *__restrict__ Pt, int64_t ntgt,
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, int64_t chunk, int64_t nsrc,
    float kscale, double inv_k, double *__restrict__ part) {
    __shared__ float4 sq[kMTile];
    __shared__ float4 sp[kMTile];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, ks = lane >> 4;
    const int64_t tbase = ((int64_t)blockIdx.x * 4 + wv) * (16 * T);

    const float4 o = Qt[tbase];  // wave origin: its first target
    const float okx = o.x * kscale, oky = o.y * kscale, okz = o.z * kscale;
    float tx[T], ty[T], tz[T];
#pragma unroll
    for (int g = 0; g < T; ++g) {
        const float4 a = Qt[tbase + 16 * g + r];
        tx[g] = fmaf(a.x, kscale, -okx);
        ty[g] = fmaf(a.y, kscale, -oky);
        tz[g] = fmaf(a.z, kscale, -okz);
    }
    // feature of this lane: r < 3 -> p_r; 3 <= r < 12 -> p_c s_d; else 0
    const int csel = r < 3 ? r : (r < 12 ? (r - 3) / 3 : 3);
    const int dsel = (r >= 3 && r < 12) ? (r - 3) % 3 : 3;
    // one-hot weights pick s_dsel (or 1) without branches; exact in FP32
    const float m0 = dsel == 0 ? 1.f : 0.f, m1 = dsel == 1 ? 1.f : 0.f;
    const float m2 = dsel == 2 ? 1.f : 0.f, m3 = dsel == 3 ? 1.f : 0.f;

    floatx4 acc[T];
    double accd[T][4];
#pragma unroll
    for (int g = 0; g < T; ++g) {
        acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) accd[g][i] = 0.0;
    }
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < nsrc ? j0 + chunk : nsrc;
    const float *spf = reinterpret_cast<const float *>(sp);
    for (int64_t jt = j0; jt < j1; jt += kMTile) {
        __syncthreads();
        sq[threadIdx.x] = Qs[jt + threadIdx.x];
        sp[threadIdx.x] = Ps[jt + threadIdx.x];
        __syncthreads();
        for (int f0 = 0; f0 < kMTile; f0 += kFlush) {
#pragma unroll
            for (int c4 = f0; c4 < f0 + kFlush; c4 += 4) {
                const float4 sj = sq[c4 + ks];
                const float pc = spf[4 * (c4 + ks) + csel];
                const float sx = fmaf(sj.x, kscale, -okx);
                const float sy = fmaf(sj.y, kscale, -oky);
                const float sz = fmaf(sj.z, kscale, -okz);
                const float feat = pc * fmaf(m0, sx, fmaf(m1, sy, fmaf(m2, sz, m3)));
#pragma unroll
                for (int g = 0; g < T; ++g) {
                    const float dx = tx[g] - sx, dy = ty[g] - sy, dz = tz[g] - sz;
                    const float gv = __builtin_amdgcn_exp2f(-(dx * dx + dy * dy + dz * dz));
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(feat, gv, acc[g], 0, 0, 0);
                }
            }
#pragma unroll
            for (int g = 0; g < T; ++g) {
#pragma unroll
                for (int i = 0; i < 4; ++i) accd[g][i] += (double)acc[g][i];
                acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
        }
    }
    // lane r + 16 b holds features 4b..4b+3 of target r; gather them in lane r
    double *dst = part + (int64_t)blockIdx.y * 6 * ntgt;
#pragma unroll
    for (int g = 0; g < T; ++g) {
        double f1[4], f2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f1[i] = __shfl(accd[g][i], r + 16, 64);
            f2[i] = __shfl(accd[g][i], r + 32, 64);
        }
        if (ks == 0) {
            const int64_t it = tbase + 16 * g + r;
            const float4 pi = Pt[it];
            const double M[3] = {accd[g][0], accd[g][1], accd[g][2]};
            const double Q[3][3] = {{accd[g][3], f1[0], f1[1]},
                                    {f1[2], f1[3], f2[0]},
                                    {f2[1], f2[2], f2[3]}};
            const double t[3] = {tx[g], ty[g], tz[g]};
            const double pc[3] = {pi.x, pi.y, pi.z};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) s += pc[c] * (t[d] * M[c] - Q[c][d]);
                dst[d * ntgt + it] = M[d];
                dst[(3 + d) * ntgt + it] = s * inv_k;
            }
        }
    }
}

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

__global__ __launch_bounds__(256) void k_combine_rhs(const double *__restrict__ part, int splits,
                                                     int64_t ntgt, int64_t n, double inv_s2,
                                                     float *__restrict__ dq,
                                                     float *__restrict__ dp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < splits; ++s)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += part[((int64_t)s * 6 + c) * ntgt + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dq[3 * i + c] = (float)acc[c];
        if (dp) dp[3 * i + c] = (float)(acc[3 + c] * inv_s2);
    }
}

__global__ __launch_bounds__(256) void k_combine_euler(const double *__restrict__ part,
                                                       int splits, int64_t ntgt, int64_t n,
                                                       double inv_s2, double dt,
                                                       double *__restrict__ Sq,
                                                       double *__restrict__ Sp,
                                                       float4 *__restrict__ Q,
                                                       float4 *__restrict__ P,
                                                       double *__restrict__ Hpart) {
    __shared__ double lds[8];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int s = 0; s < splits; ++s)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] += part[((int64_t)s * 6 + c) * ntgt + i];
        double q[3], p[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            q[c] = Sq[3 * i + c];
            p[c] = Sp[3 * i + c];
        }
        e = p[0] * acc[0] + p[1] * acc[1] + p[2] * acc[2];
        if (dt > 0.0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                q[c] += dt * acc[c];
                p[c] += dt * (acc[3 + c] * inv_s2);
                Sq[3 * i + c] = q[c];
                Sp[3 * i + c] = p[c];
            }
            Q[i] = make_float4((float)q[0], (float)q[1], (float)q[2], 0.f);
            P[i] = make_float4((float)p[0], (float)p[1], (float)p[2], 0.f);
        }
    }
    if (Hpart) {
        double s = block_sum_f64(e, lds);
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

// ---------------------------------------------------------------- batched sets
// Rows are padded per set to whole blocks of 256; block b of the rows is
// described by blk[b] = (first real point of the block, real rows in it,
// set, partial slots of the set).  Real point i of set s sits at padded row
// base_s + (i - first point of s).

__global__ __launch_bounds__(256) void k_pack_state_rows(const float *__restrict__ q,
                                                         const float *__restrict__ p,
                                                         const int4 *__restrict__ blk,
                                                         double ks, double *__restrict__ Sq,
                                                         double *__restrict__ Sp,
                                                         float4 *__restrict__ Q,
                                                         float4 *__restrict__ P) {
    const int4 d = blk[blockIdx.x];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
        const float u = p[3 * i], v = p[3 * i + 1], w = p[3 * i + 2];
        Sq[3 * i] = x;
        Sq[3 * i + 1] = y;
        Sq[3 * i + 2] = z;
        Sp[3 * i] = u;
        Sp[3 * i + 1] = v;
        Sp[3 * i + 2] = w;
        Q[row] = make_float4((float)(ks * x), (float)(ks * y), (float)(ks * z), 0.f);
        P[row] = make_float4(u, v, w, 0.f);
    } else {
        // padding: zero momentum, so a padded source adds exactly zero
        Q[row] = make_float4(0.f, 0.f, 0.f, 0.f);
        P[row] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// FP64 [n][3] pair (a, b) -> packed FP32 rows (sa a, sb b), zero padding.
__global__ __launch_bounds__(256) void k_pack_rows64(const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     const int4 *__restrict__ blk, double sa,
                                                     double sb, float4 *__restrict__ A,
                                                     float4 *__restrict__ B) {
    const int4 d = blk[blockIdx.x];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        A[row] = make_float4((float)(sa * a[3 * i]), (float)(sa * a[3 * i + 1]),
                             (float)(sa * a[3 * i + 2]), 0.f);
        B[row] = make_float4((float)(sb * b[3 * i]), (float)(sb * b[3 * i + 1]),
                             (float)(sb * b[3 * i + 2]), 0.f);
    } else {
        A[row] = make_float4(0.f, 0.f, 0.f, 0.f);
        B[row] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// inv_s2 here is 1 / (k sigma^2): the a-sums were taken on scaled positions.
__global__ __launch_bounds__(256) void k_combine_rows(const double *__restrict__ part,
                                                      int64_t npad, const int4 *__restrict__ blk,
                                                      double inv_s2, double ks, int mode,
                                                      float *__restrict__ dq,
                                                      float *__restrict__ dp, double dt,
                                                      double *__restrict__ Sq,
                                                      double *__restrict__ Sp,
                                                      float4 *__restrict__ Q,
                                                      float4 *__restrict__ P,
                                                      double *__restrict__ Hpart,
                                                      double *__restrict__ vout) {
    __shared__ double lds[8];
    const int4 d = blk[blockIdx.x];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if ((int)threadIdx.x < d.y) {
        const int64_t i = (int64_t)d.x + threadIdx.x;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int s = 0; s < d.w; ++s)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] += part[((int64_t)s * 6 + c) * npad + row];
        if (mode == 0) {  // right-hand side
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dq[3 * i + c] = (float)acc[c];
                dp[3 * i + c] = (float)(acc[3 + c] * inv_s2);
            }
        } else {
            double q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                q[c] = Sq[3 * i + c];
                p[c] = Sp[3 * i + c];
            }
            e = p[0] * acc[0] + p[1] * acc[1] + p[2] * acc[2];
            if (vout)
#pragma unroll
                for (int c = 0; c < 3; ++c) vout[3 * i + c] = acc[c];
            if (dt > 0.0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] += dt * acc[c];
                    p[c] += dt * (acc[3 + c] * inv_s2);
                    Sq[3 * i + c] = q[c];
                    Sp[3 * i + c] = p[c];
                }
                Q[row] = make_float4((float)(ks * q[0]), (float)(ks * q[1]), (float)(ks * q[2]),
                                     0.f);
                P[row] = make_float4((float)p[0], (float)p[1], (float)p[2], 0.f);
            }
        }
    }
    if (Hpart) {
        const double s = block_sum_f64(e, lds);
        if (threadIdx.x == 0) Hpart[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------- FP64 path
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
// Targets per lane of the VALU kernel: more targets give each wave more
// independent dependency chains per source; GS_EXACT_TPL (1, 2 or 4)
// overrides the default for tuning.
static int exact_tpl() {
    static int v = [] {
        const char *e = getenv("GS_EXACT_TPL");
        const int t = e ? atoi(e) : 0;
        return (t == 1 || t == 2 || t == 4) ? t : kExactTplDefault;
    }();
    return v;
}

// Source staging of the VALU kernel: scalar loads (default) or LDS tiles;
// GS_EXACT_SRC=lds selects the latter (measured equal within 1% at 200k).
static bool exact_lds() {
    static bool v = [] {
        const char *e = getenv("GS_EXACT_SRC");
        return e && e[0] == 'l';
    }();
    return v;
}

ExactPlan plan_exact(int64_t n_targets, int64_t n_sources, bool mfma) {
    ExactPlan pl{};
    pl.n = n_targets;
    pl.tpl = exact_tpl();
    pl.mfma = mfma;
    // targets per block: VALU kernel 4 waves x 64 lanes x tpl; MFMA kernel
    // 4 waves x kMfmaGroups x 16 (= 256); padded to 1024 so both fit; sources
    // in steps of 256
    const int64_t tgt_per_block = 1024;
    pl.ntgt = round_up(n_targets > 0 ? n_targets : 1, tgt_per_block);
    pl.nsrc = round_up(n_sources > 0 ? n_sources : 1, kMTile);
    // Aim at ~24k blocks of 256 targets per launch (about 96 waves per SIMD
    // in a few rounds, so the last round is a small share of the launch);
    // never split below 256 sources.  The split count depends on n only (not
    // on the kernel or its tuning), so workspace sizes never depend on those
    // choices.
    const int64_t tblocks = pl.ntgt / 256;
    int64_t s = (kSplitBlocks + tblocks - 1) / tblocks;
    const int64_t max_s = pl.nsrc / kMTile;
    if (s > max_s) s = max_s;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    pl.chunk_quantum = kMTile;
    pl.chunk = round_up((pl.nsrc + s - 1) / s, kMTile);
    pl.splits = (int)((pl.nsrc + pl.chunk - 1) / pl.chunk);
    return pl;
}

void carve_exact(Arena &a, const ExactPlan &pl, ExactBufs &b) {
    const int64_t m = pl.nsrc > pl.ntgt ? pl.nsrc : pl.ntgt;
    b.Q = a.take<float4>(m);
    b.P = a.take<float4>(m);
    b.part = a.take<double>((size_t)pl.splits * 6 * pl.ntgt);
}

int combine_blocks(int64_t n) { return (int)nblocks(n > 0 ? n : 1); }

// ---------------------------------------------------------------- launchers
gs_status launch_pack(const float *q, const float *p, int64_t n, int64_t npad, float4 *Q,
                      float4 *P, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(nblocks(npad)), dim3(kBlock), 0, s, q, p, n, npad, Q, P);
    GS_LAUNCH_CHECK("pack");
    return GS_OK;
}

gs_status launch_pack_pos(const float *x, int64_t m, int64_t npad, float4 *X, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_pos, dim3(nblocks(npad)), dim3(kBlock), 0, s, x, m, npad, X);
    GS_LAUNCH_CHECK("pack_pos");
    return GS_OK;
}

gs_status launch_exact_pairs(const ExactPlan &pl, const float4 *Qt, const float4 *Pt,
                             const float4 *Qs, const float4 *Ps, double sigma, bool with_a,
                             double *part, hipStream_t s) {
    if (with_a && pl.mfma) {
        const double c = kLog2e / (2.0 * sigma * sigma);
        const float k = (float)sqrt(c);
        dim3 grid((unsigned)(pl.ntgt / (16 * kMfmaGroups * 4)), (unsigned)pl.splits);
        timing_begin(KIND_EXACT, s);
        hipLaunchKernelGGL((k_exact_mfma<kMfmaGroups>), grid, dim3(256), 0, s, Qt, Pt, pl.ntgt, Qs,
                           Ps, pl.chunk, pl.nsrc, k, 1.0 / (double)k, part);
        timing_end(KIND_EXACT, s);
        GS_LAUNCH_CHECK("exact_mfma");
        return GS_OK;
    }
    const float negc = (float)(-kLog2e / (2.0 * sigma * sigma));
    dim3 grid((unsigned)(pl.ntgt / (64 * pl.tpl * 4) * pl.splits));
    const int kind = with_a ? KIND_EXACT : KIND_EXACT_V;
    timing_begin(kind, s);
#define GS_PAIRS(T, A)                                                                     \
    do {                                                                                   \
        if (exact_lds())                                                                   \
            hipLaunchKernelGGL((k_exact_pairs_lds<T, A>), grid, dim3(256), 0, s, Qt, Pt,   \
                               pl.ntgt, Qs, Ps, pl.chunk, pl.nsrc, pl.splits, negc, part); \
        else                                                                               \
            hipLaunchKernelGGL((k_exact_pairs<T, A>), grid, dim3(256), 0, s, Qt, Pt, pl.ntgt, \
                               Qs, Ps, pl.chunk, pl.nsrc, pl.splits, negc, part);          \
    } while (0)
    if (with_a) {
        if (pl.tpl == 1) GS_PAIRS(1, true);
        else if (pl.tpl == 4) GS_PAIRS(4, true);
        else GS_PAIRS(2, true);
    } else {
        if (pl.tpl == 1) GS_PAIRS(1, false);
        else if (pl.tpl == 4) GS_PAIRS(4, false);
        else GS_PAIRS(2, false);
    }
#undef GS_PAIRS
    timing_end(kind, s);
    GS_LAUNCH_CHECK("exact_pairs");
    return GS_OK;
}

gs_status launch_combine_rhs(const ExactPlan &pl, const double *part, double sigma, float *dq,
                             float *dp, hipStream_t s) {
    hipLaunchKernelGGL(k_combine_rhs, dim3(nblocks(pl.n)), dim3(kBlock), 0, s, part, pl.splits,
                       pl.ntgt, pl.n, 1.0 / (sigma * sigma), dq, dp);
    GS_LAUNCH_CHECK("combine_rhs");
    return GS_OK;
}

gs_status launch_combine_euler(const ExactPlan &pl, const double *part, double sigma, double dt,
                               double *Sq, double *Sp, float4 *Q, float4 *P, double *Hpart,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_combine_euler, dim3(nblocks(pl.n)), dim3(kBlock), 0, s, part,
                       pl.splits, pl.ntgt, pl.n, 1.0 / (sigma * sigma), dt, Sq, Sp, Q, P,
                       Hpart);
    GS_LAUNCH_CHECK("combine_euler");
    return GS_OK;
}

gs_status launch_pack_state(const float *q, const float *p, int64_t n, int64_t npad, double *Sq,
                            double *Sp, float4 *Q, float4 *P, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_state, dim3(nblocks(npad)), dim3(kBlock), 0, s, q, p, n, npad, Sq,
                       Sp, Q, P);
    GS_LAUNCH_CHECK("pack_state");
    return GS_OK;
}

gs_status launch_unpack_state(const double *Sq, const double *Sp, int64_t n, float *q, float *p,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_unpack_state, dim3(nblocks(3 * n)), dim3(kBlock), 0, s, Sq, Sp, n, q,
                       p);
    GS_LAUNCH_CHECK("unpack_state");
    return GS_OK;
}

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

// ---------------------------------------------------------------- batched sets
// Target number of work items (blocks) of one batched launch;
// GS_EXACT_ITEM_BLOCKS overrides it for tuning.
static int64_t item_blocks() {
    static int64_t v = [] {
        const char *e = getenv("GS_EXACT_ITEM_BLOCKS");
        const long long b = e ? atoll(e) : 0;
        return (int64_t)(b >= 256 && b <= (1 << 22) ? b : kSplitBlocks);
    }();
    return v;
}

ExactBatchPlan plan_exact_batch(const int64_t *offsets, int nsub, int64_t items) {
    ExactBatchPlan pl{};
    pl.nsub = nsub;
    pl.ntot = offsets[nsub];
    std::vector<int64_t> base(nsub), tp(nsub), sp(nsub);
    int64_t work = 0, rows = 0;
    for (int s = 0; s < nsub; ++s) {
        const int64_t n = offsets[s + 1] - offsets[s];
        base[s] = rows;
        tp[s] = round_up(n, 256);
        sp[s] = round_up(n, kTile);
        rows += tp[s];
        work += tp[s] * sp[s];
    }
    pl.npad = rows > 0 ? rows : 256;
    // Source chunk: about `items` blocks of 256 targets in a launch, never
    // below 256 sources (4 tiles).  Small sets need the short chunks to fill
    // the GPU: one RHS of 5000 / 20 000 points took 0.119 / 0.308 ms with
    // chunks of at least 2048 sources, 0.025 / 0.152 ms with at least 256.
    const int64_t blocks = items > 0 ? items : item_blocks();
    int64_t chunk = round_up((work + 256 * blocks - 1) / (256 * blocks), kTile);
    if (chunk < 256) chunk = 256;
    pl.max_chunks = 1;
    pl.bseg.resize(nsub + 1);
    struct Chunk {
        int set, c;
        int64_t j0, j1, work;
    };
    std::vector<Chunk> chunks;
    for (int s = 0; s < nsub; ++s) {
        pl.bseg[s] = (int)pl.blocks.size();
        const int64_t n = offsets[s + 1] - offsets[s];
        if (n == 0) continue;
        int nch = (int)((sp[s] + chunk - 1) / chunk);
        const int64_t csz = round_up((sp[s] + nch - 1) / nch, kTile);
        nch = (int)((sp[s] + csz - 1) / csz);
        if (nch > pl.max_chunks) pl.max_chunks = nch;
        for (int64_t b = 0; b < tp[s] / 256; ++b) {
            const int64_t cnt = n - 256 * b < 256 ? n - 256 * b : 256;
            pl.blocks.push_back(make_int4((int)(offsets[s] + 256 * b), (int)cnt, s, nch));
        }
        for (int c = 0; c < nch; ++c) {
            const int64_t j0 = base[s] + c * csz;
            const int64_t j1 = j0 + csz < base[s] + sp[s] ? j0 + csz : base[s] + sp[s];
            chunks.push_back({s, c, j0, j1, tp[s] * (j1 - j0)});
        }
    }
    pl.bseg[nsub] = (int)pl.blocks.size();
    // Every source chunk gets a home XCD (the largest chunks first, each to
    // the least loaded XCD), so that an XCD streams only its own chunks and
    // they stay in its L2.  Workgroups are dealt to the 8 XCDs in turn, so
    // item i of the launch runs on XCD i % 8: the launch interleaves the 8
    // queues, largest items first in each, and pads a short queue with empty
    // items (slot -1) to keep the interleave aligned.
    std::vector<int> order(chunks.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return chunks[a].work > chunks[b].work; });
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
        const Chunk &ch = chunks[k];
        load[x] += ch.work;
        for (int64_t b = 0; b < tp[ch.set] / 256; ++b)
            queue[x].push_back({256 * (ch.j1 - ch.j0),
                                make_int4((int)(base[ch.set] + 256 * b), (int)ch.j0, (int)ch.j1,
                                          ch.c)});
    }
    size_t longest = 0;
    for (int x = 0; x < kXcds; ++x) {
        std::stable_sort(queue[x].begin(), queue[x].end(),
                         [](const Item &a, const Item &b) { return a.cost > b.cost; });
        if (queue[x].size() > longest) longest = queue[x].size();
    }
    pl.items.reserve(longest * kXcds);
    for (size_t i = 0; i < longest; ++i)
        for (int x = 0; x < kXcds; ++x)
            pl.items.push_back(i < queue[x].size() ? queue[x][i].it : make_int4(0, 0, 0, -1));
    while (!pl.items.empty() && pl.items.back().w < 0) pl.items.pop_back();
    return pl;
}

void carve_exact_batch(Arena &a, const ExactBatchPlan &pl, int nt, ExactBatchBufs &b) {
    b.Q = a.take<float4>(pl.npad);
    b.P = a.take<float4>(pl.npad);
    b.part = a.take<double>((size_t)pl.max_chunks * 6 * pl.npad);
    const int64_t n = pl.ntot > 0 ? pl.ntot : 1;
    b.Sq = a.take<double>(3 * n);
    b.Sp = a.take<double>(3 * n);
    const size_t nb = pl.blocks.size() > 0 ? pl.blocks.size() : 1;
    b.Hpart = a.take<double>((size_t)(nt + 1) * nb);
}

// k = sqrt(log2(e) / (2 sigma^2)): the items kernel works on k q.
double position_scale(double sigma) { return sqrt(kLog2e / (2.0 * sigma * sigma)); }

gs_status launch_pack_rows64(const ExactBatchPlan &pl, const int4 *blk, const double *a,
                             const double *b, double sa, float4 *A, float4 *B, hipStream_t s,
                             double sb) {
    if (pl.blocks.empty()) return GS_OK;
    hipLaunchKernelGGL(k_pack_rows64, dim3((unsigned)pl.blocks.size()), dim3(256), 0, s, a, b,
                       blk, sa, sb, A, B);
    GS_LAUNCH_CHECK("pack_rows64");
    return GS_OK;
}

gs_status launch_pack_state_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b,
                                 const float *q, const float *p, double sigma, hipStream_t s) {
    if (pl.blocks.empty()) return GS_OK;
    hipLaunchKernelGGL(k_pack_state_rows, dim3((unsigned)pl.blocks.size()), dim3(256), 0, s, q,
                       p, b.blk, position_scale(sigma), b.Sq, b.Sp, b.Q, b.P);
    GS_LAUNCH_CHECK("pack_state_rows");
    return GS_OK;
}

gs_status launch_exact_items(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                             bool with_a, hipStream_t s) {
    (void)sigma;  // the scale is in the stored positions
    if (pl.items.empty()) return GS_OK;
    const int kind = with_a ? KIND_EXACT : KIND_EXACT_V;
    timing_begin(kind, s);
    if (with_a)
        hipLaunchKernelGGL(k_exact_items<true>, dim3((unsigned)pl.items.size()), dim3(256), 0, s,
                           b.Q, b.P, pl.npad, b.items, b.part);
    else
        hipLaunchKernelGGL(k_exact_items<false>, dim3((unsigned)pl.items.size()), dim3(256), 0, s,
                           b.Q, b.P, pl.npad, b.items, b.part);
    timing_end(kind, s);
    GS_LAUNCH_CHECK("exact_items");
    return GS_OK;
}

gs_status launch_combine_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                              int mode, float *dq, float *dp, double dt, double *Hpart,
                              hipStream_t s, double *vout) {
    if (pl.blocks.empty()) return GS_OK;
    const double ks = position_scale(sigma);
    hipLaunchKernelGGL(k_combine_rows, dim3((unsigned)pl.blocks.size()), dim3(256), 0, s, b.part,
                       pl.npad, b.blk, 1.0 / (ks * sigma * sigma), ks, mode, dq, dp, dt, b.Sq,
                       b.Sp, b.Q, b.P, Hpart, vout);
    GS_LAUNCH_CHECK("combine_rows");
    return GS_OK;
}

gs_status launch_exact_f64(const double *q, const double *p, int64_t n, double sigma,
                           bool with_a, double *v, double *a, hipStream_t s) {
    timing_begin(KIND_EXACT, s);
    if (with_a)
        hipLaunchKernelGGL(k_exact_f64<true>, dim3(nblocks(n)), dim3(kBlock), 0, s, q, p, n,
                           sigma, v, a);
    else
        hipLaunchKernelGGL(k_exact_f64<false>, dim3(nblocks(n)), dim3(kBlock), 0, s, q, p, n,
                           sigma, v, a);
    timing_end(KIND_EXACT, s);
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
    hipLaunchKernelGGL(k_copy_f64, dim3(nblocks(count)), dim3(kBlock), 0, s, src, dst, count);
    GS_LAUNCH_CHECK("copy_f64");
    return GS_OK;
}

}  // namespace gs
