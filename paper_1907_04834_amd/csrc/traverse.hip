// traverse.hip -- Barnes-Hut traversal (Sec. 2.2, "Tree-based Forward/Backward
// Gaussian Kernel Calculation", eq. 4) and the Barnes-Hut RHS / shooting.
//
// Wave-coherent traversal: a wave owns 64 consecutive targets of the Morton
// order (spatial neighbours), and walks the tree with one wave-uniform stack
// of (node, lane mask) entries in LDS.  Every lane takes its own decision at
// every node it reaches:
//   * approximate (n_k >= 2, the target is at least kappa*sigma from the
//     node's tight box, and s_k < theta |x - C_k|): the node acts as n_k
//     virtual points at C_k with momentum P_k / n_k;
//   * otherwise a leaf contributes its exact pairs;
//   * otherwise its children are pushed with the mask of the lanes that
//     opened it, so a lane that approximated a node never sees its subtree.
// Node records are read with wave-uniform addresses (scalar loads); the
// decisions are taken in FP64 from the FP32 target position, the node's
// exact FP32 box and FP64 centre, as in the definition; the contributions
// are FP32 with per-leaf sums accumulated in FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "tree.h"

namespace gs {

namespace {

typedef unsigned long long u64;
constexpr int kStack = 192;  // > 7 siblings x 22 levels + 8

__device__ inline bool decide(const BhNode &nd, double x, double y, double z,
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

enum Mode { MODE_RHS = 0, MODE_SHOOT = 1, MODE_ENERGY = 2 };

template <bool WITH_A>
__global__ __launch_bounds__(256) void k_bh_traverse(
    const BhNode *__restrict__ nodes, const float4 *__restrict__ Qs, const float4 *__restrict__ Ps,
    const unsigned *__restrict__ perm, int64_t n, BhParams bp, int mode,
    float *__restrict__ dq, float *__restrict__ dp, double *__restrict__ Sq,
    double *__restrict__ Sp, float *__restrict__ q32, float *__restrict__ p32, double dt,
    double *__restrict__ Hpart, u64 *__restrict__ counters, const TreeMeta *__restrict__ meta,
    int *__restrict__ status) {
    __shared__ int s_node[4][kStack];
    __shared__ u64 s_mask[4][kStack];
    __shared__ double s_red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = ((int64_t)blockIdx.x * 4 + wv) * 64 + lane;
    const bool active = t < n;
    const float4 xq = active ? Qs[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xp = active ? Ps[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    const double xd = xq.x, yd = xq.y, zd = xq.z;

    double V[3] = {0, 0, 0}, A[3] = {0, 0, 0};
    float mv[3] = {0.f, 0.f, 0.f}, ma[3] = {0.f, 0.f, 0.f};
    unsigned c_pairs = 0, c_mono = 0, c_visit = 0;

    int sp = 0;
    const u64 live = __ballot(active);
    if (live != 0ull) {
        s_node[wv][0] = 0;
        s_mask[wv][0] = live;
        sp = 1;
    }
    while (sp > 0) {
        --sp;
        const int k = __builtin_amdgcn_readfirstlane(s_node[wv][sp]);
        const u64 m = s_mask[wv][sp];
        const BhNode nd = nodes[k];
        const bool mine = (m >> lane) & 1ull;
        bool need = false;
        if (mine) {
            ++c_visit;
            if (decide(nd, xd, yd, zd, bp)) {
                // n_k virtual points at C_k, momentum P_k / n_k each
                const float dx = xq.x - (float)nd.cx, dy = xq.y - (float)nd.cy,
                            dz = xq.z - (float)nd.cz;
                const float g = __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * bp.negc);
                mv[0] += g * nd.px;
                mv[1] += g * nd.py;
                mv[2] += g * nd.pz;
                if (WITH_A) {
                    const float w = g * (xp.x * nd.px + xp.y * nd.py + xp.z * nd.pz);
                    ma[0] += w * dx;
                    ma[1] += w * dy;
                    ma[2] += w * dz;
                }
                ++c_mono;
            } else {
                need = true;
            }
        }
        const u64 open = __ballot(need);
        if (open == 0ull) continue;
        if (nd.nchild == 0) {
            // exact pairs with the leaf's members
            float tv[3] = {0.f, 0.f, 0.f}, ta[3] = {0.f, 0.f, 0.f};
            const int j1 = nd.first + nd.n;
            for (int j = nd.first; j < j1; ++j) {
                const float4 qj = Qs[j];
                const float4 pj = Ps[j];
                if (need) {
                    const float dx = xq.x - qj.x, dy = xq.y - qj.y, dz = xq.z - qj.z;
                    const float g =
                        __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * bp.negc);
                    tv[0] += g * pj.x;
                    tv[1] += g * pj.y;
                    tv[2] += g * pj.z;
                    if (WITH_A) {
                        const float w = g * (xp.x * pj.x + xp.y * pj.y + xp.z * pj.z);
                        ta[0] += w * dx;
                        ta[1] += w * dy;
                        ta[2] += w * dz;
                    }
                }
            }
            if (need) {
                c_pairs += (unsigned)nd.n;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    V[c] += (double)tv[c];
                    if (WITH_A) A[c] += (double)ta[c];
                }
            }
        } else {
            if (sp + nd.nchild > kStack) {
                // cannot happen for trees of at most 22 levels; stop safely
                if (lane == 0 && status) *status = 2;
                break;
            }
            for (int c = nd.nchild - 1; c >= 0; --c) {
                s_node[wv][sp] = nd.first + c;
                s_mask[wv][sp] = open;
                ++sp;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        V[c] += (double)mv[c];
        A[c] = (A[c] + (double)ma[c]) * bp.inv_s2;
    }

    // counters: wave sums, one atomic per wave (integer, order-free)
    u64 cp = c_pairs, cm = c_mono, cv = c_visit;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cp += __shfl_down(cp, off, 64);
        cm += __shfl_down(cm, off, 64);
        cv += __shfl_down(cv, off, 64);
    }
    if (lane == 0 && counters) {
        atomicAdd(&counters[0], cp);
        atomicAdd(&counters[1], cm);
        atomicAdd(&counters[2], cv);
        if (blockIdx.x == 0 && wv == 0) atomicAdd(&counters[3], (u64)meta->n_nodes);
        (void)status;
    }

    double e = 0.0;
    if (active) {
        const int64_t i = perm[t];
        if (mode == MODE_RHS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dq[3 * i + c] = (float)V[c];
                if (WITH_A) dp[3 * i + c] = (float)A[c];
            }
        } else {
            double q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                q[c] = Sq[3 * i + c];
                p[c] = Sp[3 * i + c];
            }
            e = p[0] * V[0] + p[1] * V[1] + p[2] * V[2];
            if (mode == MODE_SHOOT) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] += dt * V[c];
                    p[c] += dt * A[c];
                    Sq[3 * i + c] = q[c];
                    Sp[3 * i + c] = p[c];
                    q32[3 * i + c] = (float)q[c];
                    p32[3 * i + c] = (float)p[c];
                }
            }
        }
    }
    if (Hpart && mode != MODE_RHS) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
        if (lane == 0) s_red[wv] = e;
        __syncthreads();
        if (threadIdx.x == 0) Hpart[blockIdx.x] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
    }
}

__global__ void k_state_init(const float *__restrict__ q, const float *__restrict__ p, int64_t n3,
                             double *__restrict__ Sq, double *__restrict__ Sp,
                             float *__restrict__ q32, float *__restrict__ p32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const float a = q[i], b = p[i];
    Sq[i] = a;
    Sp[i] = b;
    q32[i] = a;
    p32[i] = b;
}

__global__ void k_state_out(const double *__restrict__ Sq, const double *__restrict__ Sp,
                            int64_t n3, float *__restrict__ q, float *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    q[i] = (float)Sq[i];
    p[i] = (float)Sp[i];
}

// Clears the status word with a kernel (no memset nodes, so the launch
// sequence can be captured in a graph).
__global__ void k_clear_status(int *__restrict__ status, u64 *__restrict__ counters) {
    if (threadIdx.x == 0) *status = 0;
    if (threadIdx.x < 4) counters[threadIdx.x] = 0ull;
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

constexpr size_t kStatusOffset = 0;  // status word at the start of the workspace

}  // namespace

int traverse_blocks(int64_t n) { return (int)nblk(n > 0 ? n : 1, 256); }

BhParams make_bh_params(const gs_params &prm) {
    BhParams b{};
    const double s = prm.sigma;
    b.negc = (float)(-1.4426950408889634074 / (2.0 * s * s));
    b.inv_s2 = 1.0 / (s * s);
    b.inv_s2f = (float)b.inv_s2;
    const double cut = prm.cutoff_sigmas * s;
    b.cut2 = cut * cut;
    b.theta_inf = std::isinf(prm.theta) ? 1 : 0;
    b.th2 = b.theta_inf ? 0.0 : prm.theta * prm.theta;
    return b;
}

gs_status launch_bh_traverse(const TreeBufs &t, const BhParams &bp, bool with_a,
                             const TraverseOut &o, unsigned long long *counters, hipStream_t s,
                             int mode, int *status) {
    const unsigned grid = (unsigned)traverse_blocks(t.n);
    const int kind = with_a ? KIND_TRAVERSE : KIND_TRAVERSE_V;
    timing_begin(kind, s);
    if (with_a)
        hipLaunchKernelGGL(k_bh_traverse<true>, dim3(grid), dim3(256), 0, s, t.nodes, t.Qs, t.Ps,
                           t.valA, t.n, bp, mode, o.dq, o.dp, o.Sq, o.Sp, o.q32, o.p32, o.dt,
                           o.Hpart, counters, t.meta, status);
    else
        hipLaunchKernelGGL(k_bh_traverse<false>, dim3(grid), dim3(256), 0, s, t.nodes, t.Qs,
                           t.Ps, t.valA, t.n, bp, mode, o.dq, o.dp, o.Sq, o.Sp, o.q32, o.p32,
                           o.dt, o.Hpart, counters, t.meta, status);
    timing_end(kind, s);
    GS_LAUNCH_CHECK("bh_traverse");
    return GS_OK;
}

gs_status launch_bh_traverse(const TreeBufs &t, const BhParams &bp, bool with_a,
                             const TraverseOut &o, unsigned long long *counters, hipStream_t s) {
    return launch_bh_traverse(t, bp, with_a, o, counters, s, MODE_RHS, nullptr);
}

ShootBhBufs layout_shoot_bh(Arena &a, int64_t n, int nt) {
    ShootBhBufs b{};
    carve_tree(a, n, b.tree);
    b.Sq = a.take<double>(3 * n);
    b.Sp = a.take<double>(3 * n);
    b.q32 = a.take<float>(3 * n);
    b.p32 = a.take<float>(3 * n);
    b.Hpart = a.take<double>((size_t)(nt + 1) * traverse_blocks(n));
    return b;
}

gs_status rhs_bh(const float *q, const float *p, int64_t n, const gs_params &prm, float *dq,
                 float *dp, TreeBufs &t, char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws + kStatusOffset);
    u64 *counters = reinterpret_cast<u64 *>(ws + 8);
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status, counters);
    GS_TRY(build_tree(q, p, n, prm.leaf_cap, t, status, s));
    TraverseOut o{};
    o.dq = dq;
    o.dp = dp;
    return launch_bh_traverse(t, make_bh_params(prm), true, o, counters, s, MODE_RHS, status);
}

gs_status shoot_bh(const float *q0, const float *p0, int64_t n, const gs_params &prm, float *q1,
                   float *p1, double *H, ShootBhBufs &b, char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws + kStatusOffset);
    u64 *counters = reinterpret_cast<u64 *>(ws + 8);
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status, counters);
    hipLaunchKernelGGL(k_state_init, dim3(nblk(3 * n)), dim3(kBlock), 0, s, q0, p0, 3 * n, b.Sq,
                       b.Sp, b.q32, b.p32);
    GS_LAUNCH_CHECK("state_init");
    const BhParams bp = make_bh_params(prm);
    const int nblk_t = traverse_blocks(n);
    TraverseOut o{};
    o.Sq = b.Sq;
    o.Sp = b.Sp;
    o.q32 = b.q32;
    o.p32 = b.p32;
    o.dt = 1.0 / prm.nt;
    for (int t = 0; t < prm.nt; ++t) {
        GS_TRY(build_tree(b.q32, b.p32, n, prm.leaf_cap, b.tree, status, s));
        o.Hpart = H ? b.Hpart + (size_t)t * nblk_t : nullptr;
        GS_TRY(launch_bh_traverse(b.tree, bp, true, o, counters, s, MODE_SHOOT, status));
    }
    if (H) {
        GS_TRY(build_tree(b.q32, b.p32, n, prm.leaf_cap, b.tree, status, s));
        o.Hpart = b.Hpart + (size_t)prm.nt * nblk_t;
        GS_TRY(launch_bh_traverse(b.tree, bp, false, o, counters, s, MODE_ENERGY, status));
        GS_TRY(launch_reduce_h(b.Hpart, nblk_t, prm.nt + 1, H, s));
    }
    hipLaunchKernelGGL(k_state_out, dim3(nblk(3 * n)), dim3(kBlock), 0, s, b.Sq, b.Sp, 3 * n, q1,
                       p1);
    GS_LAUNCH_CHECK("state_out");
    return GS_OK;
}

}  // namespace gs
