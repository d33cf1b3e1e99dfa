// bh_adjoint.hip -- Barnes-Hut backward stage (Sec. 2.2: node statistics of
// the position and momentum derivatives; tree-averaged derivatives inside
// approximated nodes).
//
// At every backward step the octree of q_t is rebuilt, each node gets the
// FP64 sums A_k = sum alpha_i and B_k = sum beta_i of its members, and every
// target walks the tree with the forward decisions.  An approximated node
// acts as n_k virtual points at C_k carrying the mean momentum P_k / n_k and
// the mean derivatives A_k / n_k, B_k / n_k, which gives, with d = x - C_k,
// G = G(|d|), s = p_x . P_k, db = beta_x - B_k / n_k:
//   g_q += sigma^-2 G { -d [ P_k . alpha_x + p_x . A_k ] + s [ db - d (d . db) / sigma^2 ] }
//   g_p += G A_k + sigma^-2 G P_k (d . db)
// A leaf that is not approximated contributes the exact adjoint pairs.  The
// kernel adds dt (g_q, g_p) to (alpha, beta) of its targets in place.
#include <hip/hip_runtime.h>

#include "adjoint.h"

namespace gs {

namespace {

typedef unsigned long long u64;
constexpr int kAdjStack = 192;
constexpr int kAdjStage = 64;

struct AdjLds {
    u64 mask[kAdjStack];
    int first[kAdjStack];
    int count[kAdjStack];
    BhNode node[8];
    double adj[8][6];
    float4 lq[kAdjStage], lp[kAdjStage], la[kAdjStage], lb[kAdjStage];
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__global__ void k_clear(int *__restrict__ status, u64 *__restrict__ counters) {
    if (threadIdx.x == 0) *status = 0;
    for (int i = threadIdx.x; i < kCounterSlots * GS_BH_COUNTERS; i += blockDim.x)
        counters[i] = 0ull;
}

__global__ void k_to_f32(const double *__restrict__ a, const double *__restrict__ b, int64_t n3,
                         float *__restrict__ fa, float *__restrict__ fb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    fa[i] = (float)a[i];
    fb[i] = (float)b[i];
}

// alpha, beta (original order, FP64) -> Morton order FP32 float4
__global__ void k_gather_ab(const double *__restrict__ al, const double *__restrict__ be,
                            const unsigned *__restrict__ perm, int64_t n,
                            float4 *__restrict__ A, float4 *__restrict__ B) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = perm[t];
    A[t] = make_float4((float)al[3 * i], (float)al[3 * i + 1], (float)al[3 * i + 2], 0.f);
    B[t] = make_float4((float)be[3 * i], (float)be[3 * i + 1], (float)be[3 * i + 2], 0.f);
}

// Exact adjoint pair: source j (q, p, alpha, beta) seen from target x.
__device__ inline void adj_pair(float4 x, float4 px, float4 ax, float4 bx, float4 qj, float4 pj,
                                float4 aj, float4 bj, float negc, float inv_s2, float *gq,
                                float *gp) {
    const float dx = x.x - qj.x, dy = x.y - qj.y, dz = x.z - qj.z;
    const float g = __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * negc);
    const float s = px.x * pj.x + px.y * pj.y + px.z * pj.z;
    const float cross = pj.x * ax.x + pj.y * ax.y + pj.z * ax.z + px.x * aj.x + px.y * aj.y +
                        px.z * aj.z;
    const float dbx = bx.x - bj.x, dby = bx.y - bj.y, dbz = bx.z - bj.z;
    const float c2 = (dx * dbx + dy * dby + dz * dbz) * inv_s2;
    const float w1 = -g * fmaf(s, c2, cross);
    const float w2 = g * s;
    const float w3 = g * c2;
    // each sum as two chained FMAs
    gq[0] = fmaf(w1, dx, gq[0]);
    gq[1] = fmaf(w1, dy, gq[1]);
    gq[2] = fmaf(w1, dz, gq[2]);
    gq[0] = fmaf(w2, dbx, gq[0]);
    gq[1] = fmaf(w2, dby, gq[1]);
    gq[2] = fmaf(w2, dbz, gq[2]);
    gp[0] = fmaf(g, aj.x, gp[0]);
    gp[1] = fmaf(g, aj.y, gp[1]);
    gp[2] = fmaf(g, aj.z, gp[2]);
    gp[0] = fmaf(w3, pj.x, gp[0]);
    gp[1] = fmaf(w3, pj.y, gp[1]);
    gp[2] = fmaf(w3, pj.z, gp[2]);
}

// One wave per traversal group: `count` consecutive sorted targets from
// `first`, all in the tree whose root is node `root` (gtab null: group g is
// targets [64 g, 64 g + 64) of the single tree rooted at node 0).
__global__ __launch_bounds__(256) void k_bh_adj_traverse(
    const BhNode *__restrict__ nodes, const double *__restrict__ adj,
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, const float4 *__restrict__ As,
    const float4 *__restrict__ Bs, const unsigned *__restrict__ perm, int64_t n,
    const GroupDesc *__restrict__ gtab, int64_t groups, BhParams bp, double dt,
    double *__restrict__ al, double *__restrict__ be, u64 *__restrict__ counters,
    int *__restrict__ status) {
    __shared__ AdjLds lds_all[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    AdjLds &L = lds_all[wv];
    const int64_t grp = (int64_t)blockIdx.x * 4 + wv;
    if (grp >= groups) return;  // wave-uniform; no block barrier in this kernel
    int64_t first, count;
    int root;
    if (gtab) {
        const GroupDesc d = gtab[grp];
        first = d.first;
        count = d.count;
        root = d.root;
    } else {
        first = grp * 64;
        count = n - first < 64 ? n - first : 64;
        root = 0;
    }
    const int64_t t = first + lane;
    const bool active = lane < count;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xq = active ? Qs[t] : z4, xp = active ? Ps[t] : z4;
    const float4 xa = active ? As[t] : z4, xb = active ? Bs[t] : z4;
    const double xd = xq.x, yd = xq.y, zd = xq.z;
    const float inv_s2 = bp.inv_s2f;
    double GQ[3] = {0, 0, 0}, GP[3] = {0, 0, 0};
    unsigned c_pairs = 0, c_mono = 0;

    int sp = 0;
    const u64 live = __ballot(active);
    if (live != 0ull) {
        L.first[0] = root;
        L.count[0] = 1;
        L.mask[0] = live;
        sp = 1;
    }
    wave_sync();
    while (sp > 0) {
        --sp;
        const int bf = __builtin_amdgcn_readfirstlane(L.first[sp]);
        const int bc = __builtin_amdgcn_readfirstlane(L.count[sp]);
        const u64 m = L.mask[sp];
        // the block's node records and adjoint sums (5 + 3 float4 per node)
        if (lane < 5 * bc)
            reinterpret_cast<float4 *>(L.node)[lane] =
                reinterpret_cast<const float4 *>(nodes + bf)[lane];
        if (lane < 3 * bc)
            reinterpret_cast<float4 *>(&L.adj[0][0])[lane] =
                reinterpret_cast<const float4 *>(adj + 6 * (int64_t)bf)[lane];
        wave_sync();
        const bool mine = (m >> lane) & 1ull;
        for (int k = 0; k < bc; ++k) {
            const BhNode nd = L.node[k];
            bool need = false;
            if (mine) {
                if (decide(nd, xd, yd, zd, bp)) {
                    // n_k virtual points: (C, P / n, A / n, B / n)
                    const float Ax = (float)L.adj[k][0], Ay = (float)L.adj[k][1],
                                Az = (float)L.adj[k][2];
                    const float inv_n = 1.f / (float)nd.n;
                    const float mbx = (float)L.adj[k][3] * inv_n, mby = (float)L.adj[k][4] * inv_n,
                                mbz = (float)L.adj[k][5] * inv_n;
                    const float dx = xq.x - (float)nd.cx, dy = xq.y - (float)nd.cy,
                                dz = xq.z - (float)nd.cz;
                    const float g =
                        __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * bp.negc);
                    const float s = xp.x * nd.px + xp.y * nd.py + xp.z * nd.pz;
                    const float cross = nd.px * xa.x + nd.py * xa.y + nd.pz * xa.z + xp.x * Ax +
                                        xp.y * Ay + xp.z * Az;
                    const float dbx = xb.x - mbx, dby = xb.y - mby, dbz = xb.z - mbz;
                    const float ddb = dx * dbx + dy * dby + dz * dbz;
                    const float w1 = g * (-cross - s * ddb * inv_s2);
                    const float w2 = g * s;
                    const float w3 = g * ddb * inv_s2;
                    GQ[0] += (double)(w1 * dx + w2 * dbx);
                    GQ[1] += (double)(w1 * dy + w2 * dby);
                    GQ[2] += (double)(w1 * dz + w2 * dbz);
                    GP[0] += (double)(g * Ax + w3 * nd.px);
                    GP[1] += (double)(g * Ay + w3 * nd.py);
                    GP[2] += (double)(g * Az + w3 * nd.pz);
                    ++c_mono;
                } else {
                    need = true;
                }
            }
            const u64 open = __ballot(need);
            if (open == 0ull) continue;
            const int nfirst = __builtin_amdgcn_readfirstlane(nd.first);
            const int ncount = __builtin_amdgcn_readfirstlane(nd.n);
            const int nchild = __builtin_amdgcn_readfirstlane(nd.nchild);
            if (nchild == 0) {
                if (need) c_pairs += (unsigned)ncount;
                for (int j0 = 0; j0 < ncount; j0 += kAdjStage) {
                    const int cnt = ncount - j0 < kAdjStage ? ncount - j0 : kAdjStage;
                    wave_sync();
                    if (lane < cnt) {
                        const int j = nfirst + j0 + lane;
                        L.lq[lane] = Qs[j];
                        L.lp[lane] = Ps[j];
                        L.la[lane] = As[j];
                        L.lb[lane] = Bs[j];
                    }
                    wave_sync();
                    if (need) {
                        float gq[3] = {0.f, 0.f, 0.f}, gp[3] = {0.f, 0.f, 0.f};
                        for (int j = 0; j < cnt; ++j)
                            adj_pair(xq, xp, xa, xb, L.lq[j], L.lp[j], L.la[j], L.lb[j], bp.negc,
                                     inv_s2, gq, gp);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            GQ[c] += (double)gq[c];
                            GP[c] += (double)gp[c];
                        }
                    }
                }
            } else {
                if (sp >= kAdjStack) {
                    if (lane == 0 && status) *status = 2;
                    sp = -1;
                    break;
                }
                L.first[sp] = nfirst;
                L.count[sp] = nchild;
                L.mask[sp] = open;
                ++sp;
            }
        }
        if (sp < 0) break;
        wave_sync();
    }
    if (active) {
        const int64_t i = perm[t];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            al[3 * i + c] += dt * (GQ[c] * bp.inv_s2);
            be[3 * i + c] += dt * GP[c];
        }
    }
    u64 cp = c_pairs, cm = c_mono;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cp += __shfl_down(cp, off, 64);
        cm += __shfl_down(cm, off, 64);
    }
    if (lane == 0 && counters) {
        u64 *c = counter_slot(counters, blockIdx.x);
        if (cp) atomicAdd(&c[0], cp);
        if (cm) atomicAdd(&c[1], cm);
    }
}

}  // namespace

BhAdjBufs layout_bh_adjoint(Arena &a, int64_t n) {
    BhAdjBufs b{};
    const int64_t m = n > 1 ? n : 1;
    b.ALs = a.take<float4>(m);
    b.BEs = a.take<float4>(m);
    return b;
}

gs_status bh_adjoint_begin(char *ws, hipStream_t s) {
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<int *>(ws),
                       reinterpret_cast<u64 *>(ws + kCountersOffset));
    GS_LAUNCH_CHECK("clear");
    return GS_OK;
}

gs_status bh_adjoint_forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                                  char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws);
    u64 *counters = reinterpret_cast<u64 *>(ws + kCountersOffset);
    const int64_t n3 = 3 * b.n;
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n3)), dim3(kBlock), 0, s, b.Sq, b.Sp, n3, b.sh.q32,
                       b.sh.p32);
    GS_LAUNCH_CHECK("to_f32");
    GS_TRY(build_tree(b.sh.q32, b.sh.p32, b.n, prm.leaf_cap, b.sh.tree, status, s));
    TraverseOut o{};
    o.Sq = b.Sq;
    o.Sp = b.Sp;
    o.q32 = b.sh.q32;
    o.p32 = b.sh.p32;
    o.dt = dt;
    o.Hpart = v0 ? b.hpart : nullptr;
    o.v64 = v0;
    return launch_bh_traverse(b.sh.tree, make_bh_params(prm), true, o, counters, s, MODE_SHOOT,
                              status);
}

gs_status bh_adjoint_step(AdjointBufs &b, const gs_params &prm, double dt, const double *sq,
                          const double *sp, char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws);
    u64 *counters = reinterpret_cast<u64 *>(ws + kCountersOffset);
    const int64_t n = b.n, n3 = 3 * n;
    TreeBufs &t = b.sh.tree;
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n3)), dim3(kBlock), 0, s, sq, sp, n3, b.sh.q32,
                       b.sh.p32);
    GS_LAUNCH_CHECK("to_f32");
    GS_TRY(build_tree(b.sh.q32, b.sh.p32, n, prm.leaf_cap, t, status, s));
    hipLaunchKernelGGL(k_gather_ab, dim3(nblk(n)), dim3(kBlock), 0, s, b.al, b.be, t.perm, n,
                       b.bhadj.ALs, b.bhadj.BEs);
    GS_LAUNCH_CHECK("gather_ab");
    GS_TRY(tree_range_sums(b.bhadj.ALs, b.bhadj.BEs, t, t.adj, s));
    timing_begin(KIND_ADJOINT, s);
    hipLaunchKernelGGL(k_bh_adj_traverse, dim3(nblk(t.groups, 4)), dim3(256), 0, s, t.nodes,
                       t.adj, t.Qs, t.Ps, b.bhadj.ALs, b.bhadj.BEs, t.perm, n, t.gtab, t.groups,
                       make_bh_params(prm), dt, b.al, b.be, counters, status);
    timing_end(KIND_ADJOINT, s);
    GS_LAUNCH_CHECK("bh_adj_traverse");
    return GS_OK;
}

}  // namespace gs
