// bh_adjoint.hip -- Barnes-Hut backward stage (Sec. 2.2: node statistics of
// the position and momentum derivatives; tree-averaged derivatives inside
// approximated nodes).
//
// At every backward step the octree of q_t is rebuilt, each node gets the
// FP64 sums A_k = sum alpha_i and B_k = sum beta_i of its members, and every
// target walks the tree with the forward decisions, in the three phases of
// the forward traversal (decisions and approximated nodes with the list of
// leaves to sum exactly; the leaves' exact pairs; a fixed-order combine).
// An approximated node
// acts as n_k virtual points at C_k carrying the mean momentum P_k / n_k and
// the mean derivatives A_k / n_k, B_k / n_k, which gives, with d = x - C_k,
// G = G(|d|), s = p_x . P_k, db = beta_x - B_k / n_k:
//   g_q += sigma^-2 G { -d [ P_k . alpha_x + p_x . A_k ] + s [ db - d (d . db) / sigma^2 ] }
//   g_p += G A_k + sigma^-2 G P_k (d . db)
// A leaf that is not approximated contributes the exact adjoint pairs.  The
// combine adds dt (g_q, g_p) to (alpha, beta) of its targets in place.
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "traverse.h"

namespace gs {

namespace {

using namespace trav;

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__global__ void k_clear(int *__restrict__ status, u64 *__restrict__ counters) {
    if (threadIdx.x == 0) *status = 0;
    for (int i = threadIdx.x; i < kCounterSlots * GS_BH_COUNTERS; i += blockDim.x)
        counters[i] = 0ull;
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

// Exact adjoint pairs of one leaf, sorted points [first, first + count), for
// the lanes with `mine` set; wave-uniform (scalar) source loads, the leaf
// summed in FP32 and added to the FP64 sums.
__device__ __forceinline__ void leaf_adjoint(const float4 *__restrict__ Qs,
                                             const float4 *__restrict__ Ps,
                                             const float4 *__restrict__ As,
                                             const float4 *__restrict__ Bs, int first, int count,
                                             bool mine, float4 x, float4 px, float4 ax, float4 bx,
                                             float negc, float inv_s2, double *GQ, double *GP) {
    if (!mine) return;
    float gq[3] = {0.f, 0.f, 0.f}, gp[3] = {0.f, 0.f, 0.f};
    for (int j = first; j < first + count; ++j)
        adj_pair(x, px, ax, bx, Qs[j], Ps[j], As[j], Bs[j], negc, inv_s2, gq, gp);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        GQ[c] += (double)gq[c];
        GP[c] += (double)gp[c];
    }
}

// The same with the leaf's points staged in LDS, 64 at a time: each lane
// loads one point (q, p, alpha, beta), then every lane reads them back with
// wave-uniform LDS addresses.  All lanes of the wave must call it.
__device__ __forceinline__ void leaf_adjoint_staged(
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, const float4 *__restrict__ As,
    const float4 *__restrict__ Bs, int first, int count, bool mine, float4 x, float4 px,
    float4 ax, float4 bx, float negc, float inv_s2, double *GQ, double *GP, float4 (*st)[64],
    int lane) {
    float gq[3] = {0.f, 0.f, 0.f}, gp[3] = {0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < count; j0 += 64) {
        const int cnt = count - j0 < 64 ? count - j0 : 64;
        wave_sync();
        if (lane < cnt) {
            const int j = first + j0 + lane;
            st[0][lane] = Qs[j];
            st[1][lane] = Ps[j];
            st[2][lane] = As[j];
            st[3][lane] = Bs[j];
        }
        wave_sync();
        if (mine)
            for (int j = 0; j < cnt; ++j)
                adj_pair(x, px, ax, bx, st[0][j], st[1][j], st[2][j], st[3][j], negc, inv_s2, gq,
                         gp);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        GQ[c] += (double)gq[c];
        GP[c] += (double)gp[c];
    }
}

// One wave's decisions of its group's nodes (backward stage); the records of
// a block are staged with the per-node sums A_k, B_k of alpha and beta.
struct AdjVisit {
    const BhNode *__restrict__ nodes;
    const double *__restrict__ adj;
    const float4 *__restrict__ Qc;
    const float4 *__restrict__ Ps;
    const float4 *__restrict__ As;
    const float4 *__restrict__ Bs;
    BhNode *rec;      // LDS: the staged block
    double (*radj)[6];  // LDS: its A_k, B_k
    LeafEntry *mylist;
    BhParams bp;
    float4 xp, xa, xb;
    double xd, yd, zd;
    int64_t t;
    bool active;
    int lane, segcap, nlist;
    double GQ[3], GP[3];
    u64 c_pairs, c_mono;  // wave totals (scalars)

    __device__ __forceinline__ void load(int first, int count, int l) {
        if (l < kNodeF4 * count)
            reinterpret_cast<float4 *>(rec)[l] = reinterpret_cast<const float4 *>(nodes + first)[l];
        if (l < 3 * count)
            reinterpret_cast<float4 *>(&radj[0][0])[l] =
                reinterpret_cast<const float4 *>(adj + 6 * (int64_t)first)[l];
    }
    __device__ __forceinline__ u64 visit(int k, u64 m, int &nfirst, int &nchild) {
        const bool mine = (m >> lane) & 1ull;
        const BhNode nd = rec[k];
        const int nn = __builtin_amdgcn_readfirstlane(nd.n);
        u64 approx = 0ull;
        if (nn >= 2) {  // a single point is never approximated
            double d[3];
            const bool ap = decide_far(nd, xd, yd, zd, bp, d) && mine;
            approx = __ballot(ap);
            if (ap) {
                // n_k virtual points: (C, P / n, A / n, B / n)
                const float inv_s2 = bp.inv_s2f;
                const float Ax = (float)radj[k][0], Ay = (float)radj[k][1], Az = (float)radj[k][2];
                const float inv_n = 1.f / (float)nn;
                const float mbx = (float)radj[k][3] * inv_n, mby = (float)radj[k][4] * inv_n,
                            mbz = (float)radj[k][5] * inv_n;
                const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
                const float g = __builtin_amdgcn_exp2f((dx * dx + dy * dy + dz * dz) * bp.negc);
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
            }
        }
        c_mono += (u64)__popcll(approx);
        const u64 open = m & ~approx;
        if (open == 0ull) return 0ull;
        nfirst = __builtin_amdgcn_readfirstlane(nd.first);
        nchild = __builtin_amdgcn_readfirstlane(nd.nchild);
        if (nchild > 0) return open;
        c_pairs += (u64)__popcll(open) * (u64)nn;
        if (nlist < segcap) {
            if (lane == 0) {
                LeafEntry e;
                e.mask = open;
                e.first = nfirst;
                e.count = nn;
                mylist[nlist] = e;
            }
            ++nlist;
        } else {  // segment full: sum this leaf here
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 xc = active ? Qc[t] : z4;
            leaf_adjoint(Qc, Ps, As, Bs, nfirst, nn, (open >> lane) & 1ull, xc, xp, xa, xb,
                         bp.negc, bp.inv_s2f, GQ, GP);
        }
        return 0ull;
    }
};
constexpr size_t kAdjRec = 8 * sizeof(BhNode) + 8 * 6 * sizeof(double);

// Phase 1 of the backward products (the work split and walk of the forward
// traversal): the decisions, the approximated nodes' contributions and the
// list of leaves to sum exactly.  Workgroups as k_bh_decide; dynamic LDS of
// walk_lds_bytes(nsub, kAdjRec).
// 6 waves per SIMD (80 VGPRs): with 5 / 7 / 8 the 50k gradient's backward
// decide phase measured 143 / 177 / 322 us against 138 us.
#ifndef GS_ADJ_DECIDE_WAVES
#define GS_ADJ_DECIDE_WAVES 6
#endif
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(GS_ADJ_DECIDE_WAVES, GS_ADJ_DECIDE_WAVES))) void k_adj_decide(
    const BhNode *__restrict__ nodes, const double *__restrict__ adj,
    const float4 *__restrict__ Qs, const float4 *__restrict__ Qc,
    const float4 *__restrict__ Ps, const float4 *__restrict__ As,
    const float4 *__restrict__ Bs, int64_t n, const GroupDesc *__restrict__ gtab, int64_t groups,
    TravSplit split, BhParams bp, LeafEntry *__restrict__ list, int *__restrict__ list_n,
    double *__restrict__ part, u64 *__restrict__ counters, int *__restrict__ status) {
    extern __shared__ __align__(16) char walk_lds[];
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const int nsub = split.nsub;
    const bool coop = nsub > 1;
    const int64_t grp = coop ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * 4 + wv;
    const int sub = coop ? wv : 0;
    if (grp >= groups) return;  // only when !coop (a whole group per workgroup otherwise)
    char *wbase = walk_lds + (size_t)wv * (sizeof(WalkStack) + kAdjRec);
    char *fbase = walk_lds + (size_t)walk_waves(nsub) * (sizeof(WalkStack) + kAdjRec) +
                  (size_t)(coop ? 0 : wv) * walk_front_bytes(nsub);
    WalkStack &S = *reinterpret_cast<WalkStack *>(wbase);
    FrontEntry *fe = reinterpret_cast<FrontEntry *>(fbase);
    int *fcnt = reinterpret_cast<int *>(fbase + (size_t)2 * nsub * kSegF * sizeof(FrontEntry));
    int *fnod = fcnt + 2 * kSub;

    const int64_t npad = groups * 64;
    const GroupDesc gd = group_desc(gtab, grp, n);
    AdjVisit vis;
    vis.nodes = nodes;
    vis.adj = adj;
    vis.Qc = Qc;
    vis.Ps = Ps;
    vis.As = As;
    vis.Bs = Bs;
    vis.rec = reinterpret_cast<BhNode *>(wbase + sizeof(WalkStack));
    vis.radj = reinterpret_cast<double(*)[6]>(wbase + sizeof(WalkStack) + 8 * sizeof(BhNode));
    vis.mylist = list + grp * kListPerGroup + (int64_t)sub * split.segcap;
    vis.bp = bp;
    vis.t = (int64_t)gd.first + lane;
    vis.active = lane < gd.count;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xs = vis.active ? Qs[vis.t] : z4;
    vis.xp = vis.active ? Ps[vis.t] : z4;
    vis.xa = vis.active ? As[vis.t] : z4;
    vis.xb = vis.active ? Bs[vis.t] : z4;
    vis.xd = xs.x;
    vis.yd = xs.y;
    vis.zd = xs.z;
    vis.lane = lane;
    vis.segcap = split.segcap;
    vis.nlist = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) vis.GQ[c] = vis.GP[c] = 0.0;
    vis.c_pairs = vis.c_mono = 0;

    // the first block: the root's children, or the root itself when it is a leaf
    const int rchild = __builtin_amdgcn_readfirstlane(nodes[gd.root].nchild);
    const int rfirst = __builtin_amdgcn_readfirstlane(nodes[gd.root].first);
    const u64 live = __ballot(vis.active);
    decide_walk(vis, S, fe, fcnt, fnod, nsub, sub, coop, rchild == 0 ? gd.root : rfirst,
                rchild == 0 ? 1 : rchild, live, lane, status);
    write_part(part, sub, npad, grp * 64 + lane, vis.GQ, vis.GP);
    if (lane == 0) list_n[grp * kSub + sub] = vis.nlist;
    if (lane == 0 && counters && (vis.c_pairs != 0 || vis.c_mono != 0)) {
        u64 *c = counter_slot(counters, blockIdx.x);
        if (vis.c_pairs) atomicAdd(&c[0], vis.c_pairs);
        if (vis.c_mono) atomicAdd(&c[1], vis.c_mono);
    }
}

// A list entry needed by at most kSparseMax of the wave's targets, summed
// compacted (as in the forward leaf phase): with k targets in the mask and k'
// the power of two >= k, lane l takes target slot i = l mod k' (the i-th lane
// of the mask; its target data are read from that lane) and the staged
// source rows l / k' + R j, R = 64 / k'.  The R partial sums of a slot are
// added across lanes (butterfly over the row bits) and moved to the target's
// lane, which adds them to its FP64 sums.  All lanes of the wave call it;
// the leaf's points (count <= 64) are already staged in st.
__device__ __forceinline__ void leaf_adjoint_compact(u64 mask, int count, float4 x, float4 px,
                                                     float4 ax, float4 bx, float negc,
                                                     float inv_s2, double *GQ, double *GP,
                                                     float4 (*st)[64], int *slot, int lane) {
    const int k = __popcll(mask);
    const u64 below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const bool mine = (mask >> lane) & 1ull;
    const int rank = __popcll(mask & below);
    if (mine) slot[rank] = lane;
    wave_sync();
    const int lg = k <= 1 ? 0 : 32 - __clz(k - 1);  // k' = 2^lg >= k
    const int R = 64 >> lg;
    const int i = lane & ((1 << lg) - 1), r = lane >> lg;
    const bool valid = i < k;
    const int tl = valid ? slot[i] : lane;
    // the slot's target data, from its lane
    const float4 tx = make_float4(__shfl(x.x, tl, 64), __shfl(x.y, tl, 64), __shfl(x.z, tl, 64), 0.f);
    const float4 tp = make_float4(__shfl(px.x, tl, 64), __shfl(px.y, tl, 64), __shfl(px.z, tl, 64), 0.f);
    const float4 ta = make_float4(__shfl(ax.x, tl, 64), __shfl(ax.y, tl, 64), __shfl(ax.z, tl, 64), 0.f);
    const float4 tb = make_float4(__shfl(bx.x, tl, 64), __shfl(bx.y, tl, 64), __shfl(bx.z, tl, 64), 0.f);
    float gq[3] = {0.f, 0.f, 0.f}, gp[3] = {0.f, 0.f, 0.f};
    if (valid)
        for (int j = r; j < count; j += R)
            adj_pair(tx, tp, ta, tb, st[0][j], st[1][j], st[2][j], st[3][j], negc, inv_s2, gq, gp);
    for (int off = 1 << lg; off < 64; off <<= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gq[c] += __shfl_xor(gq[c], off, 64);
            gp[c] += __shfl_xor(gp[c], off, 64);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float vq = __shfl(gq[c], rank, 64), vp = __shfl(gp[c], rank, 64);
        if (mine) {
            GQ[c] += (double)vq;
            GP[c] += (double)vp;
        }
    }
    wave_sync();  // slot is rewritten by the next entry
}

// Phase 2: one wave per (group, chunk of its list entries), on the positions
// relative to the set's frame origin.
__global__ __launch_bounds__(256) void k_adj_leaves(
    const float4 *__restrict__ Qs, const float4 *__restrict__ Ps, const float4 *__restrict__ As,
    const float4 *__restrict__ Bs, int64_t n, const GroupDesc *__restrict__ gtab, int64_t groups,
    TravSplit split, float negc, float inv_s2, const LeafEntry *__restrict__ list,
    const int *__restrict__ list_n,
    double *__restrict__ part) {
    __shared__ float4 stage[4][4][64];
    __shared__ int slots[4][64];
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const int64_t grp = blockIdx.x;
    const int chunk = blockIdx.y * 4 + wv;
    const ChunkSplit cs = chunk_split(list_n, grp, split);
    const int v0 = chunk * cs.per;
    if (chunk >= cs.chunks || v0 >= cs.total) return;  // wave-uniform: no entries here
    const int v1 = v0 + cs.per < cs.total ? v0 + cs.per : cs.total;
    ListCursor cur = list_seek(list_n, grp, split, v0);
    const int64_t npad = groups * 64;
    const GroupDesc gd = group_desc(gtab, grp, n);
    const int64_t t = (int64_t)gd.first + lane;
    const bool active = lane < gd.count;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xq = active ? Qs[t] : z4, xp = active ? Ps[t] : z4;
    const float4 xa = active ? As[t] : z4, xb = active ? Bs[t] : z4;
    double GQ[3] = {0, 0, 0}, GP[3] = {0, 0, 0};
    for (int r = v0; r < v1; ++r) {
        const LeafEntry e = list_take(list, list_n, grp, split, cur);
        const int first = __builtin_amdgcn_readfirstlane(e.first);
        const int count = __builtin_amdgcn_readfirstlane(e.count);
        const u64 mask = uniform_u64(e.mask);
        if (sparse_entry(count, mask)) {
            wave_sync();
            if (lane < count) {
                const int j = first + lane;
                stage[wv][0][lane] = Qs[j];
                stage[wv][1][lane] = Ps[j];
                stage[wv][2][lane] = As[j];
                stage[wv][3][lane] = Bs[j];
            }
            leaf_adjoint_compact(mask, count, xq, xp, xa, xb, negc, inv_s2, GQ, GP, stage[wv],
                                 slots[wv], lane);
        } else {
            leaf_adjoint_staged(Qs, Ps, As, Bs, first, count, ((mask >> lane) & 1ull) != 0, xq,
                                xp, xa, xb, negc, inv_s2, GQ, GP, stage[wv], lane);
        }
    }
    write_part(part, split.nsub + chunk, npad, grp * 64 + lane, GQ, GP);
}

// Phase 3: fixed-order sum of a target's parts; (alpha, beta) += dt
// (sigma^-2 g_q, g_p) in original order.
__global__ __launch_bounds__(256) void k_adj_combine(
    const double *__restrict__ part, const int *__restrict__ list_n,
    const GroupDesc *__restrict__ gtab, int64_t groups, TravSplit split,
    const unsigned *__restrict__ perm, int64_t n, double inv_s2, double dt,
    double *__restrict__ al, double *__restrict__ be) {
    const int lane = threadIdx.x & 63;
    const int64_t grp = (int64_t)blockIdx.x * 4 + wave_in_block();
    if (grp >= groups) return;
    const GroupDesc gd = group_desc(gtab, grp, n);
    if (lane >= gd.count) return;
    const int64_t npad = groups * 64, slot = grp * 64 + lane;
    const int nslots = split.nsub + chunk_split(list_n, grp, split).chunks;
    double GQ[3] = {0, 0, 0}, GP[3] = {0, 0, 0};
    for (int s = 0; s < nslots; ++s) {
        const double *d = part + ((int64_t)s * npad + slot) * 6;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            GQ[c] += d[c];
            GP[c] += d[3 + c];
        }
    }
    const int64_t i = perm[(int64_t)gd.first + lane];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        al[3 * i + c] += dt * (GQ[c] * inv_s2);
        be[3 * i + c] += dt * GP[c];
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

gs_status bh_adjoint_begin(const float *q0, AdjointBufs &b, char *ws, hipStream_t s) {
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<int *>(ws),
                       reinterpret_cast<u64 *>(ws + kCountersOffset));
    GS_LAUNCH_CHECK("clear");
    // the frame of the FP32 copies: frame origins of q0, fixed for the call
    return tree_set_centres(q0, b.sh.tree, b.sh.c0, nullptr, reinterpret_cast<int *>(ws), s);
}

gs_status bh_adjoint_forward_step(AdjointBufs &b, const gs_params &prm, double dt, double *v0,
                                  char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws);
    u64 *counters = reinterpret_cast<u64 *>(ws + kCountersOffset);
    GS_TRY(launch_state_to_f32(b.Sq, b.Sp, b.sh.tree, b.sh.c0, b.sh.q32, b.sh.p32, s));
    GS_TRY(build_tree(b.sh.q32, b.sh.p32, b.n, prm.leaf_cap, b.sh.tree, status, s));
    TraverseOut o{};
    o.Sq = b.Sq;
    o.Sp = b.Sp;
    o.q32 = b.sh.q32;
    o.p32 = b.sh.p32;
    o.c0 = b.sh.c0;
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
    const int64_t n = b.n;
    TreeBufs &t = b.sh.tree;
    GS_TRY(launch_state_to_f32(sq, sp, t, b.sh.c0, b.sh.q32, b.sh.p32, s));
    GS_TRY(build_tree(b.sh.q32, b.sh.p32, n, prm.leaf_cap, t, status, s));
    hipLaunchKernelGGL(k_gather_ab, dim3(nblk(n)), dim3(kBlock), 0, s, b.al, b.be, t.perm, n,
                       b.bhadj.ALs, b.bhadj.BEs);
    GS_LAUNCH_CHECK("gather_ab");
    GS_TRY(tree_range_sums(b.bhadj.ALs, b.bhadj.BEs, t, t.adj, s));
    const BhParams bp = make_bh_params(prm);
    LeafEntry *list = reinterpret_cast<LeafEntry *>(t.list);
    const TravSplit split = traverse_split(t.groups, n / (t.nsub > 0 ? t.nsub : 1));
    timing_begin(KIND_ADJOINT, s);
    hipLaunchKernelGGL(k_adj_decide,
                       dim3((unsigned)((t.groups + walk_groups(split.nsub) - 1) /
                                       walk_groups(split.nsub))),
                       dim3((unsigned)(64 * walk_waves(split.nsub))),
                       walk_lds_bytes(split.nsub, kAdjRec), s, t.nodes, t.adj, t.Qs, t.Qc, t.Ps, b.bhadj.ALs, b.bhadj.BEs, n, t.gtab,
                       t.groups, split, bp, list, t.list_n, t.part, counters, status);
    hipLaunchKernelGGL(k_adj_leaves, dim3((unsigned)t.groups, (split.maxc + 3) / 4), dim3(256), 0, s,
                       t.Qc, t.Ps, b.bhadj.ALs, b.bhadj.BEs, n, t.gtab, t.groups, split, bp.negc,
                       bp.inv_s2f, list, t.list_n, t.part);
    hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((t.groups + 3) / 4)), dim3(256), 0, s,
                       t.part, t.list_n, t.gtab, t.groups, split, t.perm, n, bp.inv_s2, dt, b.al,
                       b.be);
    timing_end(KIND_ADJOINT, s);
    GS_LAUNCH_CHECK("bh_adjoint phases");
    return GS_OK;
}

}  // namespace gs
