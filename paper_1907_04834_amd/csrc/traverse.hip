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
// The node records of a block of siblings are staged in LDS with one vector
// load and read back as broadcasts; the decisions are taken in FP64 from the
// FP32 target position as given, the node's exact FP32 box and FP64 centre,
// as in the definition.  The contributions are FP32; each leaf's sums (and
// the wave's monopoles) are added to Kahan-compensated FP32 sums per target,
// handed to phase 3 as double-float partials: exact pairs use the positions relative to the set's
// frame origin (Qc; the box centre rounded to a multiple of a power of two,
// 0 for a set around the origin), and a monopole's offset x - C_k is taken
// in FP64 and rounded once, so no difference loses precision to the set's
// distance from the origin.  Leaf points are streamed with wave-uniform (scalar) loads; a
// leaf's sums are added only by the lanes in its mask.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>

#include "traverse.h"

// The leaf phase is compiled for 8 waves per SIMD (at most 64 VGPRs; the
// compiler moves the surplus scalar registers into VGPR lanes): against the 7
// its register use would otherwise allow, per right-hand side the 200k leaf
// phase took 309 instead of 315 us and the 64-subject population's 839
// instead of 877 us (the decide phase of the former split: 525 / 804 instead
// of 552 / 870 us).
#define GS_TRAVERSE_ATTR __attribute__((amdgpu_waves_per_eu(8, 8)))
// The decide phase of the level walk needs 70 VGPRs: held to 64 (8 waves per
// SIMD) it spills to scratch memory, and the launch then waits longer for
// its start (10.6 -> 8.6 us on average after the octree build); compiled for
// 7 waves per SIMD the 200k Barnes-Hut shooting took 38.9 instead of 39.5 ms.
#ifndef GS_DECIDE_WPE
#define GS_DECIDE_WPE 7
#endif
#define GS_DECIDE_ATTR __attribute__((amdgpu_waves_per_eu(GS_DECIDE_WPE, 8)))

namespace gs {

namespace {

using namespace trav;


// A wave-uniform value passed through readfirstlane (a no-op on it).  Used on
// the first loads of a software-pipelined source loop: the compiler otherwise
// folds "first group, or the group loaded ahead" back into one load at the
// top of the loop, and the pipeline is lost.
__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ float4 uniform_f4(float4 v) {
    return make_float4(uniform_f(v.x), uniform_f(v.y), uniform_f(v.z), uniform_f(v.w));
}

// Pair sums of B = 4 sources (FP32 partial sums of one leaf).
template <bool WITH_A, int B>
__device__ __forceinline__ void group_pairs(const float4 *qj, const float4 *pj, float4 xq,
                                            float4 xp, float negc, float *tv, float *ta) {
    float dx[B], dy[B], dz[B], g[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
        dx[u] = xq.x - qj[u].x;
        dy[u] = xq.y - qj[u].y;
        dz[u] = xq.z - qj[u].z;
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
        g[u] = __builtin_amdgcn_exp2f((dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u]) * negc);
#pragma unroll
    for (int u = 0; u < B; ++u) {
        tv[0] += g[u] * pj[u].x;
        tv[1] += g[u] * pj[u].y;
        tv[2] += g[u] * pj[u].z;
        if (WITH_A) {
            const float w = g[u] * (xp.x * pj[u].x + xp.y * pj[u].y + xp.z * pj[u].z);
            ta[0] += w * dx[u];
            ta[1] += w * dy[u];
            ta[2] += w * dz[u];
        }
    }
}

// Exact pairs of one leaf, sorted points [first, first + count), for the
// lanes with `mine` set.  first and count are wave-uniform, so the points are
// read with wave-uniform addresses (scalar loads straight into SGPRs, as in
// the all-pairs kernel); lanes outside the leaf's mask are switched off by
// the branch.  The leaf's FP32 sums go to tv, ta (zero for other lanes).
template <bool WITH_A>
__device__ __forceinline__ void leaf_direct(const float4 *__restrict__ Qs,
                                            const float4 *__restrict__ Ps, int first, int count,
                                            bool mine, float4 xq, float4 xp, float negc,
                                            float *tv, float *ta) {
#pragma unroll
    for (int c = 0; c < 3; ++c) tv[c] = ta[c] = 0.f;
    if (!mine) return;
    constexpr int B = 4;  // sources per pipeline stage
    const int end = first + count;
    int j = first;
    if (count >= B) {
        // groups of B: the next group is loaded while the current one is
        // evaluated (the last group reloads the leaf's last B points)
        float4 qn[B], pn[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            qn[u] = uniform_f4(Qs[j + u]);
            pn[u] = uniform_f4(Ps[j + u]);
        }
        for (; j + B <= end; j += B) {
            float4 qj[B], pj[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                qj[u] = qn[u];
                pj[u] = pn[u];
            }
            const int jn = j + B < end - B ? j + B : end - B;
#pragma unroll
            for (int u = 0; u < B; ++u) {
                qn[u] = Qs[jn + u];
                pn[u] = Ps[jn + u];
            }
            group_pairs<WITH_A, B>(qj, pj, xq, xp, negc, tv, ta);
        }
    }
    for (; j < end; ++j) {
        const float4 qj = Qs[j], pj = Ps[j];
        group_pairs<WITH_A, 1>(&qj, &pj, xq, xp, negc, tv, ta);
    }
}

// A group's list entries v0 <= v < v1 (of its concatenated segments) read 64
// at a time: lane l loads entry vb + l, and entry v is then taken from lane
// v - vb with readlane (v is wave-uniform), one vector load per 64 leaves.
struct EntryBatch {
    int64_t base;     // the group's first list slot
    int segn[kSub];   // segment lengths
    int nsub, segcap, vb, v1;
    int first, count, mlo, mhi;  // lane l: entry vb + l
};
__device__ inline void batch_load(EntryBatch &b, const LeafEntry *__restrict__ list, int vb,
                                  int lane) {
    b.vb = vb;
    int v = vb + lane, s = 0;
    if (v < b.v1) {
#pragma unroll
        for (int k = 0; k < kSub - 1; ++k) {  // constant indices: segn stays in registers
            if (s == k && k < b.nsub - 1 && v >= b.segn[k]) {
                v -= b.segn[k];
                s = k + 1;
            }
        }
        const LeafEntry e = list[b.base + (int64_t)s * b.segcap + v];
        b.first = e.first;
        b.count = e.count;
        b.mlo = (int)(unsigned)e.mask;
        b.mhi = (int)(unsigned)(e.mask >> 32);
    } else {
        b.first = b.count = b.mlo = b.mhi = 0;
    }
}
__device__ inline void batch_get(const EntryBatch &b, int v, int &first, int &count, u64 &mask) {
    const int i = v - b.vb;
    first = __builtin_amdgcn_readlane(b.first, i);
    count = __builtin_amdgcn_readlane(b.count, i);
    mask = ((u64)(unsigned)__builtin_amdgcn_readlane(b.mhi, i) << 32) |
           (u64)(unsigned)__builtin_amdgcn_readlane(b.mlo, i);
}


struct LeafLds {
    float4 tq[64], tp[64];  // the wave's targets (positions in the set's frame, momenta)
    float4 sq[64], sp[64];  // the sources of the sparse entry being summed
    int slot[64];           // the lanes of the entry's mask, by rank
};

// The next dense entry at or after v (v1 if none); its fields in first /
// count / mask.
__device__ inline int next_dense(EntryBatch &eb, const LeafEntry *__restrict__ list, int v,
                                 int lane, int &first, int &count, u64 &mask) {
    for (; v < eb.v1; ++v) {
        if (v - eb.vb >= 64) batch_load(eb, list, v, lane);
        batch_get(eb, v, first, count, mask);
        if (!sparse_entry(count, mask)) return v;
    }
    first = count = 0;
    mask = 0ull;
    return v;
}

__device__ inline void entry_batch_init(EntryBatch &eb, const LeafEntry *__restrict__ list,
                                        const int *__restrict__ list_n, int64_t grp,
                                        TravSplit split, int v0, int v1, int lane) {
    eb.base = grp * kListPerGroup;
    eb.nsub = split.nsub;
    eb.segcap = split.segcap;
    eb.v1 = v1;
#pragma unroll
    for (int k = 0; k < kSub; ++k) eb.segn[k] = k < split.nsub ? list_n[grp * kSub + k] : 0;
    batch_load(eb, list, v0, lane);
}

// The dense entries of [v0, v1) as one stream of source groups: the next
// group of B sources (the next dense leaf's first group at the end of a leaf)
// is loaded while the current group is evaluated.  Every lane evaluates every
// leaf and adds the leaf's FP32 sums to its compensated sums only when the leaf's
// mask holds it; per leaf the sums are those of leaf_direct (groups of B in
// order, then single sources).
template <bool WITH_A>
__device__ __forceinline__ void leaf_dense(const float4 *__restrict__ Qs,
                                           const float4 *__restrict__ Ps,
                                           const LeafEntry *__restrict__ list,
                                           const int *__restrict__ list_n, int64_t grp,
                                           TravSplit split, int v0, int v1, int lane, float4 xq,
                                           float4 xp, float negc, TAcc &K,
                                           unsigned &steps) {
    constexpr int B = 4;
    if (v0 >= v1) return;
    EntryBatch eb;
    entry_batch_init(eb, list, list_n, grp, split, v0, v1, lane);
    int first, count;
    u64 mask;
    int v = next_dense(eb, list, v0, lane, first, count, mask);
    float4 qn[B], pn[B];
    if (v < v1 && count >= B) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
            qn[u] = uniform_f4(Qs[first + u]);
            pn[u] = uniform_f4(Ps[first + u]);
        }
    }
    while (v < v1) {
        int nfirst = 0, ncount = 0;
        u64 nmask = 0ull;
        const int vn = next_dense(eb, list, v + 1, lane, nfirst, ncount, nmask);
        steps += (unsigned)count;
        const int end = first + count;
        float tv[3] = {0.f, 0.f, 0.f}, ta[3] = {0.f, 0.f, 0.f};
        int j = first;
        for (; j + B <= end; j += B) {
            float4 qj[B], pj[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                qj[u] = qn[u];
                pj[u] = pn[u];
            }
            // ahead: this leaf's next group, else the next dense leaf's first
            // group, else (nothing to load) this leaf's last B points again
            const int jn = j + 2 * B <= end ? j + B : (ncount >= B ? nfirst : end - B);
#pragma unroll
            for (int u = 0; u < B; ++u) {
                qn[u] = Qs[jn + u];
                pn[u] = Ps[jn + u];
            }
            group_pairs<WITH_A, B>(qj, pj, xq, xp, negc, tv, ta);
        }
        for (; j < end; ++j) {
            const float4 qj = Qs[j], pj = Ps[j];
            group_pairs<WITH_A, 1>(&qj, &pj, xq, xp, negc, tv, ta);
        }
        if (count < B && ncount >= B) {  // the loop above did not load ahead
#pragma unroll
            for (int u = 0; u < B; ++u) {
                qn[u] = uniform_f4(Qs[nfirst + u]);
                pn[u] = uniform_f4(Ps[nfirst + u]);
            }
        }
        if ((mask >> lane) & 1ull) tacc_add<WITH_A>(K, tv, ta);
        first = nfirst;
        count = ncount;
        mask = nmask;
        v = vn;
    }
}

// The sparse entries of [v0, v1), compacted: with k targets in the mask and
// k' the power of two >= k, lane l takes target slot i = l mod k' (the i-th
// lane of the mask) and source rows r = l / k' + R j, R = 64 / k', so R rows
// run side by side; the leaf's points are staged in LDS (the next sparse
// leaf's points are loaded while the current one is summed).  The R partial
// sums of a target are added across lanes (butterfly over the row bits) and
// moved to the target's lane, which adds them to its compensated sums.
template <bool WITH_A>
__device__ __forceinline__ void leaf_sparse(const float4 *__restrict__ Qs,
                                            const float4 *__restrict__ Ps,
                                            const LeafEntry *__restrict__ list,
                                            const int *__restrict__ list_n, int64_t grp,
                                            TravSplit split, int v0, int v1, int lane,
                                            float negc, LeafLds &L, TAcc &K,
                                            unsigned &steps) {
    if (v0 >= v1) return;
    EntryBatch eb;
    entry_batch_init(eb, list, list_n, grp, split, v0, v1, lane);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    // the first sparse entry and its points (in registers, lane l: point l)
    int v = v0, first = 0, count = 0;
    u64 mask = 0ull;
    for (; v < v1; ++v) {
        if (v - eb.vb >= 64) batch_load(eb, list, v, lane);
        batch_get(eb, v, first, count, mask);
        if (sparse_entry(count, mask)) break;
    }
    float4 rq = z4, rp = z4;
    if (v < v1 && lane < count) {
        rq = Qs[first + lane];
        rp = Ps[first + lane];
    }
    while (v < v1) {
        // stage this entry's points, then look for the next sparse entry and
        // load its points while this one is summed
        wave_sync();
        L.sq[lane] = rq;
        L.sp[lane] = rp;
        const int k = __popcll(mask);
        const u64 below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        if ((mask >> lane) & 1ull) L.slot[__popcll(mask & below)] = lane;
        int vn = v + 1, nfirst = 0, ncount = 0;
        u64 nmask = 0ull;
        for (; vn < v1; ++vn) {
            if (vn - eb.vb >= 64) batch_load(eb, list, vn, lane);
            batch_get(eb, vn, nfirst, ncount, nmask);
            if (sparse_entry(ncount, nmask)) break;
        }
        if (vn < v1 && lane < ncount) {
            rq = Qs[nfirst + lane];
            rp = Ps[nfirst + lane];
        }
        wave_sync();
        const int lg = k <= 1 ? 0 : 32 - __clz(k - 1);  // k' = 2^lg >= k
        const int R = 64 >> lg;
        const int i = lane & ((1 << lg) - 1), r = lane >> lg;
        const bool valid = i < k;
        const int tl = valid ? L.slot[i] : 0;
        const float4 xq = L.tq[tl], xp = L.tp[tl];
        float tv[3] = {0.f, 0.f, 0.f}, ta[3] = {0.f, 0.f, 0.f};
        if (valid)
            for (int j = r; j < count; j += R) {
                const float4 qj = L.sq[j], pj = L.sp[j];
                group_pairs<WITH_A, 1>(&qj, &pj, xq, xp, negc, tv, ta);
            }
        steps += (unsigned)((count + R - 1) / R);
        // add the R rows of each target slot (lanes i + k' r)
        for (int off = 1 << lg; off < 64; off <<= 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                tv[c] += __shfl_xor(tv[c], off, 64);
                if (WITH_A) ta[c] += __shfl_xor(ta[c], off, 64);
            }
        }
        // lane of mask rank s holds slot s's sums in lane s
        const int rank = __popcll(mask & below);
        const bool mine = (mask >> lane) & 1ull;
        float gv[3], ga[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gv[c] = __shfl(tv[c], rank, 64);
            ga[c] = WITH_A ? __shfl(ta[c], rank, 64) : 0.f;
        }
        if (mine) tacc_add<WITH_A>(K, gv, ga);
        v = vn;
        first = nfirst;
        count = ncount;
        mask = nmask;
    }
}

// Phase 1: decisions, monopoles and the group's list of leaves (the walk of
// decide_walk).  Every lane evaluates the decision of every node the wave
// takes (the VALU issues for the whole wave either way); the ballot
// restricted to the block's mask gives the lanes that approximate it, and the
// wave's counters are kept as scalars from the masks.
template <bool WITH_A>
struct FwdVisit {
    const BhNode *__restrict__ nodes;
    const float4 *__restrict__ Qc;
    const float4 *__restrict__ Ps;
    BhNode *rec;  // LDS: the staged block
    LeafEntry *mylist;
    BhParams bp;
    float4 xp;
    double xd, yd, zd;
    int64_t t;
    bool active;
    int lane, segcap, nlist;
    TAcc K;
    float mv[3], ma[3];
    u64 c_pairs, c_mono, c_visit;  // wave totals (scalars)
    unsigned w_steps, w_nodes;

    __device__ __forceinline__ void load(int first, int count, int l) {
        if (l < kNodeF4 * count)
            reinterpret_cast<float4 *>(rec)[l] = reinterpret_cast<const float4 *>(nodes + first)[l];
    }
    __device__ __forceinline__ u64 visit(int k, u64 m, int &nfirst, int &nchild) {
        const bool mine = (m >> lane) & 1ull;
        ++w_nodes;
        c_visit += (u64)__popcll(m);
        const BhNode nd = rec[k];
        const int nn = __builtin_amdgcn_readfirstlane(nd.n);
        u64 approx = 0ull;
        if (nn >= 2) {  // a single point is never approximated
            double d[3];
            const bool ap = decide_far(nd, xd, yd, zd, bp, d) && mine;
            approx = __ballot(ap);
            if (ap) {
                // n_k virtual points at C_k, momentum P_k / n_k each
                const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
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
        } else {
            // list full: sum this leaf here
            w_steps += (unsigned)nn;
            const float4 xc = active ? Qc[t] : make_float4(0.f, 0.f, 0.f, 0.f);
            float tv[3], ta[3];
            leaf_direct<WITH_A>(Qc, Ps, nfirst, nn, (open >> lane) & 1ull, xc, xp, bp.negc, tv,
                                ta);
            tacc_add<WITH_A>(K, tv, ta);
        }
        return 0ull;
    }
};

// Workgroups: one group of nsub waves, or (nsub == 1) four groups of one
// wave; dynamic LDS of walk_lds_bytes(nsub, 8 records).
template <bool WITH_A>
__global__ __launch_bounds__(512) GS_DECIDE_ATTR void k_bh_decide(
    const BhNode *__restrict__ nodes, const float4 *__restrict__ Qs,
    const float4 *__restrict__ Qc, const float4 *__restrict__ Ps, int64_t n, const GroupDesc *__restrict__ gtab, int64_t groups, TravSplit split, BhParams bp,
    LeafEntry *__restrict__ list, int *__restrict__ list_n, float2 *__restrict__ part,
    u64 *__restrict__ counters, const TreeTotals *__restrict__ totals, int *__restrict__ status) {
    extern __shared__ __align__(16) char walk_lds[];
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const int nsub = split.nsub;
    const bool coop = nsub > 1;
    const int64_t grp = coop ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * 4 + wv;
    const int sub = coop ? wv : 0;
    if (grp >= groups) return;  // only when !coop (a whole group per workgroup otherwise)
    constexpr size_t kRec = 8 * sizeof(BhNode);
    char *wbase = walk_lds + (size_t)wv * (sizeof(WalkStack) + kRec);
    char *fbase = walk_lds + (size_t)walk_waves(nsub) * (sizeof(WalkStack) + kRec) +
                  (size_t)(coop ? 0 : wv) * walk_front_bytes(nsub);
    WalkStack &S = *reinterpret_cast<WalkStack *>(wbase);
    FrontEntry *fe = reinterpret_cast<FrontEntry *>(fbase);
    int *fcnt = reinterpret_cast<int *>(fbase + (size_t)2 * nsub * kSegF * sizeof(FrontEntry));
    int *fnod = fcnt + 2 * kSub;

    const int64_t npad = groups * 64;
    const GroupDesc gd = group_desc(gtab, grp, n);
    FwdVisit<WITH_A> vis;
    vis.nodes = nodes;
    vis.Qc = Qc;
    vis.Ps = Ps;
    vis.rec = reinterpret_cast<BhNode *>(wbase + sizeof(WalkStack));
    vis.mylist = list + grp * kListPerGroup + (int64_t)sub * split.segcap;
    vis.bp = bp;
    vis.t = (int64_t)gd.first + lane;
    vis.active = lane < gd.count;
    const float4 xa = vis.active ? Qs[vis.t] : make_float4(0.f, 0.f, 0.f, 0.f);
    vis.xp = vis.active ? Ps[vis.t] : make_float4(0.f, 0.f, 0.f, 0.f);
    vis.xd = xa.x;
    vis.yd = xa.y;
    vis.zd = xa.z;
    vis.lane = lane;
    vis.segcap = split.segcap;
    vis.nlist = 0;
    tacc_zero(vis.K);
#pragma unroll
    for (int c = 0; c < 3; ++c) vis.mv[c] = vis.ma[c] = 0.f;
    vis.c_pairs = vis.c_mono = vis.c_visit = 0;
    vis.w_steps = vis.w_nodes = 0;

    // the first block: the root's children, or the root itself when it is a leaf
    const int rchild = __builtin_amdgcn_readfirstlane(nodes[gd.root].nchild);
    const int rfirst = __builtin_amdgcn_readfirstlane(nodes[gd.root].first);
    const u64 live = __ballot(vis.active);
    if (rchild > 0 && sub == 0) {  // the root's visit, counted once
        vis.c_visit += (u64)__popcll(live);
        ++vis.w_nodes;
    }
    decide_walk(vis, S, fe, fcnt, fnod, nsub, sub, coop, rchild == 0 ? gd.root : rfirst,
                rchild == 0 ? 1 : rchild, live, lane, status);
    tacc_add<true>(vis.K, vis.mv, vis.ma);
    write_part_ff(part, sub, npad, grp * 64 + lane, vis.K);
    if (lane == 0) list_n[grp * kSub + sub] = vis.nlist;

    // counters: one atomic per wave and counter (integer, order-free)
    const u64 c_visit = vis.c_visit;
    const unsigned w_nodes = vis.w_nodes, w_steps = vis.w_steps;
    if (lane == 0 && counters && (c_visit != 0 || w_nodes != 0)) {
        u64 *c = counter_slot(counters, blockIdx.x);
        if (vis.c_pairs) atomicAdd(&c[0], vis.c_pairs);
        if (vis.c_mono) atomicAdd(&c[1], vis.c_mono);
        atomicAdd(&c[2], c_visit);
        if (grp == 0 && sub == 0) atomicAdd(&c[3], (u64)totals->n_nodes);
        if (w_steps) atomicAdd(&c[4], (u64)w_steps);
        atomicAdd(&c[5], (u64)w_nodes);
        atomicMax(&c[6], (u64)w_steps + (u64)w_nodes);
        atomicMax(&c[7], (u64)w_nodes);
    } else if (lane == 0 && counters && grp == 0 && sub == 0) {
        atomicAdd(&counter_slot(counters, blockIdx.x)[3], (u64)totals->n_nodes);
    }
}


// Phase 2: one wave per (group, chunk of its list entries), on the positions
// relative to the set's frame origin.
template <bool WITH_A>
__global__ __launch_bounds__(256) GS_TRAVERSE_ATTR void k_bh_leaves(const float4 *__restrict__ Qc,
                                                   const float4 *__restrict__ Ps, int64_t n,
                                                   const GroupDesc *__restrict__ gtab,
                                                   int64_t groups, TravSplit split, float negc,
                                                   const LeafEntry *__restrict__ list,
                                                   const int *__restrict__ list_n,
                                                   float2 *__restrict__ part,
                                                   u64 *__restrict__ counters) {
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const int64_t grp = blockIdx.x;
    const int chunk = blockIdx.y * 4 + wv;
    const ChunkSplit cs = chunk_split(list_n, grp, split);
    const int v0 = chunk * cs.per;
    if (chunk >= cs.chunks || v0 >= cs.total) return;  // wave-uniform: no entries here
    const int v1 = v0 + cs.per < cs.total ? v0 + cs.per : cs.total;
    const int64_t npad = groups * 64;
    const GroupDesc gd = group_desc(gtab, grp, n);
    const int64_t t = (int64_t)gd.first + lane;
    const bool active = lane < gd.count;
    const float4 xq = active ? Qc[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xp = active ? Ps[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    __shared__ LeafLds lds_all[4];
    LeafLds &L = lds_all[wv];
    L.tq[lane] = xq;
    L.tp[lane] = xp;
    TAcc K;
    tacc_zero(K);
    unsigned steps = 0;
    leaf_dense<WITH_A>(Qc, Ps, list, list_n, grp, split, v0, v1, lane, xq, xp, negc, K, steps);
    leaf_sparse<WITH_A>(Qc, Ps, list, list_n, grp, split, v0, v1, lane, negc, L, K, steps);
    write_part_ff(part, split.nsub + chunk, npad, grp * 64 + lane, K);
    if (lane == 0 && counters) {
        u64 *c = counter_slot(counters, blockIdx.x, blockIdx.y);
        atomicAdd(&c[4], (u64)steps);
        atomicMax(&c[6], (u64)steps);
    }
}

// Phase 3: fixed-order double-float sum of a target's parts and the output of
// the mode.  One thread per (group, lane) slot; the energy sum of each group
// (one wave, FP64) goes to Hpart[group].
//   MODE_RHS: v and a / sigma^2 rounded to FP32 into dq, dp;
//   MODE_SHOOT: one Euler step of the state, hi+lo (Fq, Fp: the step in
//     double-float) or FP64 (Sq, Sp), and its FP32 copies q32, p32;
//   MODE_ENERGY: only p . v (and v into v64 when given).
template <bool WITH_A>
__global__ __launch_bounds__(256) void k_bh_combine(
    const float2 *__restrict__ part, const int *__restrict__ list_n,
    const GroupDesc *__restrict__ gtab, int64_t groups, TravSplit split,
    const unsigned *__restrict__ perm, int64_t n, double inv_s2, ff inv_s2f, int mode,
    float *__restrict__ dq, float *__restrict__ dp, const float2 *__restrict__ Fq,
    const float2 *__restrict__ Fp, float2 *__restrict__ Fq_out, float2 *__restrict__ Fp_out,
    const unsigned *__restrict__ ord_in, unsigned *__restrict__ ord_out,
    double *__restrict__ Sq, double *__restrict__ Sp,
    float *__restrict__ q32, float *__restrict__ p32, const double *__restrict__ c0,
    const float2 *__restrict__ c0f, double dt, ff dtf, double *__restrict__ Hpart,
    double *__restrict__ v64) {
    const int lane = threadIdx.x & 63;
    const int64_t grp = (int64_t)blockIdx.x * 4 + wave_in_block();
    if (grp >= groups) return;  // wave-uniform; no block barrier below
    const int64_t npad = groups * 64;
    const int64_t slot = grp * 64 + lane;
    const GroupDesc gd = group_desc(gtab, grp, n);
    double e = 0.0;
    if (lane < gd.count) {
        const int nslots = split.nsub + chunk_split(list_n, grp, split).chunks;
        ff acc[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] = ff{0.f, 0.f};
        for (int s = 0; s < nslots; ++s) {
            const float2 *d = part + ((int64_t)s * npad + slot) * 6;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                if (c >= 3 && !WITH_A) break;
                const float2 u = d[c];
                acc[c] = ff_add(acc[c], ff{u.x, u.y});
            }
        }
        // k: the point's index in the order the tree was built from (the
        // state's order); i: its original index
        const int64_t j = (int64_t)gd.first + lane, k = perm[j];
        const int64_t i = ord_in ? (int64_t)ord_in[k] : k;
        double V[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) V[c] = (double)acc[c].h + (double)acc[c].l;
        if (v64)
#pragma unroll
            for (int c = 0; c < 3; ++c) v64[3 * i + c] = V[c];
        if (mode == MODE_RHS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dq[3 * i + c] = acc[c].h + acc[c].l;
                if (WITH_A) {
                    const ff a = ff_mul(acc[3 + c], inv_s2f);
                    dp[3 * i + c] = a.h + a.l;
                }
            }
        } else if (Fq) {  // hi+lo state, in the order the tree was built from
            ff q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float2 fq = Fq[3 * k + c], fp = Fp[3 * k + c];
                q[c] = ff{fq.x, fq.y};
                p[c] = ff{fp.x, fp.y};
                e += ((double)p[c].h + (double)p[c].l) * V[c];
            }
            if (mode == MODE_SHOOT) {  // advanced state in this tree's sorted order
                const float2 *cs = c0f + 3 * gd.sub;  // the shooting's frame of this set
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] = ff_add(q[c], ff_mul(dtf, acc[c]));
                    if (WITH_A) p[c] = ff_add(p[c], ff_mul(dtf, ff_mul(acc[3 + c], inv_s2f)));
                    Fq_out[3 * j + c] = make_float2(q[c].h, q[c].l);
                    Fp_out[3 * j + c] = make_float2(p[c].h, p[c].l);
                    const ff r = ff_add(q[c], ff{-cs[c].x, -cs[c].y});
                    q32[3 * j + c] = r.h + r.l;
                    p32[3 * j + c] = p[c].h + p[c].l;
                }
                ord_out[j] = (unsigned)i;
            }
        } else {  // FP64 state
            double q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                q[c] = Sq[3 * i + c];
                p[c] = Sp[3 * i + c];
            }
            e = p[0] * V[0] + p[1] * V[1] + p[2] * V[2];
            if (mode == MODE_SHOOT) {
                const double *cs = c0 + 3 * gd.sub;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double a = WITH_A ? ((double)acc[3 + c].h + (double)acc[3 + c].l) : 0.0;
                    q[c] += dt * V[c];
                    p[c] += dt * (a * inv_s2);
                    Sq[3 * i + c] = q[c];
                    Sp[3 * i + c] = p[c];
                    q32[3 * i + c] = (float)(q[c] - cs[c]);
                    p32[3 * i + c] = (float)p[c];
                }
            }
        }
    }
    if (Hpart && mode != MODE_RHS) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
        if (lane == 0) Hpart[grp] = e;
    }
}

// Clears the status word with a kernel (no memset nodes, so the launch
// sequence can be captured in a graph).
__global__ void k_clear_status(int *__restrict__ status, u64 *__restrict__ counters) {
    if (threadIdx.x == 0) *status = 0;
    for (int i = threadIdx.x; i < kCounterSlots * GS_BH_COUNTERS; i += blockDim.x)
        counters[i] = 0ull;
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

constexpr size_t kStatusOffset = 0;  // status word at the start of the workspace

}  // namespace

size_t traverse_list_bytes(int64_t groups) {
    return (size_t)groups * kListPerGroup * sizeof(LeafEntry);
}

size_t traverse_count_ints(int64_t groups) { return (size_t)groups * kSub; }

// Phase-1 waves aim at about kDecideWaves waves in all (1.5 per wave slot of
// the chip at 8 per SIMD), phase-2 waves at kLeafWaves; sweeps on the 200k
// ellipsoids and on the 64-subject population found these best (200k decide
// phase with 3 / 4 / 6 / 8 waves per group: 444 / 400 / 433 / 446 us; the
// population, at 1 wave per group, took 781 instead of 753 us with 2; other
// values are compiled only by a tuning build).
#ifndef GS_DECIDE_WAVES
#define GS_DECIDE_WAVES 12288
#endif
#ifndef GS_LEAF_WAVES
#define GS_LEAF_WAVES 65536
#endif
constexpr int64_t kDecideWaves = GS_DECIDE_WAVES;
constexpr int64_t kLeafWaves = GS_LEAF_WAVES;

namespace trav {
// Sets of fewer than 4096 points on average (shallow trees) take at most 4
// decide waves per group: 64 subjects of 500-2000 points shot in 8.69 ms
// with at most 4, 8.76 ms with 2 and 9.47 ms with 8 (40 steps).
#ifndef GS_SMALL_SET_NSUB
#define GS_SMALL_SET_NSUB 4
#endif
TravSplit traverse_split(int64_t groups, int64_t set_points) {
    const int64_t g = groups > 0 ? groups : 1;
    TravSplit split;
    split.nsub = (int)std::min<int64_t>(kSub, std::max<int64_t>(1, (kDecideWaves + g - 1) / g));
    if (set_points < 4096) split.nsub = std::min(split.nsub, GS_SMALL_SET_NSUB);
    split.maxc = (int)std::min<int64_t>(kMaxChunks, std::max<int64_t>(1, (kLeafWaves + g - 1) / g));
    split.segcap = kListPerGroup / split.nsub;
    return split;
}
}  // namespace trav

size_t traverse_part_doubles(int64_t groups) { return (size_t)kParts * groups * 64 * 6; }

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
    const int64_t groups = t.groups;
    if (groups <= 0) return GS_OK;
    LeafEntry *list = reinterpret_cast<LeafEntry *>(t.list);
    const int kind = with_a ? KIND_TRAVERSE : KIND_TRAVERSE_V;
    const TravSplit split = traverse_split(groups, t.n / (t.nsub > 0 ? t.nsub : 1));
    // the partial sums of this traversal are double-float pairs (the buffer
    // holds the backward stage's FP64 partials, of the same size)
    float2 *part = reinterpret_cast<float2 *>(t.part);
    const ff inv_s2f = ff_from_double(bp.inv_s2), dtf = ff_from_double(o.dt);
    const dim3 g1((unsigned)((groups + walk_groups(split.nsub) - 1) / walk_groups(split.nsub))),
        b1((unsigned)(64 * walk_waves(split.nsub))), g2((unsigned)groups, (split.maxc + 3) / 4),
        g3((unsigned)((groups + 3) / 4));
    const size_t lds1 = walk_lds_bytes(split.nsub, 8 * sizeof(BhNode));
    timing_begin(kind, s);
#define GS_PHASES(A)                                                                         \
    do {                                                                                     \
        hipLaunchKernelGGL(k_bh_decide<A>, g1, b1, lds1, s, t.nodes, t.Qs, t.Qc, t.Ps,        \
                           t.n, t.gtab, groups, split, bp, list, t.list_n, part, counters,     \
                           t.totals, status);                                               \
        hipLaunchKernelGGL(k_bh_leaves<A>, g2, dim3(256), 0, s, t.Qc, t.Ps, t.n, t.gtab,      \
                           groups, split, bp.negc, list, t.list_n, part, counters);            \
        hipLaunchKernelGGL(k_bh_combine<A>, g3, dim3(256), 0, s, part, t.list_n, t.gtab,      \
                           groups, split, t.perm, t.n, bp.inv_s2, inv_s2f, mode, o.dq, o.dp,   \
                           o.Fq, o.Fp, o.Fq_out, o.Fp_out, o.ord_in, o.ord_out, o.Sq, o.Sp,    \
                           o.q32, o.p32, o.c0, o.c0f, o.dt, dtf, o.Hpart, o.v64);            \
    } while (0)
    if (with_a)
        GS_PHASES(true);
    else
        GS_PHASES(false);
#undef GS_PHASES
    timing_end(kind, s);
    GS_LAUNCH_CHECK("bh_traverse");
    return GS_OK;
}

gs_status launch_bh_traverse(const TreeBufs &t, const BhParams &bp, bool with_a,
                             const TraverseOut &o, unsigned long long *counters, hipStream_t s) {
    return launch_bh_traverse(t, bp, with_a, o, counters, s, MODE_RHS, nullptr);
}

static void carve_state(Arena &a, int64_t n, int nt, int state, ShootBhBufs &b) {
    b.c0 = a.take<double>(3 * (size_t)b.tree.nsub);
    if (state == kStateFF) {
        b.c0f = a.take<float2>(3 * (size_t)b.tree.nsub);
        b.Fq = a.take<float2>(3 * n);
        b.Fp = a.take<float2>(3 * n);
        b.Fq2 = a.take<float2>(3 * n);
        b.Fp2 = a.take<float2>(3 * n);
        b.ord = a.take<unsigned>(n);
        b.ord2 = a.take<unsigned>(n);
    } else {
        b.Sq = a.take<double>(3 * n);
        b.Sp = a.take<double>(3 * n);
    }
    b.q32 = a.take<float>(3 * n);
    b.p32 = a.take<float>(3 * n);
    b.Hpart = a.take<double>((size_t)(nt + 1) * (b.tree.groups > 0 ? b.tree.groups : 1));
}

ShootBhBufs layout_shoot_bh(Arena &a, int64_t n, int nt, int state) {
    ShootBhBufs b{};
    carve_tree(a, n, b.tree);
    carve_state(a, n, nt, state, b);
    b.gseg = nullptr;
    return b;
}

ShootBhBufs layout_shoot_forest(Arena &a, int64_t n, int nsub, int64_t groups, int64_t max_set,
                                int nt, int state) {
    ShootBhBufs b{};
    carve_forest(a, n, nsub, groups, max_set, b.tree);
    carve_state(a, n, nt, state, b);
    b.gseg = nullptr;
    return b;
}

gs_status rhs_bh(const float *q, const float *p, int64_t n, const gs_params &prm, float *dq,
                 float *dp, TreeBufs &t, char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws + kStatusOffset);
    u64 *counters = reinterpret_cast<u64 *>(ws + kCountersOffset);
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(256), 0, s, status, counters);
    GS_TRY(build_tree(q, p, n, prm.leaf_cap, t, status, s));
    TraverseOut o{};
    o.dq = dq;
    o.dp = dp;
    return launch_bh_traverse(t, make_bh_params(prm), true, o, counters, s, MODE_RHS, status);
}

namespace {

// q = hi + lo of a state held in sorted order, rounded to FP32, at the
// original index ord[j] of each sorted point j.
__global__ void k_unpack_sorted(const float2 *__restrict__ Fq, const float2 *__restrict__ Fp,
                                const unsigned *__restrict__ ord, int64_t n,
                                float *__restrict__ q, float *__restrict__ p) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t i = ord ? (int64_t)ord[j] : j;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        q[3 * i + c] = Fq[3 * j + c].x + Fq[3 * j + c].y;
        p[3 * i + c] = Fp[3 * j + c].x + Fp[3 * j + c].y;
    }
}

gs_status launch_unpack_sorted(const float2 *Fq, const float2 *Fp, const unsigned *ord,
                               int64_t n, float *q, float *p, hipStream_t s) {
    if (n <= 0) return GS_OK;
    hipLaunchKernelGGL(k_unpack_sorted, dim3(nblk(n)), dim3(kBlock), 0, s, Fq, Fp, ord, n, q, p);
    GS_LAUNCH_CHECK("unpack sorted state");
    return GS_OK;
}

}  // namespace

gs_status shoot_bh(const float *q0, const float *p0, int64_t n, const gs_params &prm, float *q1,
                   float *p1, double *H, ShootBhBufs &b, char *ws, hipStream_t s) {
    int *status = reinterpret_cast<int *>(ws + kStatusOffset);
    u64 *counters = reinterpret_cast<u64 *>(ws + kCountersOffset);
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(256), 0, s, status, counters);
    // the FP32 copies that every step's tree and pairs are built from are kept
    // relative to the frame origin of q0 (fixed for the call), so their rounding
    // does not depend on where the set lies
    GS_TRY(tree_set_centres(q0, b.tree, b.c0, b.c0f, status, s));
    GS_TRY(launch_state_init(q0, p0, b.tree, b.c0, b.c0f, nullptr, nullptr, b.Fq, b.Fp, b.q32,
                             b.p32, s));
    const BhParams bp = make_bh_params(prm);
    const int64_t ng = b.tree.groups;
    // Each step leaves the state, q32 and p32 in the order of its tree
    // (ping-pong buffers), so the next build gathers points that are nearly
    // in order already and the combine reads and writes the state in order.
    float2 *fq = b.Fq, *fp = b.Fp, *fq_next = b.Fq2, *fp_next = b.Fp2;
    unsigned *ord = nullptr, *ord_next = b.ord, *ord_free = b.ord2;
    TraverseOut o{};
    o.q32 = b.q32;
    o.p32 = b.p32;
    o.c0 = b.c0;
    o.c0f = b.c0f;
    o.dt = 1.0 / prm.nt;
    for (int t = 0; t < prm.nt; ++t) {
        GS_TRY(build_tree(b.q32, b.p32, n, prm.leaf_cap, b.tree, status, s));
        o.Hpart = H ? b.Hpart + (size_t)t * ng : nullptr;
        o.Fq = fq;
        o.Fp = fp;
        o.Fq_out = fq_next;
        o.Fp_out = fp_next;
        o.ord_in = ord;
        o.ord_out = ord_next;
        GS_TRY(launch_bh_traverse(b.tree, bp, true, o, counters, s, MODE_SHOOT, status));
        std::swap(fq, fq_next);
        std::swap(fp, fp_next);
        unsigned *spare = ord ? ord : ord_free;
        ord = ord_next;
        ord_next = spare;
    }
    o.Fq = fq;
    o.Fp = fp;
    o.Fq_out = o.Fp_out = nullptr;
    o.ord_in = ord;
    o.ord_out = nullptr;
    if (H) {
        GS_TRY(build_tree(b.q32, b.p32, n, prm.leaf_cap, b.tree, status, s));
        o.Hpart = b.Hpart + (size_t)prm.nt * ng;
        GS_TRY(launch_bh_traverse(b.tree, bp, false, o, counters, s, MODE_ENERGY, status));
        GS_TRY(launch_reduce_h_seg(b.Hpart, ng, b.gseg, b.tree.nsub, prm.nt + 1, H, s));
    }
    return launch_unpack_sorted(fq, fp, ord, n, q1, p1, s);
}

}  // namespace gs
