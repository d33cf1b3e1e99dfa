// traverse.h -- work split of the Barnes-Hut traversals (forward and
// backward stage): group layout, leaf lists and partial-sum slots shared by
// traverse.hip and bh_adjoint.hip.
#pragma once

#include "tree.h"

namespace gs {
namespace trav {

typedef unsigned long long u64;

// ---------------------------------------------------------------- layout
// Work split.  A group is 64 consecutive targets of the Morton order (one
// wave's lanes).  Phase 1 walks the tree for a group with up to kSub waves
// (decide_walk below: every node is decided by one of them), which add the
// monopoles and record each leaf that some lane must sum exactly as an entry
// (leaf, lane mask) of the deciding wave's own list segment.
// Phase 2 splits the group's entries, taken segment by segment, into at
// most kMaxChunks chunks of at least kMinChunk entries and adds their exact
// pairs with one wave per chunk, so the near-field work of a dense group is
// spread over many waves.  Phase 3 adds the partial sums of a target in a
// fixed order (the phase-1 waves, then the chunks): the result does not
// depend on scheduling.
//
// How many phase-1 and phase-2 waves a group gets depends on the number of
// groups (TravSplit, chosen on the host): when there are many groups the
// launch is full anyway and splitting only adds partial sums to write and
// read back.
#ifndef GS_KSUB
#define GS_KSUB 8
#endif
constexpr int kSub = GS_KSUB;     // phase-1 waves per group, at most
constexpr int kListPerGroup = 4096;  // list entries of a group, shared out among its phase-1 waves
#ifndef GS_MAX_CHUNKS
#define GS_MAX_CHUNKS 16
#endif
#ifndef GS_MIN_CHUNK
#define GS_MIN_CHUNK 16
#endif
constexpr int kMaxChunks = GS_MAX_CHUNKS;  // phase-2 waves per group, at most
constexpr int kMinChunk = GS_MIN_CHUNK;    // entries per phase-2 wave, at least (unless fewer in all)
constexpr int kParts = kSub + kMaxChunks;

// Waves per group: nsub (<= kSub) in phase 1, each with a list segment of
// segcap = kListPerGroup / nsub entries (a leaf beyond it is summed in phase
// 1), and at most maxc (<= kMaxChunks) in phase 2.  Partial-sum slots:
// 0..nsub-1 for phase 1, then nsub + chunk.
struct TravSplit {
    int nsub, maxc, segcap;
};
TravSplit traverse_split(int64_t groups, int64_t set_points);

struct LeafEntry {
    u64 mask;
    int first;
    int count;
};

// List entries needed by at most kSparseMax of the wave's targets, of at
// most 64 points, are summed compacted (forward and backward leaf phases); the
// others by every lane.  (A leaf can exceed leaf_cap only when its points share
// one level-21 cell.)
#ifndef GS_SPARSE_MAX
#define GS_SPARSE_MAX 32
#endif
constexpr int kSparseMax = GS_SPARSE_MAX;  // a tuning build may change it (at most 32)
__device__ inline bool sparse_entry(int count, u64 mask) {
    return __popcll(mask) <= kSparseMax && count <= 64;
}

// Targets of group g: the table entry, or 64 consecutive points of one tree.
__device__ inline GroupDesc group_desc(const GroupDesc *__restrict__ gtab, int64_t g, int64_t n) {
    if (gtab) return gtab[g];
    GroupDesc d;
    d.first = (int)(g * 64);
    const int64_t r = n - g * 64;
    d.count = r < 64 ? (int)r : 64;
    d.root = 0;
    d.sub = 0;
    return d;
}

// Orders the LDS writes of this wave before its following LDS reads (all
// lanes of a wave run in lock step; this only stops compiler reordering).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- decide walk
// Phase 1 (both stages): the nsub waves of a group (one workgroup when nsub > 1)
// walk the tree level by level while the frontier is small.  The frontier is
// the list of sibling blocks that some target of the group still has to
// decide; its j-th node (counted over the blocks in order) belongs to wave
// j mod nsub, which decides it and adds the child block of an opened internal
// node to its own segment of the next level's frontier; the waves wait for
// each other (workgroup barrier) between levels.  The first level with more
// than kSegF nodes per wave ends the level walk: each wave decides its nodes
// of that level and walks below each of them depth-first on its own stack.
// Every node is decided by one wave, and which wave depends only on the tree
// and the targets, so the results do not depend on scheduling.  The walk is
// bound by the latency of each block's record load more than by the busiest
// wave: on MI355X with kSegF = 4 / 8 / 16 / 32 / 64 the 200k ellipsoids (3
// decide waves per group) took 448 / 445 / 443 / 448 / 462 us and the
// 64-subject population 763 / 747 / 752 / 762 / 794 us per forward decide
// phase, against 454 / 814 us when the nodes two levels below the root were
// dealt out by index with the levels above decided by every wave (busiest
// 200k decide wave: 790 decisions, against 675 with kSegF = 32).
#ifndef GS_SEGF
#define GS_SEGF 16
#endif
constexpr int kSegF = GS_SEGF;  // frontier blocks a wave adds per level, at most
// Depth-first entries of a wave.  Below a frontier node (depth >= 1 of at most
// 21) the stack holds at most 8 + 7 * 19 = 141 sibling blocks: the blocks of
// one node's children, then 7 waiting siblings for each level further down.
constexpr int kWalkStack = 160;

struct FrontEntry {
    u64 mask;   // targets that still decide the block
    int first;  // first node of the block
    int count;  // nodes in the block
};
struct WalkStack {
    u64 mask[kWalkStack];
    int first[kWalkStack];
    int count[kWalkStack];
};

// Workgroup shape of a decide launch: nsub waves (one group) per workgroup,
// or four groups of one wave each when nsub == 1.
__host__ __device__ inline int walk_waves(int nsub) { return nsub > 1 ? nsub : 4; }
__host__ __device__ inline int walk_groups(int nsub) { return nsub > 1 ? 1 : 4; }
// LDS of one group's frontier: two levels of nsub segments of kSegF entries,
// then the entry and node counts of each segment of both levels.
__host__ __device__ inline size_t walk_front_bytes(int nsub) {
    return (size_t)2 * nsub * kSegF * sizeof(FrontEntry) + (size_t)4 * kSub * sizeof(int);
}
// Dynamic LDS of a decide workgroup whose waves each hold a WalkStack and a
// staging area of rec_bytes (a multiple of 16).
__host__ __device__ inline size_t walk_lds_bytes(int nsub, size_t rec_bytes) {
    return (size_t)walk_waves(nsub) * (sizeof(WalkStack) + rec_bytes) +
           (size_t)walk_groups(nsub) * walk_front_bytes(nsub);
}

__device__ inline void walk_sync(bool coop) {
    if (coop)
        __syncthreads();
    else
        wave_sync();
}

// The walk of one group.  V provides
//   void load(int first, int count, int lane): stage the records of a block;
//   u64 visit(int k, u64 m, int &nfirst, int &nchild): decide node k of the
//     staged block for the targets in m (approximations, leaf entries and
//     counters are the visitor's), returning the targets that open it when
//     it is internal (its children: nfirst, nchild), else 0.
// All lanes of every wave of the group call it; coop: the group's waves
// share the workgroup (nsub > 1).  fe / fcnt / fnod: the group's frontier
// (walk_front_bytes).  Returns false when the stack overflowed (the walk of
// that wave stops; status receives kStatusOverflow).
template <class V>
__device__ __forceinline__ bool decide_walk(V &v, WalkStack &S, FrontEntry *fe, int *fcnt,
                                            int *fnod, int nsub, int sub, bool coop,
                                            int start_first, int start_count, u64 live, int lane,
                                            int *status) {
    if (lane == 0) {
        const bool has = sub == 0 && live != 0ull;
        if (has) {
            fe[0].mask = live;
            fe[0].first = start_first;
            fe[0].count = start_count;
        }
        fcnt[sub] = has ? 1 : 0;
        fnod[sub] = has ? start_count : 0;
    }
    walk_sync(coop);
    bool ok = true;
    int cur = 0;
    for (;;) {
        const FrontEntry *F = fe + cur * nsub * kSegF;
        int N = 0;
        for (int s = 0; s < nsub; ++s) N += __builtin_amdgcn_readfirstlane(fnod[cur * kSub + s]);
        if (N == 0) break;
        // wave- and group-uniform: this level's child blocks go to the next
        // frontier (each wave decides at most ceil(N / nsub) <= kSegF nodes),
        // else each wave walks below each of its nodes depth-first
        const bool level = (N + nsub - 1) / nsub <= kSegF;
        const int nxt = cur ^ 1;
        FrontEntry *out = fe + nxt * nsub * kSegF + sub * kSegF;
        int e = 0, enodes = 0, jm = 0;
        for (int s = 0; s < nsub && ok; ++s) {
            const int nb = __builtin_amdgcn_readfirstlane(fcnt[cur * kSub + s]);
            for (int b = 0; b < nb && ok; ++b) {
                const FrontEntry &f = F[s * kSegF + b];
                const int bfirst = __builtin_amdgcn_readfirstlane(f.first);
                const int bcount = __builtin_amdgcn_readfirstlane(f.count);
                const u64 m = uniform_u64(f.mask);
                // this wave's first node of the block (jm = index of the
                // block's first node in the level, mod nsub)
                int k = sub >= jm ? sub - jm : sub - jm + nsub;
                jm += bcount;
                while (jm >= nsub) jm -= nsub;
                if (k >= bcount) continue;
                v.load(bfirst, bcount, lane);
                wave_sync();
                int sp = 0;
                for (; k < bcount; k += nsub) {
                    int nf = 0, nc = 0;
                    const u64 open = v.visit(k, m, nf, nc);
                    if (open == 0ull) continue;
                    if (level) {
                        if (lane == 0) {
                            out[e].mask = open;
                            out[e].first = nf;
                            out[e].count = nc;
                        }
                        ++e;
                        enodes += nc;
                    } else {  // at most 8 entries: no overflow
                        if (lane == 0) {
                            S.mask[sp] = open;
                            S.first[sp] = nf;
                            S.count[sp] = nc;
                        }
                        ++sp;
                    }
                }
                // depth-first below this wave's nodes of the block
                while (sp > 0) {
                    wave_sync();
                    --sp;
                    const int cf = __builtin_amdgcn_readfirstlane(S.first[sp]);
                    const int cc = __builtin_amdgcn_readfirstlane(S.count[sp]);
                    const u64 cm = uniform_u64(S.mask[sp]);
                    wave_sync();
                    v.load(cf, cc, lane);
                    wave_sync();
                    for (int q = 0; q < cc; ++q) {
                        int nf = 0, nc = 0;
                        const u64 open = v.visit(q, cm, nf, nc);
                        if (open == 0ull) continue;
                        if (sp >= kWalkStack) {  // cannot happen for trees of at most 22 levels
                            if (lane == 0 && status) *status = kStatusOverflow;
                            ok = false;
                            break;
                        }
                        if (lane == 0) {
                            S.mask[sp] = open;
                            S.first[sp] = nf;
                            S.count[sp] = nc;
                        }
                        ++sp;
                    }
                    if (!ok) break;
                }
                wave_sync();
            }
        }
        if (!level || !ok) break;  // no barrier follows for any wave
        if (lane == 0) {
            fcnt[nxt * kSub + sub] = e;
            fnod[nxt * kSub + sub] = enodes;
        }
        walk_sync(coop);
        cur = nxt;
    }
    return ok;
}

// A target's (v, a) sums in a forward-traversal wave: FP32 with Kahan
// compensation (value = s - c).  Each leaf or monopole batch is summed in
// plain FP32 and then added here.
struct TAcc {
    float sV[3], cV[3], sA[3], cA[3];
};
__device__ inline void tacc_zero(TAcc &k) {
#pragma unroll
    for (int c = 0; c < 3; ++c) k.sV[c] = k.cV[c] = k.sA[c] = k.cA[c] = 0.f;
}
template <bool WITH_A>
__device__ inline void tacc_add(TAcc &k, const float *tv, const float *ta) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        kahan_add(k.sV[c], k.cV[c], tv[c]);
        if (WITH_A) kahan_add(k.sA[c], k.cA[c], ta[c]);
    }
}

// A target's compensated sums as double-float (hi, lo) partials.
__device__ inline void write_part_ff(float2 *__restrict__ part, int slot, int64_t npad,
                                     int64_t t, const TAcc &k) {
    float2 *d = part + ((int64_t)slot * npad + t) * 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const ff v = ff_fast_two_sum(k.sV[c], -k.cV[c]), a = ff_fast_two_sum(k.sA[c], -k.cA[c]);
        d[c] = make_float2(v.h, v.l);
        d[3 + c] = make_float2(a.h, a.l);
    }
}

// FP64 partials of the backward stage.
__device__ inline void write_part(double *__restrict__ part, int slot, int64_t npad, int64_t t,
                                  const double *V, const double *A) {
    double *d = part + ((int64_t)slot * npad + t) * 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = V[c];
        d[3 + c] = A[c];
    }
}

// The phase-2 split of a group: its list entries (segments 0..kSub-1 one
// after the other) in `chunks` chunks of `per` entries (the last one
// shorter).
struct ChunkSplit {
    int total, chunks, per;
};
__device__ inline ChunkSplit chunk_split(const int *__restrict__ list_n, int64_t grp,
                                         TravSplit split) {
    ChunkSplit c;
    c.total = 0;
    for (int k = 0; k < split.nsub; ++k) c.total += list_n[grp * kSub + k];
    c.chunks = (c.total + kMinChunk - 1) / kMinChunk;
    if (c.chunks > split.maxc) c.chunks = split.maxc;
    c.per = c.chunks > 0 ? (c.total + c.chunks - 1) / c.chunks : 0;
    return c;
}

// A position (segment, offset) in a group's concatenated list segments.
struct ListCursor {
    int seg, off, segn;
};
__device__ inline void list_normalize(const int *__restrict__ list_n, int64_t grp, int nsub,
                                      ListCursor &c) {
    while (c.off >= c.segn && c.seg < nsub - 1) {
        c.off -= c.segn;
        ++c.seg;
        c.segn = list_n[grp * kSub + c.seg];
    }
}
// The cursor at entry v (< the group's total) of the concatenated list.
__device__ inline ListCursor list_seek(const int *__restrict__ list_n, int64_t grp,
                                      TravSplit split, int v) {
    ListCursor c{0, v, list_n[grp * kSub]};
    list_normalize(list_n, grp, split.nsub, c);
    return c;
}
// The entry under the cursor (wave-uniform); the cursor moves to the next.
__device__ inline LeafEntry list_take(const LeafEntry *__restrict__ list,
                                      const int *__restrict__ list_n, int64_t grp,
                                      TravSplit split, ListCursor &c) {
    const LeafEntry e = list[grp * kListPerGroup + (int64_t)c.seg * split.segcap + c.off];
    ++c.off;
    list_normalize(list_n, grp, split.nsub, c);
    return e;
}

}  // namespace trav
}  // namespace gs
