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
// (the root contains every target of its tree, so it is never approximated
// and every target opens it).  Every wave decides the root's children; the
// children of those (the nodes two levels below the root) are dealt out by
// node index, node i to wave i % nsub, and each wave takes every decision
// below its nodes, adds the monopoles, and records each leaf that some lane
// must sum exactly as an entry (leaf, lane mask) of its own list segment.
// Dealing out by index mixes the group's dense near field with far nodes in
// every wave; an earlier split, each wave taking a contiguous share of the
// root's children, left most of a group's work to the wave holding the
// group's own region (at 200k points, theta 0.5, leaf_cap 64: 1143 node
// decisions in the busiest wave against 195 on average).
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
constexpr int kBlockStack = 192;  // entries of (first child, count, lane mask, ownership)
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
TravSplit traverse_split(int64_t groups);

struct LeafEntry {
    u64 mask;
    int first;
    int count;
};

// Ownership of a block of sibling nodes among the phase-1 waves of a group.
// A block at depth d >= 0 below the root (the root's children are depth 0)
// with d < kDealDepth is decided by every wave, and wave 0 records its
// monopoles, leaves and visits; the blocks at depth kDealDepth are dealt out,
// node i to wave i % nsub; below those, a wave takes every node of its own
// subtrees.
#ifndef GS_DEAL_DEPTH
#define GS_DEAL_DEPTH 1
#endif
constexpr int kDealDepth = GS_DEAL_DEPTH;
static_assert(kDealDepth >= 1, "the root's children are decided by every wave");
constexpr int kOwnAll = -2;    // this wave's own subtree: it takes every node
constexpr int kOwnDealt = -1;  // node i belongs to wave i % nsub
// (own >= 0: a shared block at that depth)
__device__ __forceinline__ int child_ownership(int own) {
    if (own < 0) return kOwnAll;
    return own + 1 < kDealDepth ? own + 1 : kOwnDealt;
}

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

struct DecideLds {
    u64 mask[kBlockStack];
    int first[kBlockStack];
    int count[kBlockStack];
    int own[kBlockStack];
    BhNode node[8];  // the sibling block being decided
};

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
