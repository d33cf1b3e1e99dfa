// internal.h -- declarations shared by the HIP translation units of the
// geodesic-shooting library (kernel launchers, workspace layout, errors).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "gs.h"

namespace gs {

// Index of the calling wave in its block as a wave-uniform value: the compiler
// does not prove threadIdx.x >> 6 uniform, and addresses derived from it would
// otherwise be computed per lane and loaded through the vector memory path.
__device__ inline int wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------------- double-float
// A value held as an unevaluated sum hi + lo of two FP32 numbers (|lo| at most
// half an ulp of hi once normalised): about 48 significant bits from FP32
// arithmetic.  The building blocks are Knuth's TwoSum (the exact rounding
// error of a sum), Dekker's Fast2Sum (the same when |a| >= |b|) and the exact
// product error given by one fused multiply-add.  None of these contains a
// product that the compiler could contract, except where fmaf is meant.
struct ff {
    float h, l;
};
__host__ __device__ inline ff ff_two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline ff ff_fast_two_sum(float a, float b) {
    const float s = a + b;
    return {s, b - (s - a)};
}
__host__ __device__ inline ff ff_add(ff x, ff y) {
    ff s = ff_two_sum(x.h, y.h);
    s.l += x.l + y.l;
    return ff_fast_two_sum(s.h, s.l);
}
__host__ __device__ inline ff ff_add(ff x, float y) {
    ff s = ff_two_sum(x.h, y);
    s.l += x.l;
    return ff_fast_two_sum(s.h, s.l);
}
__device__ inline ff ff_mul(ff x, ff y) {
    const float p = x.h * y.h;
    float e = fmaf(x.h, y.h, -p);
    e = fmaf(x.h, y.l, e);
    e = fmaf(x.l, y.h, e);
    return ff_fast_two_sum(p, e);
}
// The double-float nearest a double (host side: kernel parameters).
inline ff ff_from_double(double x) {
    const float h = (float)x;
    return {h, (float)(x - (double)h)};
}
// Kahan's compensated sum in FP32: s holds the sum, c the negated error that
// the next addition feeds back; the sum is s - c.
__device__ inline void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
gs_status hip_fail(hipError_t e, const char *what);

#define GS_HIP(call)                                       \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)
#define GS_TRY(x)                     \
    do {                              \
        gs_status st_ = (x);          \
        if (st_ != GS_OK) return st_; \
    } while (0)
#define GS_LAUNCH_CHECK(what)                              \
    do {                                                   \
        hipError_t e_ = hipGetLastError();                 \
        if (e_ != hipSuccess) return hip_fail(e_, what);   \
    } while (0)

// ---------------------------------------------------------------- timing
enum TimedKind {
    KIND_EXACT = 0,       // exact all-pairs kernel, (v, a)
    KIND_TRAVERSE = 1,    // Barnes-Hut traversal, (v, a)
    KIND_ADJOINT = 2,     // adjoint pair kernels
    KIND_TREE = 3,        // whole octree build (all its launches)
    KIND_EXACT_V = 4,     // exact all-pairs kernel, velocity only
    KIND_TRAVERSE_V = 5,  // Barnes-Hut traversal, velocity only
    KIND_COUNT = 6
};
// Bracket a launch of a timed kernel (no-ops unless timing is enabled).
void timing_begin(int kind, hipStream_t s);
void timing_end(int kind, hipStream_t s);

// ---------------------------------------------------------------- workspace
// A bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Arena {
    char *base;
    size_t off;
    size_t cap;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

constexpr int kTile = 64;       // sources per compensated tile (exact FP32 kernel)

// Workspace header: the status word at offset 0 and the Barnes-Hut counters
// at kCountersOffset, kCounterSlots copies of the GS_BH_COUNTERS values (a
// block adds into the copy of its slot; readers sum the copies, and take
// the largest for the per-wave maximum), so that the counter atomics of a
// launch do not all meet on the same addresses.
constexpr int kCounterSlots = 64;
constexpr size_t kCountersOffset = 256;
constexpr size_t kWsHeader = kCountersOffset + (size_t)kCounterSlots * GS_BH_COUNTERS * 8;
constexpr int kBlock = 256;     // threads per block for O(N) kernels

// Values of the device status word (workspace offset 0).
constexpr int kStatusNonfinite = 1;  // a coordinate was NaN or infinite (tree path)
constexpr int kStatusOverflow = 2;   // a traversal stack overflowed (cannot happen for
                                     // trees of at most 22 levels)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- exact path
// Work items of the exact FP32 kernel.  One work item is one block of
// kItemGroups x kItemSplit waves: kItemGroups groups of 64 consecutive target
// rows, each against one chunk of source rows split among kItemSplit waves
// whose sums are added in LDS, so the chunk count (the partial slots per
// target) is kItemSplit times smaller than with one wave per chunk.  The
// defaults are the measured best; other shapes are compiled only by a tuning
// build.
#ifndef GS_ITEM_GROUPS
#define GS_ITEM_GROUPS 1
#endif
#ifndef GS_ITEM_SPLIT
#define GS_ITEM_SPLIT 4
#endif
constexpr int kItemGroups = GS_ITEM_GROUPS;
constexpr int kItemSplit = GS_ITEM_SPLIT;
constexpr int kItemRows = 64 * kItemGroups;                  // target rows per item
constexpr int kItemThreads = kItemRows * kItemSplit;
constexpr int kMinWaveSources = 256;    // sources per wave of an item, at least
// Work items per launch the chunk length aims at.  At 200k points 24576
// gives 8 chunks, one per XCD; 12288 gives 4, each shared by 2 XCDs, which
// writes half the partial sums (83.5 against 134.6 MB of HBM traffic per
// launch) but measured 13.12 against 12.93 ms per RHS over 120 launches.
constexpr int64_t kItemsDefault = 24576;
constexpr int kXcds = 8;                // MI355X: workgroups are dealt to 8 XCDs in turn
static_assert(kItemThreads <= 1024, "work item too large");

// Work items of one point set without tables: the ones plan_exact_batch
// gives for offsets {0, n}, computed from this geometry.
struct ItemGeom {
    int n;     // points
    int ng;    // target groups of kItemRows rows
    int nch;   // source chunks (partial slots)
    int csz;   // sources per chunk (multiple of kTile)
    int sp;    // sources padded to kTile
    int qlen;  // items in the queue of XCD 0 (the longest)
    int rep;   // XCDs sharing each chunk (1 when nch >= kXcds, else kXcds / pw)
    int pw;    // nch rounded up to a power of two (when rep > 1)
    int gpp;   // target groups per XCD of a shared chunk
};
// Row blocks of 256 rows of one point set without tables.
struct RowGeom {
    int n;      // points
    int slots;  // partial slots
};

// Work item b: (first target row, source rows [j0, j1), slot); slot -1 is a
// padding item.  Source chunk c of a single set has home XCD c % 8 (equal
// chunks, largest first, least-loaded XCD); XCD x's queue holds its chunks'
// items chunk by chunk, and item b comes from the queue of XCD b % 8.  With
// fewer chunks than XCDs, chunk c has the rep homes c + pw r, and home r
// takes target groups [r gpp, (r + 1) gpp).
__device__ inline int4 work_item(const int4 *__restrict__ items, const ItemGeom &g, int64_t b) {
    if (items) return items[b];
    const int x = (int)(b % kXcds), k = (int)(b / kXcds);
    if (g.rep > 1) {
        const int c = x % g.pw, grp = (x / g.pw) * g.gpp + k;
        if (c >= g.nch || k >= g.gpp || grp >= g.ng) return make_int4(0, 0, 0, -1);
        const int j0 = c * g.csz;
        const int j1 = j0 + g.csz < g.sp ? j0 + g.csz : g.sp;
        return make_int4(grp * kItemRows, j0, j1, c);
    }
    if (x >= g.nch) return make_int4(0, 0, 0, -1);
    const int nq = (g.nch - x + kXcds - 1) / kXcds;
    if (k >= nq * g.ng) return make_int4(0, 0, 0, -1);
    const int c = x + kXcds * (k / g.ng), grp = k % g.ng;
    const int j0 = c * g.csz;
    const int j1 = j0 + g.csz < g.sp ? j0 + g.csz : g.sp;
    return make_int4(grp * kItemRows, j0, j1, c);
}
// Row block b: (first real point, real rows in it, set, partial slots).
__device__ inline int4 row_block(const int4 *__restrict__ blk, const RowGeom &r, int64_t b) {
    if (blk) return blk[b];
    const int first = (int)(256 * b);
    const int cnt = r.n - first < 256 ? r.n - first : 256;
    return make_int4(first, cnt, 0, r.slots);
}

// Evaluation plan of independent point sets (subjects) stored one after the
// other ([offsets[s], offsets[s+1]) is set s), or of the velocity field (m
// targets, n sources).  Rows are padded per set to whole blocks of 256.
struct ExactBatchPlan {
    int nsub = 0;
    int64_t ntot = 0;             // real target points
    int64_t npad = 0;             // padded target rows
    int64_t nsrc = 0;             // real source points (ntot except for the field)
    int64_t spad = 0;             // padded source rows
    int max_chunks = 1;           // partial slots per row
    bool single = false;          // one set, no tables (geom / rows)
    bool field = false;           // targets are not the sources
    ItemGeom geom{};
    RowGeom rows{};
    int64_t nitems = 0, nblocks = 0;   // single: grid sizes
    std::vector<int4> items;      // (first target row, j0, j1, slot); slot -1: padding
    std::vector<int4> blocks;     // per 256 target rows: (first real point, count, set, slots)
    std::vector<int> bseg;        // [nsub + 1] row-block range of each set
    std::vector<int4> sblocks;    // field: per 256 source rows
    std::vector<int> sbseg;       // field: {0, source blocks}
};
// `items`: work items a launch aims at (0: the default).
ExactBatchPlan plan_exact_batch(const int64_t *offsets, int nsub, int64_t items = 0);
ExactBatchPlan plan_exact_single(int64_t n, int64_t items = 0);
ExactBatchPlan plan_exact_field(int64_t m, int64_t n, int64_t items = 0);
ItemGeom item_geom(int64_t n, int64_t items);
RowGeom row_geom(int64_t n, int slots);
int64_t plan_item_count(const ExactBatchPlan &pl);
int64_t plan_block_count(const ExactBatchPlan &pl);
struct ExactBatchBufs {
    float4 *Q, *P;                // [spad] packed FP32 sources k (q - c), p; zero padding
    float4 *X;                    // target rows (Q itself except for the field)
    float2 *part;                 // [max_chunks][6][npad] compensated sums (hi, lo)
    float2 *Fq, *Fp;              // [ntot][3] shooting state, FP32 (hi, lo) pairs (nullable)
    double *Sq, *Sp;              // [ntot][3] FP64 state of the backward stage (nullable)
    double *Hpart;                // [nt + 1][blocks]
    float *bpart;                 // [source blocks][6] boxes of the row blocks
    double *cen;                  // [nsub][3] FP64 centres of the sets' boxes
    float2 *cenf;                 // [nsub][3] the same as double-float
    const int4 *items = nullptr, *blk = nullptr;   // device tables (null: single set)
    const int *bseg = nullptr;
    const int4 *sblk = nullptr;   // field: source row blocks
    const int *sbseg = nullptr;
};
// The state a call keeps: none (right-hand side, field), FP32 hi+lo
// (shooting), FP64 (the forward steps of the backward stage).
enum StateKind { kStateNone = 0, kStateFF = 1, kStateF64 = 2 };
// Carves the state and partial buffers (not the tables).
void carve_exact_batch(Arena &a, const ExactBatchPlan &pl, int nt, int state,
                       ExactBatchBufs &b);
void carve_exact_field(Arena &a, const ExactBatchPlan &pl, ExactBatchBufs &b);
// Centres of the sets' boxes (of the field's sources) into b.cen.
gs_status launch_set_centres(const ExactBatchPlan &pl, const ExactBatchBufs &b, const float *q,
                             hipStream_t s);
// Set centres, the state (hi+lo or FP64, whichever is carved) and its FP32
// copies (positions k (q - c)).
gs_status launch_pack_state_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b,
                                 const float *q, const float *p, double sigma, hipStream_t s);
// Field: source centre, packed sources and targets.
gs_status launch_pack_field(const ExactBatchPlan &pl, const ExactBatchBufs &b, const float *x,
                            const float *q, const float *p, double sigma, hipStream_t s);
gs_status launch_exact_items(const ExactBatchPlan &pl, const ExactBatchBufs &b, bool with_a,
                             hipStream_t s);
// mode 0: (dq, dp) = (v, a) (dp nullable); mode 1: energy partials into Hpart
// (nullable; FP64), the velocity into vout (FP64 [ntot][3], nullable) and, if
// dt > 0, the Euler step of the state (hi+lo when carved, else FP64) and its
// packed copies.
gs_status launch_combine_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                              int mode, float *dq, float *dp, double dt, double *Hpart,
                              hipStream_t s, double *vout = nullptr);
// k = sqrt(log2(e) / (2 sigma^2)), the factor of the stored positions.
double position_scale(double sigma);
// Packs FP64 [ntot][3] arrays (a, b) into rows (sa (a - c), sb b) as float4
// (zero padding); c is the set's centre when `centre`, else 0.
gs_status launch_pack_rows64(const ExactBatchPlan &pl, const ExactBatchBufs &b, const double *a,
                             const double *bb, double sa, float4 *A, float4 *B, hipStream_t s,
                             double sb, bool centre);
// q = hi + lo of the FP32 hi+lo state (Fq, Fp: [2][n][3]), rounded to FP32.
gs_status launch_unpack_state(const float2 *Fq, const float2 *Fp, int64_t n, float *q, float *p,
                              hipStream_t s);
int combine_blocks(int64_t n);
// H[t] = sum_b Hpart[t * nblk + b] for t in [0, count).
gs_status launch_reduce_h(const double *Hpart, int nblk, int count, double *H, hipStream_t s);
// Per set: H[set * count + t] = sum of Hpart[t * stride + b] for b in
// [seg[set], seg[set + 1]) (seg: device int [nsub + 1]; null = one set).
gs_status launch_reduce_h_seg(const double *Hpart, int64_t stride, const int *seg, int nsub,
                              int count, double *H, hipStream_t s);

// FP64 exact path.
gs_status launch_exact_f64(const double *q, const double *p, int64_t n, double sigma,
                           bool with_a, double *v, double *a, hipStream_t s);
gs_status launch_euler_f64(double *q, double *p, const double *v, const double *a,
                           int64_t n, double dt, double *Hpart, hipStream_t s);
gs_status launch_copy_f64(const double *src, double *dst, int64_t count, hipStream_t s);

}  // namespace gs
