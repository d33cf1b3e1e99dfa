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

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Source split of the exact all-pairs kernel: number of source ranges that
// the targets' sums are split over so that a launch has enough waves.
struct ExactPlan {
    int64_t n;        // real points
    int64_t nsrc;     // padded source count (multiple of kTile)
    int64_t ntgt;     // padded target count
    int splits;       // S
    int64_t chunk;    // sources per split (multiple of kTile)
    int tpl;          // targets per lane (VALU kernel)
    int64_t chunk_quantum;  // chunks are multiples of this many sources
    bool mfma;        // (v, a) sums on the matrix cores
};
constexpr int kMfmaGroups = 4;  // groups of 16 targets per wave (MFMA kernel)
constexpr int kExactTplDefault = 1;  // targets per lane (VALU kernel, measured best)
constexpr int64_t kSplitBlocks = 24576;  // blocks per exact launch the split count aims at
constexpr int kXcds = 8;                 // MI355X: workgroups are dealt to 8 XCDs in turn
ExactPlan plan_exact(int64_t n_targets, int64_t n_sources, bool mfma = false);

// Buffers of one exact FP32 RHS evaluation.
struct ExactBufs {
    float4 *Q;        // [nsrc] x, y, z, 0
    float4 *P;        // [nsrc] px, py, pz, 0
    double *part;     // [S][6][ntgt]
};
void carve_exact(Arena &a, const ExactPlan &pl, ExactBufs &b);

// ---------------------------------------------------------------- launchers
// exact.hip
gs_status launch_pack(const float *q, const float *p, int64_t n, int64_t npad, float4 *Q,
                      float4 *P, hipStream_t s);
gs_status launch_pack_pos(const float *x, int64_t m, int64_t npad, float4 *X, hipStream_t s);
gs_status launch_exact_pairs(const ExactPlan &pl, const float4 *Qt, const float4 *Pt,
                             const float4 *Qs, const float4 *Ps, double sigma, bool with_a,
                             double *part, hipStream_t s);
// Sums the split partials of target i and writes (v, a) as float [n][3].
gs_status launch_combine_rhs(const ExactPlan &pl, const double *part, double sigma,
                             float *dq, float *dp, hipStream_t s);
// Sums the partials, adds p_i . v_i of each block into Hpart (nullable), and,
// if dt > 0, advances the FP64 state (Sq += dt v, Sp += dt a) and refreshes
// its FP32 copies Q, P.
gs_status launch_combine_euler(const ExactPlan &pl, const double *part, double sigma,
                               double dt, double *Sq, double *Sp, float4 *Q, float4 *P,
                               double *Hpart, hipStream_t s);
// FP64 state from float [n][3] inputs, plus its FP32 packed copies.
gs_status launch_pack_state(const float *q, const float *p, int64_t n, int64_t npad, double *Sq,
                            double *Sp, float4 *Q, float4 *P, hipStream_t s);
gs_status launch_unpack_state(const double *Sq, const double *Sp, int64_t n, float *q, float *p,
                              hipStream_t s);
int combine_blocks(int64_t n);
// H[t] = sum_b Hpart[t * nblk + b] for t in [0, count).
gs_status launch_reduce_h(const double *Hpart, int nblk, int count, double *H, hipStream_t s);
// Per set: H[set * count + t] = sum of Hpart[t * stride + b] for b in
// [seg[set], seg[set + 1]) (seg: device int [nsub + 1]; null = one set).
gs_status launch_reduce_h_seg(const double *Hpart, int64_t stride, const int *seg, int nsub,
                              int count, double *H, hipStream_t s);

// ---------------------------------------------------------------- batched sets
// Exact evaluation of independent point sets (subjects) stored one after the
// other ([offsets[s], offsets[s+1]) is set s).  Rows are padded per set to
// whole blocks of 256 targets; a work item is one such block against one
// source chunk of its own set.  Each source chunk has a home XCD; items run
// on their chunk's XCD, largest first.
struct ExactBatchPlan {
    int nsub;
    int64_t ntot;                 // real points
    int64_t npad;                 // padded rows
    int max_chunks;               // partial slots per row
    std::vector<int4> items;      // (first target row, j0, j1, slot); slot -1: padding
    std::vector<int4> blocks;     // per 256-row block: (first real point, count, set, slots)
    std::vector<int> bseg;        // [nsub + 1] row-block range of each set
};
// `items`: work items a launch aims at (0: the default, or the
// GS_EXACT_ITEM_BLOCKS environment override).
ExactBatchPlan plan_exact_batch(const int64_t *offsets, int nsub, int64_t items = 0);
struct ExactBatchBufs {
    float4 *Q, *P;                // [npad] packed FP32 state (scaled positions), zero padding
    double *part;                 // [max_chunks][6][npad]
    double *Sq, *Sp;              // [ntot][3] FP64 state
    double *Hpart;                // [nt + 1][blocks]
    const int4 *items, *blk;      // device copies of the plan's tables (set by the caller)
    const int *bseg;
};
// Carves the state and partial buffers (not the tables).
void carve_exact_batch(Arena &a, const ExactBatchPlan &pl, int nt, ExactBatchBufs &b);
// Packs the FP64 state and its FP32 copies (positions scaled by
// sqrt(log2(e) / (2 sigma^2)), zero padding).
gs_status launch_pack_state_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b,
                                 const float *q, const float *p, double sigma, hipStream_t s);
gs_status launch_exact_items(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                             bool with_a, hipStream_t s);
// mode 0: (dq, dp) = (v, a); mode 1: energy partials into Hpart (nullable),
// the velocity into vout (FP64 [ntot][3], nullable) and, if dt > 0, the
// Euler step of the FP64 state and its packed copies.
gs_status launch_combine_rows(const ExactBatchPlan &pl, const ExactBatchBufs &b, double sigma,
                              int mode, float *dq, float *dp, double dt, double *Hpart,
                              hipStream_t s, double *vout = nullptr);
// k = sqrt(log2(e) / (2 sigma^2)), the factor of the stored positions.
double position_scale(double sigma);
// Packs FP64 [ntot][3] arrays (a, b) into rows (sa a, sb b) as float4 (zero
// padding), with the row blocks `blk` of the plan (device table).
gs_status launch_pack_rows64(const ExactBatchPlan &pl, const int4 *blk, const double *a,
                             const double *b, double sa, float4 *A, float4 *B, hipStream_t s,
                             double sb = 1.0);

// FP64 exact path.
gs_status launch_exact_f64(const double *q, const double *p, int64_t n, double sigma,
                           bool with_a, double *v, double *a, hipStream_t s);
gs_status launch_euler_f64(double *q, double *p, const double *v, const double *a,
                           int64_t n, double dt, double *Hpart, hipStream_t s);
gs_status launch_copy_f64(const double *src, double *dst, int64_t count, hipStream_t s);

}  // namespace gs
