// tree.hip -- GPU build of the Barnes-Hut octree (Sec. 2.2, "Oct-tree
// Representation of Space") and its node statistics.
//
// Launch sequence of one build (no host synchronisation, so it can be
// captured in a graph):
//   bbox_partial -> bbox_final     tight box of every set, E, 2^21/E
//   morton_hist                    63-bit keys: 21 bits per axis, x highest,
//                                  and the first pass's digit counts
//   7 x ([hist,] scatter)          stable LSD radix sort of (key, index),
//                                  9-bit digits (the first pass's counts come
//                                  from morton_hist)
//   1-2 x (hist, scatter)          (forest only) stable passes on the set
//                                  index, so each set is sorted in its range
//   boundaries                     sorted FP32 copies of q, p, summaries of
//                                  64-point chunks, the split level of every
//                                  pair of neighbours and the internal-node
//                                  flag of its cell
//   scan(flag)                     internal-node ranks and the boundary of
//                                  every rank
//   children                       child count of every internal node
//   scan(nchild)                   contiguous child blocks
//   nodes                          node records (roots, ranges, child links)
//                                  and summaries of 4096 points
//   stats                          FP64 sums, tight boxes, centres of every
//                                  node
// (24 launches for one set; the scans skip their first launch below 2049
// values.)
//
// Tree semantics.  For sorted keys K, the boundary between points i and i+1
// has split level L = floor(lcp(K_i, K_i+1) / 3) (21 when the keys are equal).
// The level-L cell containing both points is split there; the first such
// boundary in a cell represents the cell.  A represented cell with more than
// leaf_cap points is an internal node of the compressed octree (all its
// ancestors hold even more points, so they are split too); its children are
// the non-empty level-(L+1) sub-cells: a child with <= leaf_cap points, or
// whose points share one key, is a leaf; otherwise it is the internal node
// represented by its own first split.
//
// Forest.  Independent point sets (subjects) given as index ranges of one
// array are built in the same launches: every set gets its own root cube,
// the sort keeps each set in its own index range, the split searches stay
// inside the set's range, and node s is the root of set s.  Each tree is
// exactly the tree of its set built alone.
#include <hip/hip_runtime.h>

#include "tree.h"

namespace gs {

namespace {

typedef unsigned long long u64;

constexpr int kScanTile = 2048;                            // items per scan block
constexpr int kChunk = 64;                                 // points per range summary

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// Blocks of 4 waves for one-wave-per-node kernels over at most max_nodes.
constexpr unsigned kNodeBlocks = 4096;
inline unsigned node_blocks(int64_t max_nodes) {
    const unsigned b = nblk(max_nodes, 4);
    return b < kNodeBlocks ? b : kNodeBlocks;
}

// Set of index i: the largest s with seg[s] <= i (seg is non-decreasing, so
// this is the set whose range holds i even when empty sets precede it).
__device__ inline int set_of(const long long *__restrict__ seg, int nsub, int64_t i) {
    if (!seg) return 0;
    int lo = 0, hi = nsub - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Origin of the FP32 frame of a set along one axis (the tree path's pair
// positions q - c): the box centre rounded to a multiple of 2^m, the
// smallest power of two not below the box side.  A set whose box lies within
// half a side of the origin gets c = 0, so its FP32 differences are taken on
// the inputs themselves; for a set far from the origin, q and c lie within a
// factor of two of each other and q - c is exact (Sterbenz).  Either way the
// rounding no longer depends on the set's distance from the origin.
__device__ inline double frame_origin(float lo, float hi) {
    const double l = lo, h = hi, side = h - l, mid = 0.5 * (l + h);
    if (!(side > 0.0)) return mid;  // one value on this axis: q - c = 0
    int e;
    frexp(side, &e);  // side = f 2^e with f in [0.5, 1), so 2^e >= side
    return ldexp(rint(ldexp(mid, -e)), e);
}

// ---------------------------------------------------------------- bbox
// grid (blocks per set, sets); partials [set][block][6]
// With `clear` (nullable) the kernel also zeroes clear[0 .. nclear) (the
// sort's first superblock counts, before the Morton-key kernel adds into them).
__global__ __launch_bounds__(256) void k_bbox_partial(const float *__restrict__ q, int64_t n,
                                                      const long long *__restrict__ seg,
                                                      float *__restrict__ part,
                                                      unsigned *__restrict__ clear,
                                                      int64_t nclear) {
    __shared__ float red[6][256];
    if (clear) {
        const int64_t nb = (int64_t)gridDim.x * gridDim.y;
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        for (int64_t i = b * 256 + threadIdx.x; i < nclear; i += nb * 256) clear[i] = 0;
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float bad = 0.f;
    const int64_t a = seg ? seg[blockIdx.y] : 0, b = seg ? seg[blockIdx.y + 1] : n;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float x = q[3 * i + c];
            if (!isfinite(x)) bad = 1.f;
            lo[c] = fminf(lo[c], x);
            hi[c] = fmaxf(hi[c], x);
        }
    }
    // a non-finite coordinate is recorded in slot 0 as NaN
    if (bad != 0.f) lo[0] = NAN;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = lo[c];
        red[3 + c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float a = red[c][threadIdx.x], b = red[c][threadIdx.x + s];
                // keep a NaN flag in slot 0 sticky
                red[c][threadIdx.x] = (c == 0 && (isnan(a) || isnan(b))) ? NAN : fminf(a, b);
                red[3 + c][threadIdx.x] = fmaxf(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6)
        part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// One wave per set: reduces its nb partial boxes.
__global__ __launch_bounds__(64) void k_bbox_final(const float *__restrict__ part, int nb,
                                                   TreeMeta *__restrict__ meta_all,
                                                   int *__restrict__ status) {
    const int lane = threadIdx.x;
    const float *ps = part + (int64_t)blockIdx.x * nb * 6;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int b = lane; b < nb; b += 64) {
        if (isnan(ps[6 * b])) bad = 1;
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], ps[6 * b + c]);
            hi[c] = fmaxf(hi[c], ps[6 * b + 3 + c]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        bad |= __shfl_xor(bad, off, 64);
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], off, 64));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], off, 64));
        }
    }
    if (lane != 0) return;
    TreeMeta *meta = meta_all + blockIdx.x;
    double e = 0.0;
    for (int c = 0; c < 3; ++c) {
        meta->lo[c] = lo[c];
        meta->hi[c] = hi[c];
        const double ext = (double)hi[c] - (double)lo[c];
        if (ext > e) e = ext;
    }
    if (bad || !isfinite(e)) {
        bad = 1;
        e = 0.0;  // degenerate tree: one leaf (results are not meaningful)
    }
    for (int c = 0; c < 3; ++c) meta->cen[c] = bad ? 0.0 : frame_origin(lo[c], hi[c]);
    meta->extent = e;
    meta->scale = e > 0.0 ? 2097152.0 / e : 0.0;
    meta->nonfinite = bad;
    if (bad && status) *status = 1;
}

// ---------------------------------------------------------------- Morton keys
__device__ inline u64 spread3(unsigned v) {
    // bits b of v -> bit 3b of the result (v < 2^21)
    u64 x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline unsigned quantize(float x, float lo, double scale) {
    // c = min(2^21 - 1, floor((x - lo) * 2^21 / E)), evaluated in FP64
    const double f = floor(((double)x - (double)lo) * scale);
    if (!(f >= 0.0)) return 0u;  // also NaN
    if (f >= 2097151.0) return 2097151u;
    return (unsigned)f;
}

// Orders this wave's LDS writes before its following LDS reads.
__device__ inline void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of (key, original index) with 9-bit digits: 7 passes
// over the 63-bit keys, then (forests) 1 or 2 passes over the set index of
// the original position, so that each set ends up sorted in its own range.
// A pass is two launches over tiles of 256 x PER keys:
//   k_os_hist     per-tile digit counts (one row of kOsBins per tile), also
//                 added into the row of the tile's superblock (kSbTiles
//                 consecutive tiles);
//   k_os_scatter  each tile takes its output offsets from the superblock rows
//                 before it, the tile rows before it in its own superblock and
//                 the digit totals (the sum of all superblock rows), ranks its
//                 keys stably within the tile and writes them.
// No block waits for another; a tile reads at most (superblocks + 15) rows.
// The counts of pass 0 are taken by the Morton-key kernel.
constexpr int kOsBits = 9;
constexpr int kOsBins = 1 << kOsBits;
// Keys per thread: 4 (tiles of 1024 keys) below kOsLargeFrom points, 8 (2048)
// from there on.  Measured per 200k-point build: 0.213 / 0.179 / 0.175 ms
// with tiles of 2048 / 1024 / 512 keys; per 1.5M-point population build:
// 0.650 / 0.683 / 1.05 ms (more tiles, more prefix rows to read).
constexpr int kOsPerSmall = 4;
constexpr int kOsPerLarge = 8;
constexpr int64_t kOsLargeFrom = 1000000;
constexpr int kSbTiles = 16;                    // tiles per superblock
constexpr int kKeyPasses = 7;                   // 7 x 9 bits cover the 63-bit key

__device__ inline unsigned os_digit(int pass, u64 key, unsigned val,
                                    const long long *__restrict__ seg, int nsub) {
    if (pass < kKeyPasses) return (unsigned)(key >> (kOsBits * pass)) & (kOsBins - 1);
    return ((unsigned)set_of(seg, nsub, (int64_t)val) >> (kOsBits * (pass - kKeyPasses))) &
           (kOsBins - 1);
}

// The tile's LDS counts -> its row and its superblock's row.
__device__ inline void os_flush(const unsigned *h, unsigned *__restrict__ hist,
                                unsigned *__restrict__ sb, int tile) {
    for (int d = threadIdx.x; d < kOsBins; d += 256) {
        const unsigned c = h[d];
        hist[(int64_t)tile * kOsBins + d] = c;
        if (c) atomicAdd(&sb[(int64_t)(tile / kSbTiles) * kOsBins + d], c);
    }
}

// 63-bit Morton keys of a tile (21 bits per axis, x highest), their original
// indices, and the tile's pass-0 digit counts.
template <int PER>
__global__ __launch_bounds__(256) void k_morton_hist(const float *__restrict__ q, int64_t n,
                                                     const long long *__restrict__ seg, int nsub,
                                                     const TreeMeta *__restrict__ meta_all,
                                                     u64 *__restrict__ keys,
                                                     unsigned *__restrict__ vals,
                                                     unsigned *__restrict__ hist,
                                                     unsigned *__restrict__ sb) {
    __shared__ unsigned h[kOsBins];
    for (int d = threadIdx.x; d < kOsBins; d += 256) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (256 * PER);
    for (int r = 0; r < PER; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) {
            const TreeMeta *meta = meta_all + set_of(seg, nsub, i);
            const double sc = meta->scale;
            const unsigned cx = quantize(q[3 * i], meta->lo[0], sc);
            const unsigned cy = quantize(q[3 * i + 1], meta->lo[1], sc);
            const unsigned cz = quantize(q[3 * i + 2], meta->lo[2], sc);
            const u64 key = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
            keys[i] = key;
            vals[i] = (unsigned)i;
            atomicAdd(&h[(unsigned)key & (kOsBins - 1)], 1u);
        }
    }
    __syncthreads();
    os_flush(h, hist, sb, blockIdx.x);
}

template <int PER>
__global__ __launch_bounds__(256) void k_os_hist(const u64 *__restrict__ keys,
                                                 const unsigned *__restrict__ vals, int64_t n,
                                                 int pass, const long long *__restrict__ seg,
                                                 int nsub, unsigned *__restrict__ hist,
                                                 unsigned *__restrict__ sb) {
    __shared__ unsigned h[kOsBins];
    for (int d = threadIdx.x; d < kOsBins; d += 256) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (256 * PER);
    u64 key[PER];
    unsigned val[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {  // loads first, then the counts
        const int64_t i = base + r * 256 + threadIdx.x;
        key[r] = i < n ? keys[i] : 0ull;
        val[r] = i < n && pass >= kKeyPasses ? vals[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r)
        if (base + r * 256 + threadIdx.x < n)
            atomicAdd(&h[os_digit(pass, key[r], val[r], seg, nsub)], 1u);
    __syncthreads();
    os_flush(h, hist, sb, blockIdx.x);
}

// One pass's scatter.  sb_next (the other superblock buffer) is cleared for
// the next pass's counts.  Wave w holds tile positions [64 PER w, 64 PER (w +
// 1)) and ranks them stably by digit with ballots and its own running counts
// (no block barrier between rounds); the counts of the waves before it then
// complete each key's place within the tile.  The keys go through LDS in the
// tile's sorted order, so that the writes of a wave are runs of consecutive
// addresses.
template <int PER>
__global__ __launch_bounds__(256) void k_os_scatter(
    const u64 *__restrict__ kin, const unsigned *__restrict__ vin, u64 *__restrict__ kout,
    unsigned *__restrict__ vout, int64_t n, int pass, const long long *__restrict__ seg,
    int nsub, const unsigned *__restrict__ hist, const unsigned *__restrict__ sb, int nsb,
    unsigned *__restrict__ sb_next) {
    __shared__ unsigned dbase[kOsBins];     // output offset of each digit for this tile
    __shared__ unsigned wrun[4][kOsBins];   // per wave: keys of each digit ranked so far,
                                            // then the counts of the waves before it
    __shared__ unsigned lbase[kOsBins];     // first place of each digit in the tile's order
    __shared__ unsigned goff[kOsBins];      // dbase - lbase
    __shared__ u64 skey[256 * PER];         // the tile's keys in sorted order
    __shared__ unsigned sval[256 * PER];
    __shared__ unsigned wsum[4], wsum2[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int tile = blockIdx.x, mysb = tile / kSbTiles;
    // this thread's keys first, so that their loads overlap the prefix reads
    const int64_t base = (int64_t)tile * (256 * PER) + (int64_t)wv * (64 * PER) + lane;
    u64 key[PER];
    unsigned val[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t i = base + r * 64;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < (int64_t)nsb * kOsBins;
         i += (int64_t)gridDim.x * 256)
        sb_next[i] = 0;
    // digits 2t, 2t + 1: totals, and the counts of the tiles before this one
    // (every row load is issued before any is added)
    unsigned tot[2] = {0, 0}, pre[2] = {0, 0};
    {
        const int j0 = mysb * kSbTiles;
        uint2 h[kSbTiles];
#pragma unroll
        for (int u = 0; u < kSbTiles; ++u)
            h[u] = j0 + u < tile
                       ? *reinterpret_cast<const uint2 *>(hist + (int64_t)(j0 + u) * kOsBins + 2 * t)
                       : make_uint2(0u, 0u);
        for (int b0 = 0; b0 < nsb; b0 += 16) {
            uint2 v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = b0 + u < nsb ? *reinterpret_cast<const uint2 *>(
                                          sb + (int64_t)(b0 + u) * kOsBins + 2 * t)
                                    : make_uint2(0u, 0u);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                tot[0] += v[u].x;
                tot[1] += v[u].y;
                if (b0 + u < mysb) {
                    pre[0] += v[u].x;
                    pre[1] += v[u].y;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kSbTiles; ++u) {
            pre[0] += h[u].x;
            pre[1] += h[u].y;
        }
    }
    // exclusive scan of the totals over the digits (thread t holds 2t, 2t+1)
    const unsigned s2 = tot[0] + tot[1];
    unsigned incl = s2;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        wrun[w][2 * t] = 0;
        wrun[w][2 * t + 1] = 0;
    }
    __syncthreads();
    unsigned ex = incl - s2;
    for (int w = 0; w < wv; ++w) ex += wsum[w];
    dbase[2 * t] = ex + pre[0];
    dbase[2 * t + 1] = ex + tot[0] + pre[1];
    // stable ranks within the wave's keys: rounds in index order, lanes in order
    const u64 lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned dig[PER], rank[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t i = base + r * 64;
        const bool valid = i < n;
        const unsigned d = valid ? os_digit(pass, key[r], val[r], seg, nsub) : 0u;
        dig[r] = d;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kOsBits; ++b) {
            const u64 m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const unsigned lr = __popcll(peers & lt);
        rank[r] = valid ? wrun[wv][d] + lr : 0u;
        wave_lds_order();
        if (valid && lr == 0) wrun[wv][d] += (unsigned)__popcll(peers);
        wave_lds_order();
    }
    __syncthreads();
    // the counts of the waves before each wave, per digit, and the tile's
    // count of each digit
    unsigned cnt[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int d = 2 * t + j;
        unsigned acc = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const unsigned c = wrun[w][d];
            wrun[w][d] = acc;
            acc += c;
        }
        cnt[j] = acc;
    }
    // the tile's keys in sorted order go to LDS first (local offset lbase of
    // each digit: an exclusive scan of the tile's counts), then out in that
    // order, so that the lanes of a wave write runs of consecutive addresses
    const unsigned c2 = cnt[0] + cnt[1];
    unsigned lin = c2;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(lin, o, 64);
        if (lane >= o) lin += u;
    }
    if (lane == 63) wsum2[wv] = lin;
    __syncthreads();
    unsigned lex = lin - c2;
    for (int w = 0; w < wv; ++w) lex += wsum2[w];
    lbase[2 * t] = lex;
    lbase[2 * t + 1] = lex + cnt[0];
    goff[2 * t] = dbase[2 * t] - lex;
    goff[2 * t + 1] = dbase[2 * t + 1] - (lex + cnt[0]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t i = base + r * 64;
        if (i < n) {
            const unsigned d = dig[r];
            const unsigned lp = lbase[d] + wrun[wv][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const int64_t t0 = (int64_t)tile * (256 * PER);
    const int cnt_tile = (int)(n - t0 < 256 * PER ? n - t0 : 256 * PER);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = r * 256 + t;
        if (e < cnt_tile) {
            const u64 k = skey[e];
            const unsigned v = sval[e];
            const unsigned pos = goff[os_digit(pass, k, v, seg, nsub)] + (unsigned)e;
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

// Sets of at most kBlockSortMax points: one block per set computes the keys
// of its points and sorts them in LDS (k_block_radix), in the order of the
// stable radix sort (key, then index): identical results in one launch
// instead of 15 to 17.  With tile > 0 (one set of n points) block b sorts the
// tile [b tile, (b + 1) tile) instead, for k_merge_rank.
constexpr int kBlockSortMax = 2048;
constexpr int kMergeTiles = 16;  // one set of at most 16 x 2048 points: tiles + merge

// LSD radix sort of one set or tile in LDS (7 passes of 9-bit digits, stable):
// position p = 512 w + 64 r + l is held by lane l of wave w in round r.  In a
// pass every wave ranks its 8 rounds by digit with ballots and its own
// running digit counts (no block barrier), then the digit totals and the
// counts of earlier waves give each key its place.
__global__ __launch_bounds__(256) void k_block_radix(const float *__restrict__ q,
                                                     const long long *__restrict__ seg,
                                                     const TreeMeta *__restrict__ meta_all,
                                                     int64_t n, int tile, u64 *__restrict__ kout,
                                                     unsigned *__restrict__ vout) {
    __shared__ u64 bk[kBlockSortMax];
    __shared__ unsigned bv[kBlockSortMax];
    __shared__ unsigned wrun[4][kOsBins];  // per wave: keys of each digit so far
    __shared__ unsigned wsum[4];
    const int set = tile > 0 ? 0 : blockIdx.x;
    const int64_t base = tile > 0 ? (int64_t)blockIdx.x * tile : (seg ? seg[set] : 0);
    const int64_t end = tile > 0 ? (base + tile < n ? base + tile : n) : (seg ? seg[set + 1] : n);
    const int m = (int)(end - base);
    if (m <= 0) return;  // block-uniform
    const TreeMeta *meta = meta_all + set;
    const double sc = meta->scale;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    u64 K[8];
    unsigned V[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = 512 * wv + 64 * r + lane;
        if (i < m) {
            const int64_t g = base + i;
            const unsigned cx = quantize(q[3 * g], meta->lo[0], sc);
            const unsigned cy = quantize(q[3 * g + 1], meta->lo[1], sc);
            const unsigned cz = quantize(q[3 * g + 2], meta->lo[2], sc);
            K[r] = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
            V[r] = (unsigned)i;
        } else {  // padding: the largest digit in every pass, after every key
            K[r] = ~0ull;
            V[r] = 0xffffffffu;
        }
    }
    for (int pass = 0; pass < kKeyPasses; ++pass) {
        const int sh = kOsBits * pass;
        for (int d = t; d < 4 * kOsBins; d += 256) (&wrun[0][0])[d] = 0;
        __syncthreads();
        unsigned dig[8], rk[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const unsigned d = (unsigned)(K[r] >> sh) & (kOsBins - 1);
            dig[r] = d;
            u64 peers = ~0ull;
#pragma unroll
            for (int b = 0; b < kOsBits; ++b) {
                const u64 mb = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? mb : ~mb;
            }
            const unsigned lr = __popcll(peers & lt);
            rk[r] = wrun[wv][d] + lr;  // keys of this digit before this one in the wave
            wave_lds_order();
            if (lr == 0) wrun[wv][d] += __popcll(peers);
            wave_lds_order();
        }
        __syncthreads();
        // digits 2t, 2t + 1: totals over the waves, exclusive scan over the
        // digits, and the counts of the waves before each wave
        unsigned tot[2], pw[4][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            unsigned acc = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                pw[w][c] = acc;
                acc += wrun[w][2 * t + c];
            }
            tot[c] = acc;
        }
        const unsigned s2 = tot[0] + tot[1];
        unsigned incl = s2;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        unsigned ex = incl - s2;
        for (int w = 0; w < wv; ++w) ex += wsum[w];
        // the place of digit d's first key of wave w: into wrun (read back below)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            wrun[w][2 * t] = ex + pw[w][0];
            wrun[w][2 * t + 1] = ex + tot[0] + pw[w][1];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const unsigned pos = wrun[wv][dig[r]] + rk[r];
            bk[pos] = K[r];
            bv[pos] = V[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = 512 * wv + 64 * r + lane;
            K[r] = bk[i];
            V[r] = bv[i];
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = 512 * wv + 64 * r + lane;
        if (i < m) {
            kout[base + i] = K[r];
            vout[base + i] = (unsigned)(base + V[r]);
        }
    }
}

// Merge of the sorted tiles of one set: the final position of a pair is its
// rank in its own tile plus, in every other tile, the number of pairs that
// order before it (binary search by key, then index).
__global__ __launch_bounds__(256) void k_merge_rank(const u64 *__restrict__ tk,
                                                    const unsigned *__restrict__ tv, int64_t n,
                                                    int tile, u64 *__restrict__ kout,
                                                    unsigned *__restrict__ vout) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const u64 key = tk[t];
    const unsigned idx = tv[t];
    const int64_t mine = t / tile;
    int64_t rank = t - mine * tile;
    const int64_t tiles = (n + tile - 1) / tile;
    for (int64_t u = 0; u < tiles; ++u) {
        if (u == mine) continue;
        const int64_t lo = u * tile;
        int64_t a = lo, b = lo + tile < n ? lo + tile : n;
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            const u64 km = tk[mid];
            if (km < key || (km == key && tv[mid] < idx))
                a = mid + 1;
            else
                b = mid;
        }
        rank += a - lo;
    }
    kout[rank] = key;
    vout[rank] = idx;
}

// Statistics of contiguous ranges of sorted points.  A two-level summary
// (chunks of 64 points, super-chunks of 64 chunks) lets every node reduce
// its own range [start, start + n) independently: no inter-node ordering,
// atomics or fences, and a fixed summation order (bitwise deterministic).
struct RangeStat {
    double s[6];  // sums of q (3) and p (3)
    float lo[3], hi[3];
};

__device__ inline void rs_init(RangeStat &r) {
    for (int c = 0; c < 6; ++c) r.s[c] = 0.0;
    for (int c = 0; c < 3; ++c) {
        r.lo[c] = INFINITY;
        r.hi[c] = -INFINITY;
    }
}
__device__ inline void rs_add(RangeStat &r, const RangeStat &o) {
    for (int c = 0; c < 6; ++c) r.s[c] += o.s[c];
    for (int c = 0; c < 3; ++c) {
        r.lo[c] = fminf(r.lo[c], o.lo[c]);
        r.hi[c] = fmaxf(r.hi[c], o.hi[c]);
    }
}
__device__ inline void rs_point(RangeStat &r, const float4 a, const float4 b) {
    r.s[0] += a.x;
    r.s[1] += a.y;
    r.s[2] += a.z;
    r.s[3] += b.x;
    r.s[4] += b.y;
    r.s[5] += b.z;
    r.lo[0] = fminf(r.lo[0], a.x);
    r.lo[1] = fminf(r.lo[1], a.y);
    r.lo[2] = fminf(r.lo[2], a.z);
    r.hi[0] = fmaxf(r.hi[0], a.x);
    r.hi[1] = fmaxf(r.hi[1], a.y);
    r.hi[2] = fmaxf(r.hi[2], a.z);
}

// One wave per chunk: lane l takes item l of the chunk; fixed shuffle tree.
__device__ inline void rs_wave_reduce(RangeStat &r) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 6; ++c) r.s[c] += __shfl_down(r.s[c], off, 64);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r.lo[c] = fminf(r.lo[c], __shfl_down(r.lo[c], off, 64));
            r.hi[c] = fmaxf(r.hi[c], __shfl_down(r.hi[c], off, 64));
        }
    }
}

// ---------------------------------------------------------------- generic scan
// Exclusive scan of n u32 values: per-block totals, then each block adds the
// totals of the blocks before it.  out may equal in.  *total (nullable)
// receives the sum.  A block covers kScanTile = 256 threads x 8 contiguous
// values; a thread scans its 8 values serially, a wave scans its 64 thread
// sums with shuffles, and the 4 wave sums are combined through LDS.
constexpr int kScanPer = kScanTile / 256;  // values per thread

__global__ __launch_bounds__(256) void k_scan_blocksum(const unsigned *__restrict__ in,
                                                       int64_t n, unsigned *__restrict__ part) {
    __shared__ unsigned wsum[4];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
    unsigned s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (i0 + k < n) s += in[i0 + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((t & 63) == 0) wsum[t >> 6] = s;
    __syncthreads();
    if (t == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// With `scatter` (nullable), every i < nscatter with in[i] != 0 also writes i
// to scatter[out[i]] (for 0/1 flags: the position of the flag of each rank).
__global__ __launch_bounds__(256) void k_scan_apply(const unsigned *__restrict__ in,
                                                    unsigned *__restrict__ out, int64_t n,
                                                    const unsigned *__restrict__ part,
                                                    unsigned *__restrict__ total,
                                                    unsigned *__restrict__ scatter,
                                                    int64_t nscatter) {
    __shared__ unsigned wsum[4];
    __shared__ unsigned carry_s;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // offset of this block: sum of the previous block totals
    unsigned off = 0;
    for (int b = t; b < (int)blockIdx.x; b += 256) off += part[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) off += __shfl_down(off, o, 64);
    if (lane == 0) wsum[wv] = off;
    __syncthreads();
    if (t == 0) carry_s = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    const unsigned carry = carry_s;
    __syncthreads();  // wsum is reused below
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
    unsigned v[kScanPer];
    unsigned run = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = i0 + k < n ? in[i0 + k] : 0u;
        run += v[k];
    }
    // inclusive scan of the thread sums within the wave
    unsigned incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    unsigned base = carry;
    for (int w = 0; w < wv; ++w) base += wsum[w];
    base += incl - run;  // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (i0 + k < n) out[i0 + k] = base;
        if (scatter && v[k] != 0u && i0 + k < nscatter) scatter[base] = (unsigned)(i0 + k);
        base += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && t == 255)
        *total = carry + wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// ---------------------------------------------------------------- tree
__device__ inline int split_level(u64 a, u64 b) {
    const u64 x = a ^ b;
    if (x == 0ull) return kLevels;
    return (__clzll((long long)x) - 1) / 3;
}

__device__ inline int level_shift(int L) { return 63 - 3 * L; }

// first index in [lo, hi) with K[i] >= key
__device__ inline int64_t lower_bound(const u64 *__restrict__ K, int64_t lo, int64_t hi, u64 key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (K[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Per sorted position i: the gathered point (Qs, Ps), the summary of each
// 64-point chunk (one wave per chunk), and the boundary after i (its split
// level and, for the first split of an over-full cell, the cell's range).
__global__ __launch_bounds__(256) void k_boundaries(const u64 *__restrict__ K, int64_t n,
                                                    const long long *__restrict__ seg, int nsub,
                                                    int leaf_cap, const float *__restrict__ q,
                                                    const float *__restrict__ p,
                                                    const unsigned *__restrict__ perm,
                                                    const TreeMeta *__restrict__ meta,
                                                    float4 *__restrict__ Qs,
                                                    float4 *__restrict__ Ps,
                                                    float4 *__restrict__ Qc,
                                                    RangeStat *__restrict__ c0, int64_t nc0,
                                                    unsigned char *__restrict__ lvl,
                                                    unsigned *__restrict__ flag,
                                                    unsigned *__restrict__ bs,
                                                    unsigned *__restrict__ be) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    {
        RangeStat r;
        rs_init(r);
        if (i < n) {
            const int64_t src = perm[i];
            const float4 a = make_float4(q[3 * src], q[3 * src + 1], q[3 * src + 2], 0.f);
            const float4 b = make_float4(p[3 * src], p[3 * src + 1], p[3 * src + 2], 0.f);
            Qs[i] = a;
            Ps[i] = b;
            // pair arithmetic works relative to the set's frame origin (FP64 difference,
            // rounded once), so its accuracy does not depend on where the set lies
            const double *cen = meta[set_of(seg, nsub, i)].cen;
            Qc[i] = make_float4((float)((double)a.x - cen[0]), (float)((double)a.y - cen[1]),
                                (float)((double)a.z - cen[2]), 0.f);
            rs_point(r, a, b);
        }
        rs_wave_reduce(r);  // the wave's 64 positions are chunk i / kChunk
        const int64_t c = i / kChunk;
        if ((threadIdx.x & 63) == 0 && c < nc0) c0[c] = r;
    }
    if (i >= n) return;
    // the range [a0, b0) of the set holding point i
    int64_t a0 = 0, b0 = n;
    if (seg) {
        const int si = set_of(seg, nsub, i);
        a0 = seg[si];
        b0 = seg[si + 1];
    }
    if (i == b0 - 1) {  // no boundary after the last point of a set
        flag[i] = 0;
        return;
    }
    const u64 a = K[i];
    const int L = split_level(a, K[i + 1]);
    lvl[i] = (unsigned char)L;
    unsigned f = 0;
    if (L < kLevels) {
        const int sh = level_shift(L);
        const u64 pre = L == 0 ? 0ull : (a >> sh);
        const u64 cell_lo = L == 0 ? 0ull : (pre << sh);
        const u64 cell_hi = L == 0 ? ~0ull : (((pre + 1) << sh) - 1);
        const int64_t s = lower_bound(K, a0, i, cell_lo);
        // end: first index after i + 1 with a key above the cell
        int64_t lo = i + 1, hi = b0;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (K[mid] <= cell_hi)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int64_t e = lo;
        // representative: the first split of the cell, i.e. K[s] and K[i]
        // share the level-(L+1) prefix
        const bool rep = ((K[s] ^ a) >> level_shift(L + 1)) == 0ull;
        if (rep && e - s > leaf_cap) {
            f = 1;
            bs[i] = (unsigned)s;
            be[i] = (unsigned)e;
        }
    }
    flag[i] = f;
}

// Representative boundary of the compressed internal node covering [a, b)
// (b - a > leaf_cap, keys not all equal).
__device__ inline int64_t child_rep(const u64 *__restrict__ K, int64_t a, int64_t b) {
    const int L = split_level(K[a], K[b - 1]);
    const int sh = level_shift(L + 1);
    const u64 pre = K[a] >> sh;
    return lower_bound(K, a, b, (pre + 1) << sh) - 1;
}

// Child runs of every internal node, one wave per node: lane d (1..7)
// searches where octant d starts, so the searches run side by side; the
// non-empty octants in order are the children.  crun[9 r + k] is the first
// sorted point of child k of rank r, crun[9 r + nchild] the end of the cell.
__global__ __launch_bounds__(256) void k_children(const u64 *__restrict__ K,
                                                  const unsigned char *__restrict__ lvl,
                                                  const TreeTotals *__restrict__ totals,
                                                  const unsigned *__restrict__ bs,
                                                  const unsigned *__restrict__ be,
                                                  const unsigned *__restrict__ rank_bnd,
                                                  unsigned *__restrict__ nchild,
                                                  unsigned *__restrict__ crun) {
    const int lane = threadIdx.x & 63;
    const int64_t nint = totals->n_internal, waves = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nint; r += waves) {
        const unsigned i = rank_bnd[r];
        const int64_t s = bs[i], e = be[i];
        const int L = lvl[i];
        const u64 pre = L == 0 ? 0ull : (K[s] >> level_shift(L));
        const int sh = level_shift(L + 1);
        // start of octant `lane` (lanes 0..8; octant 0 starts at s, "octant 8" at e)
        int64_t pos = s;
        if (lane >= 1 && lane <= 7) pos = lower_bound(K, s, e, ((pre << 3) | (u64)lane) << sh);
        if (lane == 8) pos = e;
        const int64_t next = __shfl_down(pos, 1, 64);
        const bool nonempty = lane < 8 && next > pos;
        const u64 m = __ballot(nonempty);
        const int cnt = __popcll(m);
        if (nonempty) {
            const int k = __popcll(m & ((1ull << lane) - 1ull));
            crun[9 * r + k] = (unsigned)pos;
        }
        if (lane == 0) {
            crun[9 * r + cnt] = (unsigned)e;
            nchild[r] = (unsigned)cnt;
        }
    }
}

__device__ inline void zero_stats(BhNode &nd) {
    nd.cx = nd.cy = nd.cz = nd.s2 = 0.0;
    for (int c = 0; c < 3; ++c) nd.lo[c] = nd.hi[c] = 0.0;
    nd.px = nd.py = nd.pz = 0.f;
    nd.pad0 = nd.pad1 = 0;
}

// Root records: one thread per set, after the scans.  Node s is the root of
// set s; children of internal rank r start at node nsub + cstart[r].

// Node records of the children of every internal node, one wave per node:
// lane k builds child k (its representative found by its own search).
// The root of set si (node si): a leaf, or the internal node of its first
// split.
__device__ inline void make_root(int si, const u64 *__restrict__ K, int64_t n,
                                 const long long *__restrict__ seg, int nsub, int leaf_cap,
                                 const unsigned *__restrict__ rank,
                                 const unsigned *__restrict__ nchild,
                                 const unsigned *__restrict__ cstart,
                                 TreeTotals *__restrict__ totals, TreeMeta *__restrict__ meta,
                                 BhNode *__restrict__ nodes, int *__restrict__ node_start) {
    const int64_t a = seg ? seg[si] : 0, b = seg ? seg[si + 1] : n;
    BhNode nd;
    zero_stats(nd);
    nd.n = (int)(b - a);
    if (b - a <= leaf_cap || K[a] == K[b - 1]) {
        nd.first = (int)a;
        nd.nchild = 0;
        meta[si].root_leaf = 1;
        meta[si].root_rank = -1;
    } else {
        const unsigned r = rank[child_rep(K, a, b)];
        nd.first = nsub + (int)cstart[r];
        nd.nchild = (int)nchild[r];
        meta[si].root_leaf = 0;
        meta[si].root_rank = (int)r;
    }
    nodes[si] = nd;
    node_start[si] = (int)a;
    if (si == 0) {
        const int m = totals->n_internal;
        totals->n_nodes = nsub + (m > 0 ? (int)(cstart[m - 1] + nchild[m - 1]) : 0);
    }
}

// Node records: the roots (one thread each), then the children of every
// internal rank (one wave per rank, a lane per child).
__global__ __launch_bounds__(256) void k_nodes(const u64 *__restrict__ K, int64_t n,
                                               const long long *__restrict__ seg, int leaf_cap,
                                               int nsub, TreeTotals *__restrict__ totals,
                                               TreeMeta *__restrict__ meta,
                                               const unsigned *__restrict__ rank,
                                               const unsigned *__restrict__ nchild,
                                               const unsigned *__restrict__ cstart,
                                               const unsigned *__restrict__ crun,
                                               BhNode *__restrict__ nodes,
                                               int *__restrict__ node_start,
                                               const RangeStat *__restrict__ c0, int64_t nc0,
                                               RangeStat *__restrict__ c1, int64_t nc1) {
    {  // summaries of 4096 sorted points (one wave each), for the statistics
        const int64_t waves = (int64_t)gridDim.x * 4;
        for (int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < nc1; c += waves) {
            RangeStat r;
            rs_init(r);
            const int64_t i = c * kChunk + (threadIdx.x & 63);
            if (i < nc0) r = c0[i];
            rs_wave_reduce(r);
            if ((threadIdx.x & 63) == 0) c1[c] = r;
        }
    }
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < nsub;
         si += gridDim.x * blockDim.x)
        make_root(si, K, n, seg, nsub, leaf_cap, rank, nchild, cstart, totals, meta, nodes,
                  node_start);
    const int lane = threadIdx.x & 63;
    const int64_t nint = totals->n_internal, waves = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nint; r += waves) {
        const int cnt = (int)nchild[r];
        if (lane >= cnt) continue;
        const int id = nsub + (int)cstart[r] + lane;
        const int64_t a = crun[9 * r + lane], b = crun[9 * r + lane + 1];
        BhNode nd;
        zero_stats(nd);
        nd.n = (int)(b - a);
        if (b - a <= leaf_cap || K[a] == K[b - 1]) {
            nd.first = (int)a;
            nd.nchild = 0;
        } else {
            const unsigned rc = rank[child_rep(K, a, b)];
            nd.first = nsub + (int)cstart[rc];
            nd.nchild = (int)nchild[rc];
        }
        nodes[id] = nd;
        node_start[id] = (int)a;
    }
}

// Statistics of a node from FP64 sums, box and count.
__device__ inline void finish_node(BhNode &nd, const double *sum, const float *lo,
                                   const float *hi) {
    const double inv = nd.n > 0 ? 1.0 / (double)nd.n : 0.0;  // n == 0: an empty set's root
    nd.cx = sum[0] * inv;
    nd.cy = sum[1] * inv;
    nd.cz = sum[2] * inv;
    nd.px = (float)sum[3];
    nd.py = (float)sum[4];
    nd.pz = (float)sum[5];
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        nd.lo[c] = (double)lo[c];
        nd.hi[c] = (double)hi[c];
        const double side = (double)hi[c] - (double)lo[c];
        if (side > s) s = side;
    }
    nd.s2 = s * s;
}

__global__ __launch_bounds__(256) void k_chunks0(const float4 *__restrict__ Qs,
                                                 const float4 *__restrict__ Ps, int64_t n,
                                                 RangeStat *__restrict__ c0, int64_t nc0) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nc0) return;
    RangeStat r;
    rs_init(r);
    const int64_t i = c * kChunk + lane;
    if (i < n) rs_point(r, Qs[i], Ps[i]);
    rs_wave_reduce(r);
    if (lane == 0) c0[c] = r;
}

__global__ __launch_bounds__(256) void k_chunks1(const RangeStat *__restrict__ c0, int64_t nc0,
                                                 RangeStat *__restrict__ c1, int64_t nc1) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nc1) return;
    RangeStat r;
    rs_init(r);
    const int64_t i = c * kChunk + lane;
    if (i < nc0) r = c0[i];
    rs_wave_reduce(r);
    if (lane == 0) c1[c] = r;
}

// Statistics of the sorted range [a, b) by one wave: the range splits into
// points up to the first chunk boundary, chunks up to the first super-chunk
// boundary, super-chunks, chunks and points; the lanes take the items of
// each part in turn and the wave adds its lanes in a fixed shuffle tree
// (bitwise deterministic).
__device__ inline void wave_range_stat(const float4 *__restrict__ A, const float4 *__restrict__ B,
                                       const RangeStat *__restrict__ c0,
                                       const RangeStat *__restrict__ c1, int64_t a, int64_t b,
                                       int lane, RangeStat &r) {
    constexpr int64_t C0 = kChunk, C1 = (int64_t)kChunk * kChunk;
    const int64_t ra = (a + C0 - 1) / C0 * C0, rb = b / C0 * C0;
    const int64_t p0 = ra < b ? ra : b;        // end of the leading points
    const int64_t p1 = rb > p0 ? rb : p0;      // start of the trailing points
    const int64_t sa = (p0 + C1 - 1) / C1 * C1, sb = p1 / C1 * C1;
    const int64_t s0 = sa < p1 ? sa : p1;      // end of the leading chunks
    const int64_t s1 = sb > s0 ? sb : s0;      // start of the trailing chunks
    rs_init(r);
    for (int64_t i = a + lane; i < p0; i += 64) rs_point(r, A[i], B[i]);
    for (int64_t c = p0 / C0 + lane; c < s0 / C0; c += 64) rs_add(r, c0[c]);
    for (int64_t c = s0 / C1 + lane; c < s1 / C1; c += 64) rs_add(r, c1[c]);
    for (int64_t c = s1 / C0 + lane; c < p1 / C0; c += 64) rs_add(r, c0[c]);
    for (int64_t i = p1 + lane; i < b; i += 64) rs_point(r, A[i], B[i]);
    rs_wave_reduce(r);
}

// Sums of a RangeStat over the 16 lanes of each quarter of the wave.
__device__ inline void rs_quarter_reduce(RangeStat &r) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 6; ++c) r.s[c] += __shfl_xor(r.s[c], off, 16);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r.lo[c] = fminf(r.lo[c], __shfl_xor(r.lo[c], off, 16));
            r.hi[c] = fmaxf(r.hi[c], __shfl_xor(r.hi[c], off, 16));
        }
    }
}

// Nodes of at most kQuarterNode points are summed by a quarter of a wave
// (four nodes at once, a 16-lane reduction each), larger ones by a whole
// wave from the range summaries.  At 1.5M points (95k nodes, most of them
// leaves) the node statistics took 87 us with one wave per node.
constexpr int kQuarterNode = 256;

// Node statistics from its point range: wave w takes nodes 4 w .. 4 w + 3
// (a grid of at most kNodeBlocks blocks loops over the nodes).
__global__ __launch_bounds__(256) void k_node_stats(const float4 *__restrict__ Qs,
                                                    const float4 *__restrict__ Ps,
                                                    const RangeStat *__restrict__ c0,
                                                    const RangeStat *__restrict__ c1,
                                                    const TreeTotals *__restrict__ totals,
                                                    const int *__restrict__ node_start,
                                                    BhNode *__restrict__ nodes,
                                                    double *__restrict__ nsum) {
    const int lane = threadIdx.x & 63, qk = lane >> 4, ql = lane & 15;
    const int64_t nn = totals->n_nodes, waves = (int64_t)gridDim.x * 4;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); 4 * w < nn; w += waves) {
        const int64_t id = 4 * w + qk;
        const bool has = id < nn;
        const int cnt = has ? nodes[id].n : 0;
        const int64_t a = has ? node_start[id] : 0;
        if (__all(cnt <= kQuarterNode)) {
            RangeStat r;
            rs_init(r);
            for (int64_t i = a + ql; i < a + cnt; i += 16) rs_point(r, Qs[i], Ps[i]);
            rs_quarter_reduce(r);
            if (ql == 0 && has) {
                BhNode nd = nodes[id];
                finish_node(nd, r.s, r.lo, r.hi);
                nodes[id] = nd;
                for (int c = 0; c < 6; ++c) nsum[6 * id + c] = r.s[c];
            }
        } else {
            for (int k = 0; k < 4 && 4 * w + k < nn; ++k) {
                const int64_t idk = 4 * w + k;
                BhNode nd = nodes[idk];
                const int64_t ak = node_start[idk];
                RangeStat r;
                wave_range_stat(Qs, Ps, c0, c1, ak, ak + nd.n, lane, r);
                if (lane == 0) {
                    finish_node(nd, r.s, r.lo, r.hi);
                    nodes[idk] = nd;
                    for (int c = 0; c < 6; ++c) nsum[6 * idk + c] = r.s[c];
                }
            }
        }
    }
}

// Node sums of two fields over node ranges (the sums part of k_node_stats,
// split the same way).
__global__ __launch_bounds__(256) void k_node_sums(const float4 *__restrict__ A,
                                                   const float4 *__restrict__ B,
                                                   const RangeStat *__restrict__ c0,
                                                   const RangeStat *__restrict__ c1,
                                                   const TreeTotals *__restrict__ totals,
                                                   const int *__restrict__ node_start,
                                                   const BhNode *__restrict__ nodes,
                                                   double *__restrict__ out) {
    const int lane = threadIdx.x & 63, qk = lane >> 4, ql = lane & 15;
    const int64_t nn = totals->n_nodes, waves = (int64_t)gridDim.x * 4;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); 4 * w < nn; w += waves) {
        const int64_t id = 4 * w + qk;
        const bool has = id < nn;
        const int cnt = has ? nodes[id].n : 0;
        const int64_t a = has ? node_start[id] : 0;
        if (__all(cnt <= kQuarterNode)) {
            RangeStat r;
            rs_init(r);
            for (int64_t i = a + ql; i < a + cnt; i += 16) rs_point(r, A[i], B[i]);
            rs_quarter_reduce(r);
            if (ql == 0 && has)
                for (int c = 0; c < 6; ++c) out[6 * id + c] = r.s[c];
        } else {
            for (int k = 0; k < 4 && 4 * w + k < nn; ++k) {
                const int64_t idk = 4 * w + k;
                const int64_t ak = node_start[idk];
                RangeStat r;
                wave_range_stat(A, B, c0, c1, ak, ak + nodes[idk].n, lane, r);
                if (lane == 0)
                    for (int c = 0; c < 6; ++c) out[6 * idk + c] = r.s[c];
            }
        }
    }
}

__global__ void k_copy_centres(const TreeMeta *__restrict__ meta, int nsub,
                               double *__restrict__ c0, float2 *__restrict__ c0f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * nsub) return;
    const double c = meta[i / 3].cen[i % 3];
    c0[i] = c;
    if (c0f) {
        const float ch = (float)c;
        c0f[i] = make_float2(ch, (float)(c - (double)ch));  // exact split
    }
}

// The state of float inputs: FP64 (Sq, Sp non-null) or hi+lo (Fq, Fp,
// (hi, lo) pairs), and its FP32 copies q32 = q - c0[set], p32 = p.
__global__ void k_state_init(const float *__restrict__ q, const float *__restrict__ p, int64_t n,
                             const long long *__restrict__ seg, int nsub,
                             const double *__restrict__ c0, const float2 *__restrict__ c0f,
                             double *__restrict__ Sq, double *__restrict__ Sp,
                             float2 *__restrict__ Fq, float2 *__restrict__ Fp,
                             float *__restrict__ q32, float *__restrict__ p32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int si = set_of(seg, nsub, i);
    for (int k = 0; k < 3; ++k) {
        const float a = q[3 * i + k], b = p[3 * i + k];
        if (Fq) {
            Fq[3 * i + k] = make_float2(a, 0.f);
            Fp[3 * i + k] = make_float2(b, 0.f);
            const float2 c = c0f[3 * si + k];
            const ff r = ff_add(ff_two_sum(a, -c.x), -c.y);
            q32[3 * i + k] = r.h + r.l;
        } else {
            Sq[3 * i + k] = a;
            Sp[3 * i + k] = b;
            q32[3 * i + k] = (float)((double)a - c0[3 * si + k]);
        }
        p32[3 * i + k] = b;
    }
}

__global__ void k_state_to_f32(const double *__restrict__ Sq, const double *__restrict__ Sp,
                               int64_t n, const long long *__restrict__ seg, int nsub,
                               const double *__restrict__ c0, float *__restrict__ q32,
                               float *__restrict__ p32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *c = c0 + 3 * set_of(seg, nsub, i);
    for (int k = 0; k < 3; ++k) {
        q32[3 * i + k] = (float)(Sq[3 * i + k] - c[k]);
        p32[3 * i + k] = (float)Sp[3 * i + k];
    }
}

gs_status scan_u32(const unsigned *in, unsigned *out, int64_t n, unsigned *part, unsigned *total,
                   hipStream_t s, unsigned *scatter = nullptr, int64_t nscatter = 0) {
    const unsigned nb = (unsigned)((n + kScanTile - 1) / kScanTile);
    // one block needs no block totals (its carry is zero)
    if (nb > 1) hipLaunchKernelGGL(k_scan_blocksum, dim3(nb), dim3(256), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, in, out, n, part, total, scatter,
                       nscatter);
    GS_LAUNCH_CHECK("scan");
    return GS_OK;
}

}  // namespace

// ---------------------------------------------------------------- host side
void carve_forest(Arena &a, int64_t n, int nsub, int64_t groups, int64_t max_set, TreeBufs &t) {
    const int64_t m = n > 1 ? n : 1;
    const int64_t ms = max_set > 1 ? max_set : 1;
    const int64_t g = groups > 1 ? groups : 1;
    const int64_t nodes = 2 * m + nsub;
    t.n = n;
    t.nsub = nsub;
    t.seg = nullptr;
    t.gtab = nullptr;
    t.groups = groups;
    t.bbox_blocks = (int)((ms + 2047) / 2048 < 1024 ? (ms + 2047) / 2048 : 1024);
    t.sort_per = m >= kOsLargeFrom ? kOsPerLarge : kOsPerSmall;
    t.sort_tiles = (int)((m + 256 * t.sort_per - 1) / (256 * t.sort_per));
    t.sort_sbs = (t.sort_tiles + kSbTiles - 1) / kSbTiles;
    t.sort_passes = kKeyPasses + (nsub > 1 ? (nsub > kOsBins ? 2 : 1) : 0);
    // 1: one block per set; 2: one set sorted in tiles and merged; 0: radix passes
    t.block_sort = max_set <= kBlockSortMax                                   ? 1
                   : nsub == 1 && n <= (int64_t)kMergeTiles * kBlockSortMax ? 2
                                                                            : 0;
    t.meta = a.take<TreeMeta>(nsub);
    t.totals = a.take<TreeTotals>(1);
    t.bbox_part = a.take<float>(6 * (size_t)t.bbox_blocks * nsub);
    t.keyA = a.take<u64>(m);
    t.keyB = a.take<u64>(m);
    t.valA = a.take<unsigned>(m);
    t.valB = a.take<unsigned>(m);
    t.K = (t.sort_passes & 1) && !t.block_sort ? t.keyB : t.keyA;
    t.perm = (t.sort_passes & 1) && !t.block_sort ? t.valB : t.valA;
    t.hist = a.take<unsigned>((size_t)kOsBins * t.sort_tiles);
    t.sb = a.take<unsigned>((size_t)2 * kOsBins * t.sort_sbs);
    t.scan_part = a.take<unsigned>((m + kScanTile - 1) / kScanTile + 1);
    t.Qs = a.take<float4>(m);
    t.Ps = a.take<float4>(m);
    t.Qc = a.take<float4>(m);
    t.lvl = a.take<unsigned char>(m);
    t.flag = a.take<unsigned>(m);
    t.rank = a.take<unsigned>(m);
    t.bnd_s = a.take<unsigned>(m);
    t.bnd_e = a.take<unsigned>(m);
    t.rank_bnd = a.take<unsigned>(m);
    t.nchild = a.take<unsigned>(m);
    t.cstart = a.take<unsigned>(m);
    t.crun = a.take<unsigned>(9 * (size_t)m);
    t.node_start = a.take<int>(nodes);
    t.chunk0 = reinterpret_cast<char *>(a.take<RangeStat>((m + kChunk - 1) / kChunk));
    t.chunk1 = reinterpret_cast<char *>(
        a.take<RangeStat>((m + kChunk * kChunk - 1) / (kChunk * kChunk)));
    t.nsum = a.take<double>(6 * nodes);
    t.nodes = a.take<BhNode>(nodes);
    t.adj = a.take<double>(6 * nodes);
    t.list = a.take<char>(traverse_list_bytes(g));
    t.list_n = a.take<int>(traverse_count_ints(g));
    t.part = a.take<double>(traverse_part_doubles(g));
}

void carve_tree(Arena &a, int64_t n, TreeBufs &t) { carve_forest(a, n, 1, (n + 63) / 64, n, t); }

static gs_status build_from_sorted(const float *q, const float *p, int64_t n, int leaf_cap,
                                   TreeBufs &t, hipStream_t s);

gs_status build_tree(const float *q, const float *p, int64_t n, int leaf_cap, TreeBufs &t,
                     int *status, hipStream_t s) {
    timing_begin(KIND_TREE, s);
    const int nsub = t.nsub;
    const int64_t sbn = (int64_t)kOsBins * t.sort_sbs;  // counts per superblock buffer
    hipLaunchKernelGGL(k_bbox_partial, dim3(t.bbox_blocks, nsub), dim3(256), 0, s, q, n, t.seg,
                       t.bbox_part, t.sb, sbn);
    hipLaunchKernelGGL(k_bbox_final, dim3(nsub), dim3(64), 0, s, t.bbox_part, t.bbox_blocks,
                       t.meta, status);
    if (t.block_sort == 1) {
        hipLaunchKernelGGL(k_block_radix, dim3(nsub), dim3(256), 0, s, q, t.seg, t.meta, n, 0,
                           t.keyA, t.valA);
        GS_LAUNCH_CHECK("block sort");
        return build_from_sorted(q, p, n, leaf_cap, t, s);
    }
    if (t.block_sort == 2) {
        const int tiles = (int)((n + kBlockSortMax - 1) / kBlockSortMax);
        hipLaunchKernelGGL(k_block_radix, dim3(tiles), dim3(256), 0, s, q, t.seg, t.meta, n,
                           kBlockSortMax, t.keyB, t.valB);
        hipLaunchKernelGGL(k_merge_rank, dim3(nblk(n)), dim3(256), 0, s, t.keyB, t.valB, n,
                           kBlockSortMax, t.keyA, t.valA);
        GS_LAUNCH_CHECK("tile sort and merge");
        return build_from_sorted(q, p, n, leaf_cap, t, s);
    }
    const unsigned tiles = (unsigned)t.sort_tiles;
    const bool large = t.sort_per == kOsPerLarge;
    if (large)
        hipLaunchKernelGGL(k_morton_hist<kOsPerLarge>, dim3(tiles), dim3(256), 0, s, q, n, t.seg,
                           nsub, t.meta, t.keyA, t.valA, t.hist, t.sb);
    else
        hipLaunchKernelGGL(k_morton_hist<kOsPerSmall>, dim3(tiles), dim3(256), 0, s, q, n, t.seg,
                           nsub, t.meta, t.keyA, t.valA, t.hist, t.sb);
    GS_LAUNCH_CHECK("bbox/morton");
    u64 *ki = t.keyA, *ko = t.keyB;
    unsigned *vi = t.valA, *vo = t.valB;
    for (int pass = 0; pass < t.sort_passes; ++pass) {
        unsigned *sb_cur = t.sb + (pass & 1) * sbn, *sb_next = t.sb + ((pass + 1) & 1) * sbn;
#define GS_OS_PASS(PER)                                                                       \
    do {                                                                                      \
        if (pass > 0)                                                                         \
            hipLaunchKernelGGL(k_os_hist<PER>, dim3(tiles), dim3(256), 0, s, ki, vi, n, pass,  \
                               t.seg, nsub, t.hist, sb_cur);                                  \
        hipLaunchKernelGGL(k_os_scatter<PER>, dim3(tiles), dim3(256), 0, s, ki, vi, ko, vo, n, \
                           pass, t.seg, nsub, t.hist, sb_cur, t.sort_sbs, sb_next);           \
    } while (0)
        if (large)
            GS_OS_PASS(kOsPerLarge);
        else
            GS_OS_PASS(kOsPerSmall);
#undef GS_OS_PASS
        u64 *tk = ki;
        ki = ko;
        ko = tk;
        unsigned *tv = vi;
        vi = vo;
        vo = tv;
    }
    GS_LAUNCH_CHECK("radix sort");
    return build_from_sorted(q, p, n, leaf_cap, t, s);
}

// The octree from the sorted keys and permutation (t.K, t.perm).
static gs_status build_from_sorted(const float *q, const float *p, int64_t n, int leaf_cap,
                                   TreeBufs &t, hipStream_t s) {
    const int nsub = t.nsub;
    const u64 *K = t.K;
    const int64_t nc0 = (n + kChunk - 1) / kChunk, nc1 = (nc0 + kChunk - 1) / kChunk;
    RangeStat *c0 = reinterpret_cast<RangeStat *>(t.chunk0);
    RangeStat *c1 = reinterpret_cast<RangeStat *>(t.chunk1);
    hipLaunchKernelGGL(k_boundaries, dim3(nblk(n)), dim3(256), 0, s, K, n, t.seg, nsub, leaf_cap,
                       q, p, t.perm, t.meta, t.Qs, t.Ps, t.Qc, c0, nc0, t.lvl, t.flag, t.bnd_s,
                       t.bnd_e);
    GS_LAUNCH_CHECK("boundaries");
    unsigned *n_internal = reinterpret_cast<unsigned *>(&t.totals->n_internal);
    // ranks of the internal boundaries, and the boundary of every rank
    GS_TRY(scan_u32(t.flag, t.rank, n, t.scan_part, n_internal, s, t.rank_bnd, n - 1));
    hipLaunchKernelGGL(k_children, dim3(node_blocks(n)), dim3(256), 0, s, K, t.lvl, t.totals,
                       t.bnd_s, t.bnd_e, t.rank_bnd, t.nchild, t.crun);
    GS_LAUNCH_CHECK("children");
    // nchild of ranks >= n_internal is never read; the scan covers n - 1
    // entries whose tail beyond n_internal may hold stale values, which only
    // affects cstart of ranks that do not exist.
    GS_TRY(scan_u32(t.nchild, t.cstart, n > 1 ? n - 1 : 1, t.scan_part, nullptr, s));
    hipLaunchKernelGGL(k_nodes, dim3(node_blocks(n)), dim3(256), 0, s, K, n, t.seg, leaf_cap,
                       nsub, t.totals, t.meta, t.rank, t.nchild, t.cstart, t.crun, t.nodes,
                       t.node_start, c0, nc0, c1, nc1);
    hipLaunchKernelGGL(k_node_stats, dim3(node_blocks(2 * n + nsub)), dim3(256), 0, s, t.Qs, t.Ps, c0,
                       c1, t.totals, t.node_start, t.nodes, t.nsum);
    timing_end(KIND_TREE, s);
    GS_LAUNCH_CHECK("nodes/stats");
    return GS_OK;
}

gs_status tree_set_centres(const float *q, TreeBufs &t, double *c0, float2 *c0f, int *status,
                           hipStream_t s) {
    const int nsub = t.nsub;
    hipLaunchKernelGGL(k_bbox_partial, dim3(t.bbox_blocks, nsub), dim3(256), 0, s, q, t.n, t.seg,
                       t.bbox_part, nullptr, (int64_t)0);
    hipLaunchKernelGGL(k_bbox_final, dim3(nsub), dim3(64), 0, s, t.bbox_part, t.bbox_blocks,
                       t.meta, status);
    hipLaunchKernelGGL(k_copy_centres, dim3(nblk(3 * (int64_t)nsub)), dim3(256), 0, s, t.meta,
                       nsub, c0, c0f);
    GS_LAUNCH_CHECK("set_centres");
    return GS_OK;
}

gs_status launch_state_init(const float *q0, const float *p0, const TreeBufs &t, const double *c0,
                            const float2 *c0f, double *Sq, double *Sp, float2 *Fq, float2 *Fp,
                            float *q32, float *p32, hipStream_t s) {
    if (t.n == 0) return GS_OK;
    hipLaunchKernelGGL(k_state_init, dim3(nblk(t.n)), dim3(256), 0, s, q0, p0, t.n, t.seg, t.nsub,
                       c0, c0f, Sq, Sp, Fq, Fp, q32, p32);
    GS_LAUNCH_CHECK("state_init");
    return GS_OK;
}

gs_status launch_state_to_f32(const double *Sq, const double *Sp, const TreeBufs &t,
                              const double *c0, float *q32, float *p32, hipStream_t s) {
    if (t.n == 0) return GS_OK;
    hipLaunchKernelGGL(k_state_to_f32, dim3(nblk(t.n)), dim3(256), 0, s, Sq, Sp, t.n, t.seg,
                       t.nsub, c0, q32, p32);
    GS_LAUNCH_CHECK("state_to_f32");
    return GS_OK;
}

gs_status tree_range_sums(const float4 *A, const float4 *B, TreeBufs &t, double *out,
                          hipStream_t s) {
    const int64_t n = t.n;
    const int64_t nc0 = (n + kChunk - 1) / kChunk, nc1 = (nc0 + kChunk - 1) / kChunk;
    RangeStat *c0 = reinterpret_cast<RangeStat *>(t.chunk0);
    RangeStat *c1 = reinterpret_cast<RangeStat *>(t.chunk1);
    hipLaunchKernelGGL(k_chunks0, dim3(nblk(nc0, 4)), dim3(256), 0, s, A, B, n, c0, nc0);
    hipLaunchKernelGGL(k_chunks1, dim3(nblk(nc1, 4)), dim3(256), 0, s, c0, nc0, c1, nc1);
    hipLaunchKernelGGL(k_node_sums, dim3(node_blocks(2 * n + t.nsub)), dim3(256), 0, s, A, B, c0, c1,
                       t.totals, t.node_start, t.nodes, out);
    GS_LAUNCH_CHECK("range sums");
    return GS_OK;
}

}  // namespace gs
