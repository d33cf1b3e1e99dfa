// capi.cpp -- the extern "C" entry points of gs.h: argument validation,
// workspace planning and the launch sequences of each operation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "adjoint.h"
#include "internal.h"
#include "tree.h"

namespace gs {

// ---------------------------------------------------------------- errors
static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

gs_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return GS_ERR_HIP;
}

// ---------------------------------------------------------------- timing
namespace {
// set while a launch sequence is being captured into a graph: the timing
// events are then left out
thread_local bool g_capturing = false;

struct TimingState {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[KIND_COUNT];
    hipEvent_t open[KIND_COUNT] = {};
};
TimingState &timing() {
    static TimingState t;
    return t;
}
}  // namespace

void timing_begin(int kind, hipStream_t s) {
    if (g_capturing) return;
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    t.open[kind] = e;
}

void timing_end(int kind, hipStream_t s) {
    if (g_capturing) return;
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.on || !t.open[kind]) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    t.ev[kind].push_back({t.open[kind], e});
    t.open[kind] = nullptr;
}

}  // namespace gs

using namespace gs;

namespace {

// Every workspace starts with the status word and the Barnes-Hut counters
// (kWsHeader bytes).
constexpr size_t kHeader = kWsHeader;

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

gs_status check_params(const gs_params *prm, bool need_nt, bool need_tree) {
    if (!prm) {
        set_error("params is NULL");
        return GS_ERR_INVALID;
    }
    if (!finite_pos(prm->sigma)) {
        set_error("sigma must be finite and > 0 (got %g)", prm->sigma);
        return GS_ERR_INVALID;
    }
    if (need_nt && prm->nt < 1) {
        set_error("nt must be >= 1 (got %d)", prm->nt);
        return GS_ERR_INVALID;
    }
    if (need_tree) {
        if (std::isnan(prm->theta) || prm->theta < 0.0) {
            set_error("theta must be >= 0 (got %g)", prm->theta);
            return GS_ERR_INVALID;
        }
        if (std::isnan(prm->cutoff_sigmas) || prm->cutoff_sigmas <= 0.0) {
            set_error("cutoff_sigmas must be > 0 (got %g)", prm->cutoff_sigmas);
            return GS_ERR_INVALID;
        }
        if (prm->leaf_cap < 1 || prm->leaf_cap > 64) {
            set_error("leaf_cap must be in [1, 64] (got %d)", prm->leaf_cap);
            return GS_ERR_INVALID;
        }
    }
    if (prm->flags & ~(uint32_t)(GS_FLAG_F64 | GS_FLAG_GRAPH)) {
        set_error("unknown flags 0x%x", (unsigned)prm->flags);
        return GS_ERR_INVALID;
    }
    if (prm->exact_items != 0 && (prm->exact_items < 256 || prm->exact_items > (1 << 22))) {
        set_error("exact_items must be 0 or in [256, 4194304] (got %d)", prm->exact_items);
        return GS_ERR_INVALID;
    }
    return GS_OK;
}

gs_status check_n(int64_t n) {
    if (n < 0) {
        set_error("n must be >= 0 (got %lld)", (long long)n);
        return GS_ERR_INVALID;
    }
    if (n > (int64_t(1) << 31) - 4096) {
        set_error("n too large (%lld)", (long long)n);
        return GS_ERR_INVALID;
    }
    return GS_OK;
}

gs_status check_ptrs(std::initializer_list<const void *> ptrs) {
    for (const void *p : ptrs)
        if (!p) {
            set_error("NULL array argument");
            return GS_ERR_INVALID;
        }
    return GS_OK;
}

gs_status check_ws(void *ws, size_t have, size_t need) {
    if (!ws || have < need) {
        set_error("workspace too small: need %zu bytes, got %zu", need, have);
        return GS_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return GS_ERR_WORKSPACE;
    }
    return GS_OK;
}

// ---------------------------------------------------------------- layouts
// Every operation lays out its buffers with the same code whether it is
// measuring (base == nullptr) or carving the caller's workspace.
struct ShootF64Bufs {
    double *q, *p, *v, *a, *Hpart;
};

ShootF64Bufs layout_shoot_f64(Arena &a, int64_t n, int nt) {
    ShootF64Bufs b{};
    b.q = a.take<double>(3 * n);
    b.p = a.take<double>(3 * n);
    b.v = a.take<double>(3 * n);
    b.a = a.take<double>(3 * n);
    b.Hpart = a.take<double>((size_t)(nt + 1) * combine_blocks(n));
    return b;
}

size_t measure_batch(const int64_t *off, int nsub, const gs_params &prm, int method, int op,
                     int ckpt = 8);
size_t measure_field(int64_t m, int64_t n, const gs_params &prm);

size_t measure_bytes(int64_t n, const gs_params *prm, int32_t method, int32_t op) {
    const bool f64 = (prm->flags & GS_FLAG_F64) != 0;
    if (op == GS_OP_FIELD) return measure_field(n, n, *prm);
    if (f64) {
        if (method != GS_EXACT) return 0;
        Arena a{nullptr, kHeader, 0};
        if (op == GS_OP_SHOOT) layout_shoot_f64(a, n, prm->nt);
        return op == GS_OP_RHS || op == GS_OP_SHOOT ? a.off + 256 : 0;
    }
    if (op != GS_OP_RHS && op != GS_OP_SHOOT && op != GS_OP_ADJOINT) return 0;
    const int64_t off[2] = {0, n};
    return measure_batch(off, 1, *prm, method, op);
}

// ---------------------------------------------------------------- batched sets
gs_status check_offsets(const int64_t *off, int32_t nsub) {
    if (!off) {
        set_error("offsets is NULL");
        return GS_ERR_INVALID;
    }
    if (nsub < 1 || nsub > 65536) {
        set_error("nsub must be in [1, 65536] (got %d)", nsub);
        return GS_ERR_INVALID;
    }
    if (off[0] != 0) {
        set_error("offsets[0] must be 0 (got %lld)", (long long)off[0]);
        return GS_ERR_INVALID;
    }
    int64_t rows = 0;
    for (int s = 0; s < nsub; ++s) {
        if (off[s + 1] < off[s]) {
            set_error("offsets must be non-decreasing (offsets[%d] > offsets[%d])", s, s + 1);
            return GS_ERR_INVALID;
        }
        rows += round_up(off[s + 1] - off[s], 256);
    }
    GS_TRY(check_n(off[nsub]));
    if (rows > (int64_t(1) << 31) - 4096) {
        set_error("too many points once every set is padded to 256 (%lld)", (long long)rows);
        return GS_ERR_INVALID;
    }
    return GS_OK;
}

// Host image of the small device tables of a batched call (uploaded once per
// call); entries start at 256-byte boundaries.
struct TableImage {
    std::vector<char> bytes;
    template <class T>
    size_t add(const T *src, size_t count) {
        const size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + count * sizeof(T));
        if (count) memcpy(bytes.data() + off, src, count * sizeof(T));
        return off;
    }
};

// Work-item plans of the exact path, kept for repeated calls with the same
// set sizes: planning takes host time (about 0.1 ms for 20 000 points,
// 0.5 ms for 200 000) that a short call would otherwise wait for, and every
// call plans twice (workspace check and layout).  At most 8 plans are kept,
// least recently used dropped; the cache lives until the process ends.
struct PlanCache {
    std::mutex mu;
    struct Entry {
        std::vector<int64_t> key;
        std::shared_ptr<const ExactBatchPlan> plan;
        uint64_t used;
    };
    std::vector<Entry> entries;
    uint64_t clock = 0;
};

std::shared_ptr<const ExactBatchPlan> exact_plan(const int64_t *off, int nsub, int64_t items) {
    static PlanCache *c = new PlanCache;
    std::vector<int64_t> key(off, off + nsub + 1);
    key.push_back(items);
    std::lock_guard<std::mutex> g(c->mu);
    ++c->clock;
    for (auto &e : c->entries)
        if (e.key == key) {
            e.used = c->clock;
            return e.plan;
        }
    auto plan = std::make_shared<const ExactBatchPlan>(plan_exact_batch(off, nsub, items));
    if (c->entries.size() >= 8) {
        size_t old = 0;
        for (size_t i = 1; i < c->entries.size(); ++i)
            if (c->entries[i].used < c->entries[old].used) old = i;
        c->entries.erase(c->entries.begin() + (long)old);
    }
    c->entries.push_back({std::move(key), plan, c->clock});
    return plan;
}

struct Batch {
    std::shared_ptr<const ExactBatchPlan> plan;  // keeps *xp alive (several sets)
    ExactBatchPlan own;                          // one set: no tables
    const ExactBatchPlan *xp = nullptr;
    ExactBatchBufs ex{};
    ShootBhBufs bh{};
    AdjointBufs adj{};
    TableImage img;
    char *tables = nullptr;
};

// Lays out (or measures, when the arena has no base) the buffers of a
// batched call and prepares its tables.  `ckpt` is the checkpoint interval
// of op GS_OP_ADJOINT.  One set (nsub == 1) needs no tables: its kernels
// compute the work items, row blocks and traversal groups from its size, so
// such a call copies nothing from the host.  The Batch must stay where it is
// while in use (b.adj points into it).
void layout_batch(Arena &a, const int64_t *off, int nsub, const gs_params &prm, int method,
                  int op, Batch &b, int ckpt = 8) {
    const int nt = op == GS_OP_SHOOT ? prm.nt : 0;
    const bool adj = op == GS_OP_ADJOINT;
    const bool single = nsub == 1;
    const int ck = ckpt < prm.nt ? ckpt : prm.nt;
    const int64_t ntot = off[nsub];
    std::vector<double> setn;  // points of each set (backward stage)
    if (adj && !single)
        for (int s = 0; s < nsub; ++s) setn.push_back((double)(off[s + 1] - off[s]));
    if (method == GS_EXACT) {
        if (single) {
            b.own = plan_exact_single(ntot, prm.exact_items);
            b.xp = &b.own;
        } else {
            b.plan = exact_plan(off, nsub, prm.exact_items);
            b.xp = b.plan.get();
        }
        carve_exact_batch(a, *b.xp, nt,
                          op == GS_OP_SHOOT ? kStateFF : (adj ? kStateF64 : kStateNone), b.ex);
        const int nb = (int)plan_block_count(*b.xp);
        if (adj) {
            b.adj.AL = a.take<float4>(b.xp->npad);
            b.adj.BE = a.take<float4>(b.xp->npad);
            carve_adjoint_common(a, ntot, nsub, prm.nt, ck, nb, b.adj);
        }
        size_t o_items = 0, o_blk = 0, o_bseg = 0, o_setn = 0;
        if (!single) {
            o_items = b.img.add(b.xp->items.data(), b.xp->items.size());
            o_blk = b.img.add(b.xp->blocks.data(), b.xp->blocks.size());
            o_bseg = b.img.add(b.xp->bseg.data(), b.xp->bseg.size());
            o_setn = b.img.add(setn.data(), setn.size());
            b.tables = a.take<char>(b.img.bytes.size());
        }
        if (b.tables) {
            b.ex.items = reinterpret_cast<const int4 *>(b.tables + o_items);
            b.ex.blk = reinterpret_cast<const int4 *>(b.tables + o_blk);
            b.ex.bseg = reinterpret_cast<const int *>(b.tables + o_bseg);
        }
        if (adj) {  // reduction units: the row blocks, which never straddle two sets
            b.adj.bh = false;
            b.adj.xp = b.xp;
            b.adj.ex = b.ex;
            b.adj.Sq = b.ex.Sq;
            b.adj.Sp = b.ex.Sp;
            b.adj.hpart = b.ex.Hpart;
            b.adj.nh = nb;
            b.adj.hseg = b.ex.bseg;
            b.adj.units = b.ex.blk;
            b.adj.urows = b.xp->rows;
            b.adj.useg = b.ex.bseg;
            b.adj.setn = b.tables ? reinterpret_cast<const double *>(b.tables + o_setn) : nullptr;
        }
        return;
    }
    // forest: one tree per set; traversal groups never straddle two sets
    std::vector<long long> seg(nsub + 1);
    std::vector<GroupDesc> gt;
    std::vector<int> gseg(nsub + 1);
    int64_t max_set = 0, ngroups = 0;
    for (int s = 0; s < nsub; ++s) {
        seg[s] = off[s];
        gseg[s] = (int)ngroups;
        const int64_t n = off[s + 1] - off[s];
        if (n > max_set) max_set = n;
        for (int64_t g = 0; g * 64 < n; ++g, ++ngroups) {
            if (single) continue;  // group g of one set: points [64 g, 64 g + 64)
            GroupDesc d;
            d.first = (int)(off[s] + 64 * g);
            d.count = (int)(n - 64 * g < 64 ? n - 64 * g : 64);
            d.root = s;
            d.sub = s;
            gt.push_back(d);
        }
    }
    seg[nsub] = off[nsub];
    gseg[nsub] = (int)ngroups;
    if (op == GS_OP_SHOOT || adj)
        b.bh = layout_shoot_forest(a, ntot, nsub, ngroups, max_set, nt,
                                   adj ? kStateF64 : kStateFF);
    else
        carve_forest(a, ntot, nsub, ngroups, max_set, b.bh.tree);
    // reduction units of the backward stage: blocks of <= 256 points of one set
    std::vector<int4> units;
    std::vector<int> useg(nsub + 1);
    int64_t nunits = 0;
    if (adj) {
        for (int s = 0; s < nsub; ++s) {
            useg[s] = (int)nunits;
            for (int64_t i = off[s]; i < off[s + 1]; i += 256, ++nunits)
                if (!single)
                    units.push_back(make_int4((int)i, (int)std::min<int64_t>(256, off[s + 1] - i),
                                              s, 0));
        }
        useg[nsub] = (int)nunits;
        b.adj.bhadj = layout_bh_adjoint(a, ntot);
        carve_adjoint_common(a, ntot, nsub, prm.nt, ck, (int)nunits, b.adj);
    }
    size_t o_seg = 0, o_gt = 0, o_gseg = 0, o_units = 0, o_useg = 0, o_setn = 0;
    if (!single) {
        o_seg = b.img.add(seg.data(), seg.size());
        o_gt = b.img.add(gt.data(), gt.size());
        o_gseg = b.img.add(gseg.data(), gseg.size());
        o_units = b.img.add(units.data(), units.size());
        o_useg = b.img.add(useg.data(), adj ? useg.size() : 0);
        o_setn = b.img.add(setn.data(), setn.size());
        b.tables = a.take<char>(b.img.bytes.size());
    }
    if (b.tables) {
        b.bh.tree.seg = reinterpret_cast<const long long *>(b.tables + o_seg);
        b.bh.tree.gtab = reinterpret_cast<const GroupDesc *>(b.tables + o_gt);
        b.bh.gseg = reinterpret_cast<const int *>(b.tables + o_gseg);
    }
    if (adj) {
        b.adj.bh = true;
        b.adj.xp = nullptr;
        b.adj.sh = b.bh;
        b.adj.Sq = b.bh.Sq;
        b.adj.Sp = b.bh.Sp;
        b.adj.hpart = b.bh.Hpart;
        b.adj.nh = (int)ngroups;
        b.adj.hseg = b.bh.gseg;
        b.adj.urows = row_geom(ntot, 0);
        if (b.tables) {
            b.adj.units = reinterpret_cast<const int4 *>(b.tables + o_units);
            b.adj.useg = reinterpret_cast<const int *>(b.tables + o_useg);
            b.adj.setn = reinterpret_cast<const double *>(b.tables + o_setn);
        } else {
            b.adj.units = nullptr;
            b.adj.useg = nullptr;
            b.adj.setn = nullptr;
        }
    }
}

size_t measure_batch(const int64_t *off, int nsub, const gs_params &prm, int method, int op,
                     int ckpt) {
    Arena a{nullptr, kHeader, 0};
    Batch b;
    layout_batch(a, off, nsub, prm, method, op, b, ckpt);
    return a.off + 256;
}

// Buffers and tables of the velocity field (m targets, n sources).
struct Field {
    ExactBatchPlan plan;
    ExactBatchBufs ex{};
    TableImage img;
    char *tables = nullptr;
};

void layout_field(Arena &a, int64_t m, int64_t n, const gs_params &prm, Field &f) {
    f.plan = plan_exact_field(m, n, prm.exact_items);
    carve_exact_field(a, f.plan, f.ex);
    const size_t o_items = f.img.add(f.plan.items.data(), f.plan.items.size());
    const size_t o_blk = f.img.add(f.plan.blocks.data(), f.plan.blocks.size());
    const size_t o_sblk = f.img.add(f.plan.sblocks.data(), f.plan.sblocks.size());
    const size_t o_sbseg = f.img.add(f.plan.sbseg.data(), f.plan.sbseg.size());
    f.tables = a.take<char>(f.img.bytes.size());
    if (f.tables) {
        f.ex.items = reinterpret_cast<const int4 *>(f.tables + o_items);
        f.ex.blk = reinterpret_cast<const int4 *>(f.tables + o_blk);
        f.ex.sblk = reinterpret_cast<const int4 *>(f.tables + o_sblk);
        f.ex.sbseg = reinterpret_cast<const int *>(f.tables + o_sbseg);
        f.ex.bseg = nullptr;
    }
}

size_t measure_field(int64_t m, int64_t n, const gs_params &prm) {
    Arena a{nullptr, kHeader, 0};
    Field f;
    layout_field(a, m, n, prm, f);
    return a.off + 256;
}

// Pinned staging buffers for the table uploads of batched calls (several
// sets) and of the velocity field, per thread.  A call takes the next buffer
// whose previous copy has completed (hipEventQuery, no waiting); when every
// buffer is still in flight the ring grows, up to kStageMax buffers, so a
// call waits on the host only when it is issued while kStageMax earlier
// uploads of its thread are still queued on the device.  The buffers live
// until the process ends.
constexpr size_t kStageMax = 32;
struct StageSlot {
    void *buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
struct Stage {
    std::vector<StageSlot> slot;
    size_t next = 0;
};
thread_local Stage g_stage;

gs_status upload_tables(const TableImage &img, char *dev, hipStream_t s) {
    const size_t bytes = img.bytes.size();
    if (bytes == 0) return GS_OK;
    Stage &st = g_stage;
    StageSlot *sl = nullptr;
    for (size_t k = 0; k < st.slot.size() && !sl; ++k) {
        const size_t i = (st.next + k) % st.slot.size();
        StageSlot &c = st.slot[i];
        if (c.pending) {
            const hipError_t q = hipEventQuery(c.ev);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
            c.pending = false;
        }
        sl = &c;
        st.next = i + 1;
    }
    if (!sl && st.slot.size() < kStageMax) {
        st.slot.emplace_back();
        sl = &st.slot.back();
        st.next = st.slot.size();
    }
    if (!sl) {  // kStageMax uploads in flight: wait for the oldest
        const size_t i = st.next % st.slot.size();
        sl = &st.slot[i];
        GS_HIP(hipEventSynchronize(sl->ev));
        sl->pending = false;
        st.next = i + 1;
    }
    if (sl->cap < bytes) {
        if (sl->buf) GS_HIP(hipHostFree(sl->buf));
        sl->buf = nullptr;
        sl->cap = 0;
        GS_HIP(hipHostMalloc(&sl->buf, bytes, hipHostMallocDefault));
        sl->cap = bytes;
    }
    if (!sl->ev) GS_HIP(hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming));
    memcpy(sl->buf, img.bytes.data(), bytes);
    GS_HIP(hipMemcpyAsync(dev, sl->buf, bytes, hipMemcpyHostToDevice, s));
    GS_HIP(hipEventRecord(sl->ev, s));
    sl->pending = true;
    return GS_OK;
}

gs_status check_batch_call(const int64_t *offsets, int32_t nsub, const gs_params *prm,
                           int32_t method, bool need_nt) {
    GS_TRY(check_offsets(offsets, nsub));
    if (method != GS_EXACT && method != GS_BH) {
        set_error("unknown method %d", method);
        return GS_ERR_INVALID;
    }
    return check_params(prm, need_nt, method == GS_BH);
}

gs_status exact_batch_rhs(const float *q, const float *p, const int64_t *off, int nsub,
                          const gs_params &prm, float *dq, float *dp, void *ws, size_t ws_bytes,
                          hipStream_t stream) {
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Batch b;
    layout_batch(a, off, nsub, prm, GS_EXACT, GS_OP_RHS, b);
    GS_TRY(upload_tables(b.img, b.tables, stream));
    GS_TRY(launch_pack_state_rows(*b.xp, b.ex, q, p, prm.sigma, stream));
    GS_TRY(launch_exact_items(*b.xp, b.ex, true, stream));
    return launch_combine_rows(*b.xp, b.ex, prm.sigma, 0, dq, dp, 0.0, nullptr, stream);
}

gs_status exact_batch_shoot(const float *q0, const float *p0, const int64_t *off, int nsub,
                            const gs_params &prm, float *q1, float *p1, double *H, void *ws,
                            size_t ws_bytes, hipStream_t stream, bool upload = true) {
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Batch b;
    layout_batch(a, off, nsub, prm, GS_EXACT, GS_OP_SHOOT, b);
    if (upload) GS_TRY(upload_tables(b.img, b.tables, stream));
    const double dt = 1.0 / prm.nt;
    const size_t nb = (size_t)plan_block_count(*b.xp);
    GS_TRY(launch_pack_state_rows(*b.xp, b.ex, q0, p0, prm.sigma, stream));
    for (int t = 0; t < prm.nt; ++t) {
        GS_TRY(launch_exact_items(*b.xp, b.ex, true, stream));
        GS_TRY(launch_combine_rows(*b.xp, b.ex, prm.sigma, 1, nullptr, nullptr, dt,
                                   H ? b.ex.Hpart + (size_t)t * nb : nullptr, stream));
    }
    if (H) {
        // energy of the final state: one velocity-only pass
        GS_TRY(launch_exact_items(*b.xp, b.ex, false, stream));
        GS_TRY(launch_combine_rows(*b.xp, b.ex, prm.sigma, 1, nullptr, nullptr, 0.0,
                                   b.ex.Hpart + (size_t)prm.nt * nb, stream));
        GS_TRY(launch_reduce_h_seg(b.ex.Hpart, (int64_t)nb, b.ex.bseg, nsub, prm.nt + 1, H,
                                   stream));
    }
    return launch_unpack_state(b.ex.Fq, b.ex.Fp, off[nsub], q1, p1, stream);
}

// ---------------------------------------------------------------- graphs
// With GS_FLAG_GRAPH a call's kernel sequence is captured once into a HIP
// graph and replayed by later calls with the same arguments.  Capture runs on
// a library stream (the caller's stream may be the null stream, which cannot
// be captured); the graph is then launched on the caller's stream.  The
// small host-planned tables are uploaded by every call, before the graph, so
// a workspace that served other calls in between is refreshed.
struct GraphKey {
    int entry = 0;
    int device = 0;
    std::vector<uintptr_t> ptrs;
    std::vector<int64_t> ints;
    std::vector<double> dbls;
    bool operator==(const GraphKey &o) const {
        return entry == o.entry && device == o.device && ptrs == o.ptrs && ints == o.ints &&
               dbls == o.dbls;
    }
};

struct GraphCache {
    std::mutex mu;
    struct Entry {
        GraphKey key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<Entry> entries;
    uint64_t clock = 0;
    hipStream_t cap[64] = {};  // capture stream per device
};
GraphCache &graphs() {
    static GraphCache *c = new GraphCache;  // lives until the process ends
    return *c;
}
constexpr size_t kMaxGraphs = 16;

GraphKey graph_key(int entry, std::initializer_list<const void *> ptrs,
                   std::initializer_list<int64_t> ints, const gs_params &prm) {
    GraphKey k;
    k.entry = entry;
    (void)hipGetDevice(&k.device);
    for (const void *p : ptrs) k.ptrs.push_back(reinterpret_cast<uintptr_t>(p));
    k.ints.assign(ints.begin(), ints.end());
    k.ints.push_back(prm.leaf_cap);
    k.ints.push_back(prm.nt);
    k.ints.push_back((int64_t)prm.flags);
    k.ints.push_back(prm.exact_items);
    k.dbls = {prm.sigma, prm.cutoff_sigmas, prm.theta};
    return k;
}

// Replays the graph of `key`, capturing it first from `launches(stream)`.
template <class F>
gs_status run_graphed(GraphKey &&key, hipStream_t stream, F &&launches) {
    GraphCache &c = graphs();
    std::lock_guard<std::mutex> g(c.mu);
    ++c.clock;
    for (auto &e : c.entries)
        if (e.key == key) {
            e.used = c.clock;
            GS_HIP(hipGraphLaunch(e.exec, stream));
            return GS_OK;
        }
    if (key.device < 0 || key.device >= 64) {
        set_error("graph: device index out of range");
        return GS_ERR_UNSUPPORTED;
    }
    hipStream_t &cs = c.cap[key.device];
    if (!cs) GS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    GS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    const gs_status st = launches(cs);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (st != GS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
    if (c.entries.size() >= kMaxGraphs) {  // drop the least recently used graph
        size_t old = 0;
        for (size_t i = 1; i < c.entries.size(); ++i)
            if (c.entries[i].used < c.entries[old].used) old = i;
        (void)hipGraphExecDestroy(c.entries[old].exec);
        c.entries.erase(c.entries.begin() + (long)old);
    }
    c.entries.push_back({std::move(key), exec, c.clock});
    GS_HIP(hipGraphLaunch(exec, stream));
    return GS_OK;
}

// Objective and gradient of every set (one set: a batch of one); with
// GS_FLAG_GRAPH the kernel sequence is replayed from a graph.
gs_status adjoint_batch_call(const float *q0, const float *p0, const float *y,
                             const int64_t *off, int nsub, const gs_params &prm, int method,
                             double lambda, int ckpt, double *objective, float *grad, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_ws(ws, ws_bytes, measure_batch(off, nsub, prm, method, GS_OP_ADJOINT, ckpt)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Batch b;
    layout_batch(a, off, nsub, prm, method, GS_OP_ADJOINT, b, ckpt);
    GS_TRY(upload_tables(b.img, b.tables, stream));
    auto body = [&](hipStream_t s) -> gs_status {
        return shoot_adjoint(q0, p0, y, prm, lambda, objective, grad, b.adj,
                             static_cast<char *>(ws), s);
    };
    if (!(prm.flags & GS_FLAG_GRAPH)) return body(stream);
    GraphKey key = graph_key(3, {q0, p0, y, objective, grad, ws},
                             {method, (int64_t)ws_bytes, nsub, ckpt}, prm);
    key.ints.insert(key.ints.end(), off, off + nsub + 1);
    key.dbls.push_back(lambda);
    return run_graphed(std::move(key), stream, body);
}

}  // namespace

extern "C" {

const char *gs_version(void) { return "gsbh 0.1 (gfx950, HIP)"; }

const char *gs_last_error(void) { return g_err; }

void gs_params_default(gs_params *p) {
    if (!p) return;
    p->sigma = 1.0;
    p->cutoff_sigmas = 3.0;
    p->theta = 0.5;
    p->leaf_cap = 1;
    p->nt = 40;
    p->flags = 0;
    p->exact_items = 0;
}

size_t gs_workspace_bytes(int64_t n, const gs_params *prm, int32_t method, int32_t op) {
    if (check_n(n) != GS_OK || !prm) return 0;
    if (method != GS_EXACT && method != GS_BH) return 0;
    if (op == GS_OP_SHOOT && prm->nt < 1) return 0;
    return measure_bytes(n, prm, method, op);
}

gs_status gs_rhs_exact(const float *q, const float *p, int64_t n, const gs_params *prm,
                       float *dq, float *dp, void *ws, size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, false, false));
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp}));
    gs_params pr = *prm;
    pr.flags &= ~GS_FLAG_F64;
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, GS_EXACT, GS_OP_RHS)));
    const int64_t off[2] = {0, n};
    return exact_batch_rhs(q, p, off, 1, pr, dq, dp, ws, ws_bytes, stream);
}

gs_status gs_rhs_exact_f64(const double *q, const double *p, int64_t n, const gs_params *prm,
                           double *dq, double *dp, void *ws, size_t ws_bytes,
                           hipStream_t stream) {
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, false, false));
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp}));
    gs_params pr = *prm;
    pr.flags |= GS_FLAG_F64;
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, GS_EXACT, GS_OP_RHS)));
    return launch_exact_f64(q, p, n, prm->sigma, true, dq, dp, stream);
}

gs_status gs_shoot(const float *q0, const float *p0, int64_t n, const gs_params *prm,
                   int32_t method, float *q1, float *p1, double *H, void *ws, size_t ws_bytes,
                   hipStream_t stream) {
    GS_TRY(check_n(n));
    if (method != GS_EXACT && method != GS_BH) {
        set_error("unknown method %d", method);
        return GS_ERR_INVALID;
    }
    GS_TRY(check_params(prm, true, method == GS_BH));
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q0, p0, q1, p1}));
    gs_params pr = *prm;
    pr.flags &= ~(GS_FLAG_F64 | GS_FLAG_GRAPH);
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, method, GS_OP_SHOOT)));
    const int64_t off[2] = {0, n};
    // one set: no host tables, so the whole call is its kernel sequence
    auto body = [&](hipStream_t s) -> gs_status {
        if (method == GS_EXACT)
            return exact_batch_shoot(q0, p0, off, 1, pr, q1, p1, H, ws, ws_bytes, s, false);
        Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
        ShootBhBufs b = layout_shoot_bh(a, n, pr.nt);
        return shoot_bh(q0, p0, n, pr, q1, p1, H, b, static_cast<char *>(ws), s);
    };
    if (!(prm->flags & GS_FLAG_GRAPH)) return body(stream);
    return run_graphed(graph_key(1, {q0, p0, q1, p1, H, ws}, {n, method, (int64_t)ws_bytes}, *prm),
                       stream, body);
}

gs_status gs_shoot_f64(const double *q0, const double *p0, int64_t n, const gs_params *prm,
                       double *q1, double *p1, double *H, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, true, false));
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q0, p0, q1, p1}));
    gs_params pr = *prm;
    pr.flags |= GS_FLAG_F64;
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, GS_EXACT, GS_OP_SHOOT)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    ShootF64Bufs b = layout_shoot_f64(a, n, prm->nt);
    const int nblk = combine_blocks(n);
    const double dt = 1.0 / prm->nt;
    GS_TRY(launch_copy_f64(q0, b.q, 3 * n, stream));
    GS_TRY(launch_copy_f64(p0, b.p, 3 * n, stream));
    for (int t = 0; t < prm->nt; ++t) {
        GS_TRY(launch_exact_f64(b.q, b.p, n, prm->sigma, true, b.v, b.a, stream));
        GS_TRY(launch_euler_f64(b.q, b.p, b.v, b.a, n, dt,
                                H ? b.Hpart + (size_t)t * nblk : nullptr, stream));
    }
    if (H) {
        GS_TRY(launch_exact_f64(b.q, b.p, n, prm->sigma, false, b.v, b.a, stream));
        GS_TRY(launch_euler_f64(b.q, b.p, b.v, b.a, n, 0.0, b.Hpart + (size_t)prm->nt * nblk,
                                stream));
        GS_TRY(launch_reduce_h(b.Hpart, nblk, prm->nt + 1, H, stream));
    }
    GS_TRY(launch_copy_f64(b.q, q1, 3 * n, stream));
    return launch_copy_f64(b.p, p1, 3 * n, stream);
}

gs_status gs_rhs_bh(const float *q, const float *p, int64_t n, const gs_params *prm, float *dq,
                    float *dp, void *ws, size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, false, true));
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp}));
    gs_params pr = *prm;
    pr.flags &= ~GS_FLAG_F64;
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, GS_BH, GS_OP_RHS)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    TreeBufs t;
    carve_tree(a, n, t);
    return rhs_bh(q, p, n, *prm, dq, dp, t, static_cast<char *>(ws), stream);
}

size_t gs_adjoint_workspace_bytes(int64_t n, const gs_params *prm, int32_t method,
                                  int32_t ckpt_every) {
    if (check_n(n) != GS_OK || !prm || prm->nt < 1 || ckpt_every < 1) return 0;
    if (method != GS_EXACT && method != GS_BH) return 0;
    const int64_t off[2] = {0, n};
    return measure_batch(off, 1, *prm, method, GS_OP_ADJOINT, ckpt_every);
}

gs_status gs_shoot_adjoint(const float *q0, const float *p0, const float *target, int64_t n,
                           const gs_params *prm, int32_t method, double lambda,
                           int32_t ckpt_every, double *objective, float *grad_p0, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_n(n));
    if (method != GS_EXACT && method != GS_BH) {
        set_error("unknown method %d", method);
        return GS_ERR_INVALID;
    }
    GS_TRY(check_params(prm, true, method == GS_BH));
    if (!std::isfinite(lambda)) {
        set_error("lambda must be finite");
        return GS_ERR_INVALID;
    }
    if (ckpt_every < 1) {
        set_error("ckpt_every must be >= 1 (got %d)", ckpt_every);
        return GS_ERR_INVALID;
    }
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q0, p0, target, objective, grad_p0}));
    const int64_t off[2] = {0, n};
    return adjoint_batch_call(q0, p0, target, off, 1, *prm, method, lambda, ckpt_every,
                              objective, grad_p0, ws, ws_bytes, stream);
}

size_t gs_adjoint_batch_workspace_bytes(const int64_t *offsets, int32_t nsub,
                                        const gs_params *prm, int32_t method,
                                        int32_t ckpt_every) {
    if (check_batch_call(offsets, nsub, prm, method, true) != GS_OK || ckpt_every < 1) return 0;
    return measure_batch(offsets, nsub, *prm, method, GS_OP_ADJOINT, ckpt_every);
}

gs_status gs_shoot_adjoint_batch(const float *q0, const float *p0, const float *target,
                                 const int64_t *offsets, int32_t nsub, const gs_params *prm,
                                 int32_t method, double lambda, int32_t ckpt_every,
                                 double *objective, float *grad_p0, void *ws, size_t ws_bytes,
                                 hipStream_t stream) {
    GS_TRY(check_batch_call(offsets, nsub, prm, method, true));
    if (!std::isfinite(lambda)) {
        set_error("lambda must be finite");
        return GS_ERR_INVALID;
    }
    if (ckpt_every < 1) {
        set_error("ckpt_every must be >= 1 (got %d)", ckpt_every);
        return GS_ERR_INVALID;
    }
    if (offsets[nsub] == 0) return GS_OK;
    GS_TRY(check_ptrs({q0, p0, target, objective, grad_p0}));
    return adjoint_batch_call(q0, p0, target, offsets, nsub, *prm, method, lambda, ckpt_every,
                              objective, grad_p0, ws, ws_bytes, stream);
}

size_t gs_field_workspace_bytes(int64_t m, int64_t n, const gs_params *prm) {
    if (check_n(m) != GS_OK || check_n(n) != GS_OK || !prm) return 0;
    return measure_field(m, n, *prm);
}

gs_status gs_field(const float *x, int64_t m, const float *q, const float *p, int64_t n,
                   const gs_params *prm, float *v, void *ws, size_t ws_bytes,
                   hipStream_t stream) {
    GS_TRY(check_n(m));
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, false, false));
    if (m == 0) return GS_OK;
    GS_TRY(check_ptrs({x, v}));
    if (n == 0) {
        set_error("gs_field: no sources (n == 0) but m > 0 targets");
        return GS_ERR_INVALID;
    }
    GS_TRY(check_ptrs({q, p}));
    GS_TRY(check_ws(ws, ws_bytes, measure_field(m, n, *prm)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Field f;
    layout_field(a, m, n, *prm, f);
    GS_TRY(upload_tables(f.img, f.tables, stream));
    GS_TRY(launch_pack_field(f.plan, f.ex, x, q, p, prm->sigma, stream));
    GS_TRY(launch_exact_items(f.plan, f.ex, false, stream));
    return launch_combine_rows(f.plan, f.ex, prm->sigma, 0, v, nullptr, 0.0, nullptr, stream);
}

size_t gs_batch_workspace_bytes(const int64_t *offsets, int32_t nsub, const gs_params *prm,
                                int32_t method, int32_t op) {
    if (op != GS_OP_RHS && op != GS_OP_SHOOT && op != GS_OP_ADJOINT) return 0;
    if (check_batch_call(offsets, nsub, prm, method, op != GS_OP_RHS) != GS_OK) return 0;
    return measure_batch(offsets, nsub, *prm, method, op);
}

gs_status gs_rhs_batch(const float *q, const float *p, const int64_t *offsets, int32_t nsub,
                       const gs_params *prm, int32_t method, float *dq, float *dp, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_batch_call(offsets, nsub, prm, method, false));
    const int64_t n = offsets[nsub];
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp}));
    GS_TRY(check_ws(ws, ws_bytes, measure_batch(offsets, nsub, *prm, method, GS_OP_RHS)));
    if (method == GS_EXACT)
        return exact_batch_rhs(q, p, offsets, nsub, *prm, dq, dp, ws, ws_bytes, stream);
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Batch b;
    layout_batch(a, offsets, nsub, *prm, method, GS_OP_RHS, b);
    GS_TRY(upload_tables(b.img, b.tables, stream));
    return rhs_bh(q, p, n, *prm, dq, dp, b.bh.tree, static_cast<char *>(ws), stream);
}

gs_status gs_shoot_batch(const float *q0, const float *p0, const int64_t *offsets, int32_t nsub,
                         const gs_params *prm, int32_t method, float *q1, float *p1, double *H,
                         void *ws, size_t ws_bytes, hipStream_t stream) {
    GS_TRY(check_batch_call(offsets, nsub, prm, method, true));
    const int64_t n = offsets[nsub];
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q0, p0, q1, p1}));
    GS_TRY(check_ws(ws, ws_bytes, measure_batch(offsets, nsub, *prm, method, GS_OP_SHOOT)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    Batch b;
    layout_batch(a, offsets, nsub, *prm, method, GS_OP_SHOOT, b);
    GS_TRY(upload_tables(b.img, b.tables, stream));
    auto body = [&](hipStream_t s) -> gs_status {
        if (method == GS_EXACT)
            return exact_batch_shoot(q0, p0, offsets, nsub, *prm, q1, p1, H, ws, ws_bytes, s,
                                     false);
        return shoot_bh(q0, p0, n, *prm, q1, p1, H, b.bh, static_cast<char *>(ws), s);
    };
    if (!(prm->flags & GS_FLAG_GRAPH)) return body(stream);
    GraphKey key = graph_key(2, {q0, p0, q1, p1, H, ws}, {n, method, (int64_t)ws_bytes, nsub},
                             *prm);
    key.ints.insert(key.ints.end(), offsets, offsets + nsub + 1);
    return run_graphed(std::move(key), stream, body);
}

gs_status gs_autotune_leaf_cap(const float *q, const float *p, const int64_t *offsets,
                               int32_t nsub, gs_params *prm, float *dq, float *dp, void *ws,
                               size_t ws_bytes, hipStream_t stream, double *best_ms) {
    GS_TRY(check_batch_call(offsets, nsub, prm, GS_BH, false));
    const int64_t n = offsets[nsub];
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp}));
    GS_TRY(check_ws(ws, ws_bytes, measure_batch(offsets, nsub, *prm, GS_BH, GS_OP_RHS)));
    hipEvent_t e0, e1;
    GS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("autotune: hipEventCreate failed");
        return GS_ERR_HIP;
    }
    static const int caps[] = {8, 16, 32, 48, 64};
    gs_params trial = *prm;
    double best = 1e300;
    int best_cap = prm->leaf_cap;
    gs_status st = GS_OK;
    for (int cap : caps) {
        trial.leaf_cap = cap;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3 && st == GS_OK; ++rep) {  // the first run warms up
            if (hipEventRecord(e0, stream) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK)
                st = gs_rhs_batch(q, p, offsets, nsub, &trial, GS_BH, dq, dp, ws, ws_bytes,
                                  stream);
            if (st == GS_OK && hipEventRecord(e1, stream) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK && hipEventSynchronize(e1) != hipSuccess) st = GS_ERR_HIP;
            float ms = 0.f;
            if (st == GS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK && rep > 0 && ms < ms_min) ms_min = ms;
        }
        if (st != GS_OK) break;
        if (ms_min < best) {
            best = ms_min;
            best_cap = cap;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GS_OK) {
        if (st == GS_ERR_HIP) set_error("autotune: a HIP call failed");
        return st;
    }
    prm->leaf_cap = best_cap;
    if (best_ms) *best_ms = best;
    return GS_OK;
}

gs_status gs_autotune_exact(const float *q, const float *p, const int64_t *offsets, int32_t nsub,
                            gs_params *prm, float *dq, float *dp, void *ws, size_t ws_bytes,
                            hipStream_t stream, double *best_ms) {
    GS_TRY(check_batch_call(offsets, nsub, prm, GS_EXACT, false));
    const int64_t n = offsets[nsub];
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, dq, dp, ws}));
    static const int cands[] = {6144, 12288, 24576, 49152};
    gs_params trial = *prm;
    bool fits[4], any = false;
    for (int k = 0; k < 4; ++k) {
        trial.exact_items = cands[k];
        fits[k] = measure_batch(offsets, nsub, trial, GS_EXACT, GS_OP_RHS) <= ws_bytes;
        any = any || fits[k];
    }
    if (!any) {
        set_error("autotune: the workspace fits none of the candidates");
        return GS_ERR_WORKSPACE;
    }
    hipEvent_t e0, e1;
    GS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("autotune: hipEventCreate failed");
        return GS_ERR_HIP;
    }
    double best = 1e300;
    int best_items = cands[0];
    gs_status st = GS_OK;
    for (int k = 0; k < 4; ++k) {
        if (!fits[k]) continue;
        const int items = cands[k];
        trial.exact_items = items;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3 && st == GS_OK; ++rep) {  // the first run warms up
            if (hipEventRecord(e0, stream) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK)
                st = gs_rhs_batch(q, p, offsets, nsub, &trial, GS_EXACT, dq, dp, ws, ws_bytes,
                                  stream);
            if (st == GS_OK && hipEventRecord(e1, stream) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK && hipEventSynchronize(e1) != hipSuccess) st = GS_ERR_HIP;
            float ms = 0.f;
            if (st == GS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = GS_ERR_HIP;
            if (st == GS_OK && rep > 0 && ms < ms_min) ms_min = ms;
        }
        if (st != GS_OK) break;
        if (ms_min < best) {
            best = ms_min;
            best_items = items;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GS_OK) {
        if (st == GS_ERR_HIP) set_error("autotune: a HIP call failed");
        return st;
    }
    prm->exact_items = best_items;
    if (best_ms) *best_ms = best;
    return GS_OK;
}

gs_status gs_tree_export(const float *q, const float *p, int64_t n, const gs_params *prm,
                         void *ws, size_t ws_bytes, hipStream_t stream, int64_t max_nodes,
                         int64_t *n_nodes, uint64_t *keys, uint32_t *perm, int32_t *node_start,
                         int32_t *node_count, int32_t *node_first, int32_t *node_nchild,
                         double *node_stats) {
    GS_TRY(check_n(n));
    GS_TRY(check_params(prm, false, true));
    if (!n_nodes) {
        set_error("n_nodes is NULL");
        return GS_ERR_INVALID;
    }
    *n_nodes = 0;
    if (n == 0) return GS_OK;
    GS_TRY(check_ptrs({q, p, keys, perm}));
    if (max_nodes < 0) {
        set_error("max_nodes must be >= 0");
        return GS_ERR_INVALID;
    }
    if (max_nodes > 0)
        GS_TRY(check_ptrs({node_start, node_count, node_first, node_nchild, node_stats}));
    gs_params pr = *prm;
    pr.flags &= ~(GS_FLAG_F64 | GS_FLAG_GRAPH);
    GS_TRY(check_ws(ws, ws_bytes, measure_bytes(n, &pr, GS_BH, GS_OP_RHS)));
    Arena a{static_cast<char *>(ws), kHeader, ws_bytes};
    TreeBufs t;
    carve_tree(a, n, t);
    GS_TRY(build_tree(q, p, n, pr.leaf_cap, t, reinterpret_cast<int *>(ws), stream));
    GS_HIP(hipStreamSynchronize(stream));
    TreeTotals tot;
    GS_HIP(hipMemcpy(&tot, t.totals, sizeof(tot), hipMemcpyDeviceToHost));
    *n_nodes = tot.n_nodes;
    GS_HIP(hipMemcpy(keys, t.K, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    GS_HIP(hipMemcpy(perm, t.perm, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (tot.n_nodes > max_nodes) return GS_OK;
    std::vector<BhNode> nodes((size_t)tot.n_nodes);
    GS_HIP(hipMemcpy(nodes.data(), t.nodes, nodes.size() * sizeof(BhNode), hipMemcpyDeviceToHost));
    GS_HIP(hipMemcpy(node_start, t.node_start, nodes.size() * sizeof(int32_t),
                     hipMemcpyDeviceToHost));
    for (size_t k = 0; k < nodes.size(); ++k) {
        const BhNode &d = nodes[k];
        node_count[k] = d.n;
        node_first[k] = d.first;
        node_nchild[k] = d.nchild;
        const double st[13] = {d.cx, d.cy, d.cz, d.px, d.py, d.pz, d.lo[0], d.lo[1], d.lo[2],
                               d.hi[0], d.hi[1], d.hi[2], d.s2};
        memcpy(node_stats + 13 * k, st, sizeof(st));
    }
    return GS_OK;
}

gs_status gs_get_status(const void *ws, hipStream_t stream) {
    if (!ws) {
        set_error("workspace is NULL");
        return GS_ERR_INVALID;
    }
    GS_HIP(hipStreamSynchronize(stream));
    int32_t status = 0;
    GS_HIP(hipMemcpy(&status, ws, sizeof(status), hipMemcpyDeviceToHost));
    if (status == kStatusNonfinite) {
        set_error("non-finite coordinates met while building the octree");
        return GS_ERR_NONFINITE;
    }
    if (status == kStatusOverflow) {
        set_error("a Barnes-Hut traversal stack overflowed (its results are incomplete)");
        return GS_ERR_OVERFLOW;
    }
    if (status != 0) {
        set_error("unknown device status %d", (int)status);
        return GS_ERR_HIP;
    }
    return GS_OK;
}

gs_status gs_bh_counters(const void *ws, hipStream_t stream, int64_t out[GS_BH_COUNTERS]) {
    if (!ws || !out) {
        set_error("NULL argument");
        return GS_ERR_INVALID;
    }
    GS_HIP(hipStreamSynchronize(stream));
    unsigned long long c[kCounterSlots][GS_BH_COUNTERS];
    GS_HIP(hipMemcpy(c, static_cast<const char *>(ws) + kCountersOffset, sizeof(c),
                     hipMemcpyDeviceToHost));
    for (int k = 0; k < GS_BH_COUNTERS; ++k) {
        unsigned long long v = 0;
        for (int s = 0; s < kCounterSlots; ++s)
            v = k >= 6 ? (c[s][k] > v ? c[s][k] : v) : v + c[s][k];
        out[k] = (int64_t)v;
    }
    return GS_OK;
}

gs_status gs_kernel_timing(int32_t enable) {
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.on = enable != 0;
    return GS_OK;
}

gs_status gs_kernel_timing_read(int64_t counts[GS_TIMING_KINDS], double ms[GS_TIMING_KINDS]) {
    static_assert(GS_TIMING_KINDS == KIND_COUNT, "timing kinds");
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    for (int k = 0; k < KIND_COUNT; ++k) {
        double sum = 0.0;
        for (auto &pr : t.ev[k]) {
            GS_HIP(hipEventSynchronize(pr.second));
            float e = 0.f;
            GS_HIP(hipEventElapsedTime(&e, pr.first, pr.second));
            sum += e;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        if (counts) counts[k] = (int64_t)t.ev[k].size();
        if (ms) ms[k] = sum;
        t.ev[k].clear();
    }
    return GS_OK;
}

}  // extern "C"
