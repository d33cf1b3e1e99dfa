// noalloc.hip -- the exact right-hand side with its workspace in a static
// device array of the library, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).
//
// `scratch` below is a device-side array: in host code its name is only a
// host stand-in, never a device address.  Its device address is taken once
// per device with hipGetSymbolAddress (each device holds its own copy) and
// only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace gs {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // GS_STATIC_SCRATCH_BYTES
constexpr int64_t kStaticMaxN = 500000;               // GS_STATIC_MAX_N
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (set up on the
// first call there, with that device current).
gs_status scratch_ptr(void **out) {
    int dev = -1;
    GS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("gs_rhs_exact_static: device index %d out of range", dev);
        return GS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        GS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("gs_rhs_exact_static: no device address for the scratch array");
            return GS_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return GS_OK;
}

}  // namespace
}  // namespace gs

using gs::kScratchBytes;
using gs::kStaticMaxN;

static_assert(kScratchBytes == GS_STATIC_SCRATCH_BYTES, "header and library disagree");
static_assert(kStaticMaxN == GS_STATIC_MAX_N, "header and library disagree");

extern "C" gs_status gs_rhs_exact_static(const float *q, const float *p, int64_t n,
                                         const gs_params *prm, float *dq, float *dp,
                                         hipStream_t stream) {
    if (!prm) {
        gs::set_error("params is NULL");
        return GS_ERR_INVALID;
    }
    if (prm->exact_items != 0 && (prm->exact_items < 256 || prm->exact_items > (1 << 22))) {
        gs::set_error("exact_items must be 0 or in [256, 4194304] (got %d)", prm->exact_items);
        return GS_ERR_INVALID;
    }
    if (n > kStaticMaxN) {
        gs::set_error("gs_rhs_exact_static: n = %lld exceeds GS_STATIC_MAX_N = %lld",
                      (long long)n, (long long)kStaticMaxN);
        return GS_ERR_WORKSPACE;
    }
    if (n <= 0) return gs_rhs_exact(q, p, n, prm, dq, dp, nullptr, 0, stream);
    // the argument checks of gs_rhs_exact, before the array is set up
    if (!q || !p || !dq || !dp) {
        gs::set_error("NULL array argument");
        return GS_ERR_INVALID;
    }
    if (!(prm->sigma > 0.0) || !(prm->sigma < INFINITY)) {
        gs::set_error("sigma must be finite and > 0 (got %g)", prm->sigma);
        return GS_ERR_INVALID;
    }
    if (prm->flags & ~(uint32_t)(GS_FLAG_F64 | GS_FLAG_GRAPH)) {
        gs::set_error("unknown flags 0x%x", (unsigned)prm->flags);
        return GS_ERR_INVALID;
    }
    // Work-item target: the caller's (0: the default), halved (not below 256)
    // until the workspace fits the array; it moves only the FP64 chunk
    // boundaries of the source sums, not the FP32 tiles.
    gs_params pr = *prm;
    pr.flags &= ~GS_FLAG_F64;
    int64_t items = pr.exact_items > 0 ? pr.exact_items : gs::kItemsDefault;
    for (;;) {
        pr.exact_items = (int32_t)items;
        const size_t need = gs_workspace_bytes(n, &pr, GS_EXACT, GS_OP_RHS);
        if (need == 0) return gs_rhs_exact(q, p, n, prm, dq, dp, nullptr, 0, stream);
        if (need <= kScratchBytes) break;
        if (items <= 256) {
            gs::set_error("gs_rhs_exact_static: workspace of %zu bytes exceeds the %zu-byte "
                          "static array", need, kScratchBytes);
            return GS_ERR_WORKSPACE;
        }
        items = items / 2 > 256 ? items / 2 : 256;
    }
    void *ws = nullptr;
    GS_TRY(gs::scratch_ptr(&ws));
    return gs_rhs_exact(q, p, n, &pr, dq, dp, ws, kScratchBytes, stream);
}
