// tree.hip -- Barnes-Hut octree (placeholder until the tree path lands).
#include "tree.h"

namespace gs {

void carve_tree(Arena &a, int64_t n, TreeBufs &t) { t.unused = a.take<char>(n); }

ShootBhBufs layout_shoot_bh(Arena &a, int64_t n, int nt) {
    (void)nt;
    ShootBhBufs b{};
    carve_tree(a, n, b.tree);
    return b;
}

gs_status rhs_bh(const float *, const float *, int64_t, const gs_params &, float *, float *,
                 TreeBufs &, char *, hipStream_t) {
    set_error("Barnes-Hut path not built yet");
    return GS_ERR_UNSUPPORTED;
}

gs_status shoot_bh(const float *, const float *, int64_t, const gs_params &, float *, float *,
                   double *, ShootBhBufs &, char *, hipStream_t) {
    set_error("Barnes-Hut path not built yet");
    return GS_ERR_UNSUPPORTED;
}

}  // namespace gs
