// Multi-tree evaluation.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <vector>

#include "mg_batch.h"

namespace mgb {
void forget_tree(mg_tree) {}
}  // namespace mgb

extern "C" int mg_eval_marginal_batch(const mg_tree* trees, int32_t n_trees, void* hip_stream, uint32_t* gain,
                                      int32_t* yaw_bin, float* depth) {
    if (!trees || n_trees < 1 || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "bad batch arguments");
    size_t off = 0, doff = 0;
    for (int32_t i = 0; i < n_trees; ++i) {
        mgb::TreeView v;
        if (!trees[i]) return mgb::set_error(MG_E_INVALID, "NULL tree in batch");
        mgb::tree_view(trees[i], &v);
        int rc = mg_eval_marginal(trees[i], hip_stream, gain + off, yaw_bin + off, depth ? depth + doff : nullptr);
        if (rc != MG_OK) return rc;
        off += v.n;
        doff += (size_t)v.n * v.sd->H * v.sd->WB;
    }
    return MG_OK;
}
