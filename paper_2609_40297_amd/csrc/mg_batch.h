// Internal interface between the C ABI and the multi-tree scheduler.
#pragma once
#include "../../include/mg.h"
#include "mg_internal.h"

#include <vector>

namespace mgb {

struct TreeView {
    const mgk::MapDev* map;
    const mgk::SensorDev* sd;
    const mgk::TreeDev* td;
    const std::vector<int32_t>* level_ptr;     // host copy, [levels + 1]
    const std::vector<int32_t>* level_nodes;   // host copy, [n]
    mg_sensor params;
    int32_t n, levels, device;
};

int tree_view(mg_tree t, TreeView* v);     // mg_api.hip
int set_error(int code, const char* msg);  // mg_api.hip
void forget_tree(mg_tree t);               // mg_batch.hip: drop cached launch plans that use t

}  // namespace mgb
