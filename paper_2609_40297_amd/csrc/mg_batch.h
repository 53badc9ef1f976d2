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
    const std::vector<int32_t>* mask_level_ptr;// host copy, [levels + 1]: nodes with children by level
    const std::vector<int32_t>* mask_nodes;    // host copy
    const std::vector<int32_t>* parent;        // host copy, [n]
    const std::vector<int32_t>* depth;         // host copy, [n]
    uint32_t* scratch_gain;                    // device outputs inside the tree's block
    int32_t* scratch_yaw;
    mg_sensor params;
    float voxel_m;                             // edge of the tree's map voxels (metres)
    int32_t n, levels, device;
};

int tree_view(mg_tree t, TreeView* v);     // mg_api.hip
const mgk::MapDev* map_dev(mg_map m);      // mg_api.hip
size_t map_voxel_count(mg_map m);          // mg_api.hip
void map_ref(mg_map m, int delta);         // mg_api.hip: holders that keep mg_map_destroy from freeing m
int set_error(int code, const char* msg);  // mg_api.hip

// Tree uploads into memory the caller provides (mg_api.hip), for the server's arena.
struct HostTree;
HostTree* new_host_tree();
void free_host_tree(HostTree* H);
int prepare(mg_map map, const float* pos_m, const int32_t* parent, int32_t n, const mg_sensor* sensor, HostTree* H);
size_t block_bytes(const HostTree& H);
int upload_into(mg_map map, const HostTree& H, const mg_sensor* sensor, hipStream_t s, void* block, mg_tree* out);
void forget_tree(mg_tree t);               // mg_batch.hip: drop cached launch plans that use t
void forget_interval(mg_tree t);           // mg_interval.hip: free t's interval-mode buffers
void forget_exact(mg_tree t);              // mg_exact.hip: free t's hash tables

}  // namespace mgb
