// Batch evaluation that allocates nothing: the kernels of mg_eval_marginal_batch
// (trace, window selection and path masks, level by level) with their launch
// descriptors and per-level work lists kept in one fixed device array.
//
// `scratch` is a file-scope device array of kScratchBytes; every device the
// library runs on holds its own copy until the process ends. Host code never
// passes the array's name to a kernel or a copy (on the host it is a stand-in,
// not a device address): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that pointer is used
// everywhere. The descriptors and lists are written into it from a fixed host
// staging array on the caller's stream, so a call is ordered after earlier
// work on that stream; calls that overlap on one device (different streams,
// or threads) share the array and race.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "mg_batch.h"

using namespace mgk;

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // descriptors | items | items with children
constexpr int32_t kMaxTrees = 4096;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

// Host side: staging of the scratch's contents, the sorted tree list used to
// refuse duplicates, per-level offsets, and per device the scratch's address
// and an event marking the end of the last copy out of the staging array.
alignas(256) uint8_t g_stage[kScratchBytes];
mg_tree g_sorted[kMaxTrees];
int64_t g_level_item[kMaxAnc + 2], g_level_mitem[kMaxAnc + 2];
uint8_t* g_scratch_ptr[kMaxDevices] = {};
hipEvent_t g_copied[kMaxDevices] = {};
std::mutex g_mu;

int hip_fail(hipError_t e, const char* what) {
    char msg[256];
    snprintf(msg, sizeof(msg), "%s: %s", what, hipGetErrorString(e));
    return mgb::set_error(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, msg);
}

// Set-up on the first call on a device (the device is current): the device
// address of `scratch`, and the event of the copies.
int setup_device(int dev) {
    if (g_scratch_ptr[dev]) return MG_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch address");
    e = hipEventCreateWithFlags(&g_copied[dev], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "scratch copy event");
    g_scratch_ptr[dev] = (uint8_t*)p;
    return MG_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

bool same_geometry(const mg_sensor& a, const mg_sensor& b) {
    return a.n_az == b.n_az && a.n_el == b.n_el && a.yaw_bins == b.yaw_bins && a.fov_h_deg == b.fov_h_deg &&
           a.fov_v_deg == b.fov_v_deg && a.az_offset_deg == b.az_offset_deg;
}

}  // namespace

extern "C" int mg_eval_marginal_batch_noalloc(const mg_tree* trees, int32_t n_trees, void* hip_stream,
                                              uint32_t* gain, int32_t* yaw_bin, float* depth) {
    if (!trees || n_trees < 1 || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "bad batch arguments");
    if (n_trees > kMaxTrees)
        return mgb::set_error(MG_E_UNSUPPORTED, "more than 4096 trees in one allocation-free batch");
    for (int32_t i = 0; i < n_trees; ++i)
        if (!trees[i]) return mgb::set_error(MG_E_INVALID, "NULL tree in batch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return mgb::set_error(MG_E_UNSUPPORTED, "device index above 63");
    hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = setup_device(dev);
    if (rc != MG_OK) return rc;
    // a tree listed twice would have two descriptors writing its bins and buffers
    std::copy(trees, trees + n_trees, g_sorted);
    std::sort(g_sorted, g_sorted + n_trees);
    if (std::adjacent_find(g_sorted, g_sorted + n_trees) != g_sorted + n_trees)
        return mgb::set_error(MG_E_INVALID, "a tree appears twice in the batch");
    // sizes: descriptors, then every level's items, then every level's items with children
    mgb::TreeView v0;
    mgb::tree_view(trees[0], &v0);
    int32_t levels = 0;
    uint64_t total = 0, total_m = 0;
    uint32_t max_nodes = 0, mask_bricks = 0;
    for (int32_t i = 0; i < n_trees; ++i) {
        mgb::TreeView v;
        mgb::tree_view(trees[i], &v);
        if (!same_geometry(v.params, v0.params))
            return mgb::set_error(MG_E_INVALID, "trees in a batch must share the sensor geometry");
        if (v.device != dev) return mgb::set_error(MG_E_INVALID, "batch trees live on another device");
        levels = std::max(levels, v.levels);
        total += (uint64_t)v.n;
        total_m += (uint64_t)v.mask_nodes->size();
        max_nodes = std::max(max_nodes, (uint32_t)v.n);
        mask_bricks = std::max(mask_bricks, v.map->build_slots);
    }
    if (total >= (1ull << 31)) return mgb::set_error(MG_E_UNSUPPORTED, "batch has 2^31 nodes or more");
    const size_t o_items = align256(sizeof(BatchTree) * (size_t)n_trees);
    const size_t o_mitems = o_items + align256(sizeof(unsigned long long) * total);
    const size_t bytes = o_mitems + sizeof(unsigned long long) * total_m;
    if (bytes > kScratchBytes)
        return mgb::set_error(MG_E_UNSUPPORTED,
                              "the batch needs more than the 16 MiB of scratch of the allocation-free entry point "
                              "(descriptors and work lists: 8 bytes per node and per node with children)");
    // the staging array may still be the source of the previous call's copies
    e = hipEventSynchronize(g_copied[dev]);
    if (e != hipSuccess) return hip_fail(e, "previous scratch copy");
    BatchTree* bt = reinterpret_cast<BatchTree*>(g_stage);
    unsigned long long* items = reinterpret_cast<unsigned long long*>(g_stage + o_items);
    unsigned long long* mitems = reinterpret_cast<unsigned long long*>(g_stage + o_mitems);
    uint32_t off = 0;
    for (int32_t i = 0; i < n_trees; ++i) {
        mgb::TreeView v;
        mgb::tree_view(trees[i], &v);
        std::memset(&bt[i], 0, sizeof(BatchTree));
        bt[i].map = *v.map;
        bt[i].td = *v.td;
        bt[i].rv = v.sd->rv;
        bt[i].rv2 = v.sd->rv2;
        bt[i].vox3 = (double)v.voxel_m * (double)v.voxel_m * (double)v.voxel_m;
        bt[i].out_off = off;
        bt[i].gain = gain + off;
        bt[i].yaw = yaw_bin + off;
        bt[i].depth = depth ? depth + (size_t)off * v.sd->H * v.sd->WB : nullptr;
        off += (uint32_t)v.n;
    }
    int64_t k = 0, km = 0;
    for (int32_t d = 0; d < levels; ++d) {
        g_level_item[d] = k;
        g_level_mitem[d] = km;
        for (int32_t i = 0; i < n_trees; ++i) {
            mgb::TreeView v;
            mgb::tree_view(trees[i], &v);
            if (d >= v.levels) continue;
            const std::vector<int32_t>& lp = *v.level_ptr;
            const std::vector<int32_t>& ln = *v.level_nodes;
            const std::vector<int32_t>& mp = *v.mask_level_ptr;
            const std::vector<int32_t>& mn = *v.mask_nodes;
            for (int32_t j = lp[d]; j < lp[d + 1]; ++j) items[k++] = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)ln[j];
            for (int32_t j = mp[d]; j < mp[d + 1]; ++j) mitems[km++] = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)mn[j];
        }
    }
    g_level_item[levels] = k;
    g_level_mitem[levels] = km;
    uint8_t* base = g_scratch_ptr[dev];
    e = hipMemcpyAsync(base, g_stage, o_items + sizeof(unsigned long long) * total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && total_m > 0)
        e = hipMemcpyAsync(base + o_mitems, g_stage + o_mitems, sizeof(unsigned long long) * total_m,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(g_copied[dev], s);
    if (e != hipSuccess) return hip_fail(e, "scratch upload");
    const BatchTree* dtrees = reinterpret_cast<const BatchTree*>(base);
    const unsigned long long* ditems = reinterpret_cast<const unsigned long long*>(base + o_items);
    const unsigned long long* dmitems = reinterpret_cast<const unsigned long long*>(base + o_mitems);
    e = launch_batch_zero(dtrees, n_trees, max_nodes, *v0.sd, s);
    for (int32_t d = 0; d < levels && e == hipSuccess; ++d)
        e = launch_batch_level(dtrees, ditems + g_level_item[d], (int32_t)(g_level_item[d + 1] - g_level_item[d]),
                               dmitems + g_level_mitem[d], (int32_t)(g_level_mitem[d + 1] - g_level_mitem[d]),
                               mask_bricks, *v0.sd, s, 0);
    if (e != hipSuccess) return hip_fail(e, "batch level");
    return MG_OK;
}
