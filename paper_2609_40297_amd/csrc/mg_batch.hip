// Multi-tree evaluation: trees advance one depth level at a time; each level
// is one trace launch over every (tree, node) of that depth followed by one
// window-selection launch. A node needs only its own ancestors, so the plan
// splits the work into up to kGroups independent groups (whole trees, or the
// subtrees below a shared prefix of levels when there are few trees), each
// advancing level by level on its own stream: one group's small levels run
// while another's are still in flight, instead of all waiting for the slowest
// node of a global level. Launch plans are cached per tree list; a new
// plan gets its trace launch shape from the autotuner (every compiled shape
// timed on the plan itself, the result kept per workload shape) and, when
// configured, its launches are captured once into a HIP graph that later
// calls replay. Configured persistent, a plan is instead one cooperative
// launch of co-resident workgroups that walks every level of every tree with
// grid barriers between the phases (the same kernels' device code).
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mg_batch.h"

using namespace mgk;

namespace {

struct Plan {
    std::vector<mg_tree> trees;
    uint32_t* gain = nullptr;             // output buffers the descriptors point into
    int32_t* yaw = nullptr;
    float* depth = nullptr;
    void* block = nullptr;                 // BatchTree[n_trees] | items[total] | mitems (nodes with children)
    const BatchTree* dtrees = nullptr;
    const unsigned long long* ditems = nullptr;
    const unsigned long long* dmitems = nullptr;
    uint32_t mask_bricks = 0;              // build slots of the largest map among the trees
    // Launch records in host order: stream 0 is the caller's (the shared
    // prefix of levels), stream g + 1 runs group g. [mbegin, mbegin + mcount)
    // are the launch's nodes with children (their path masks are built).
    struct Launch {
        int32_t stream, begin, count, mbegin, mcount, depth;
    };
    std::vector<Launch> launches;
    int32_t groups = 0;
    int32_t levels = 0;                    // deepest level + 1 over the trees
    SensorDev sd{};
    uint32_t total = 0, max_nodes = 0;
    int device = 0;
    int shape = 0;                         // launch shape of the trace kernel
    hipGraph_t graph = nullptr;            // the plan's launches, captured once
    hipGraphExec_t exec = nullptr;
    // The persistent form: items and nodes with children of all trees by
    // level (level_ptr / mlevel_ptr: levels + 1 offsets each), the barrier
    // words, and a pinned word the barrier's give-up flag is read into.
    bool persistent = false;
    const unsigned long long* pitems = nullptr;
    const unsigned long long* pmitems = nullptr;
    const int32_t* plevel = nullptr;
    const int32_t* pmlevel = nullptr;
    uint32_t* psync = nullptr;
    uint32_t* h_abort = nullptr;
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (block) (void)hipFree(block);
        if (h_abort) (void)hipHostFree(h_abort);
    }
};

// Configuration for plans built from now on (mg_batch_config).
int g_cfg_shape = -1;                      // -1: autotune
bool g_cfg_graph = false;                  // replaying a graph measured slower than direct launches
bool g_cfg_persistent = false;             // one persistent cooperative launch per call
uint32_t g_barrier_polls = 1u << 25;       // polls of a grid-barrier wait before it gives up (seconds)
// Autotuned shapes per workload shape (sensor, range, map dims, sizes).
std::map<std::vector<int64_t>, int> g_tuned;

// Per-device stream that replays plan graphs, joined to the caller's stream
// with events on both sides.
struct Replay {
    hipStream_t stream = nullptr;
    hipEvent_t in = nullptr, out = nullptr;
};
std::map<int, Replay> g_replay;

std::mutex g_mu;
std::map<std::vector<mg_tree>, std::unique_ptr<Plan>> g_plans;
constexpr size_t kMaxPlans = 64;
constexpr int32_t kGroups = 3;             // independent groups of a plan, one stream each (3 measured best of 1/2/3/4/8)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int hip_fail(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return mgb::set_error(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, m.c_str());
}

bool same_geometry(const mg_sensor& a, const mg_sensor& b) {
    return a.n_az == b.n_az && a.n_el == b.n_el && a.yaw_bins == b.yaw_bins && a.fov_h_deg == b.fov_h_deg &&
           a.fov_v_deg == b.fov_v_deg && a.az_offset_deg == b.az_offset_deg;
}

int build_plan(const std::vector<mg_tree>& trees, uint32_t* gain, int32_t* yaw, float* depth, hipStream_t stream,
               std::unique_ptr<Plan>* out) {
    std::unique_ptr<Plan> P(new Plan());
    P->trees = trees;
    const int32_t nt = (int32_t)trees.size();
    std::vector<BatchTree> bt(nt);
    mgb::TreeView v0;
    mgb::tree_view(trees[0], &v0);
    int32_t levels = 0;
    std::vector<mgb::TreeView> views(nt);
    for (int32_t i = 0; i < nt; ++i) {
        mgb::TreeView& v = views[i];
        mgb::tree_view(trees[i], &v);
        if (!same_geometry(v.params, v0.params))
            return mgb::set_error(MG_E_INVALID, "trees in a batch must share the sensor geometry");
        if (v.device != v0.device) return mgb::set_error(MG_E_INVALID, "trees in a batch must share a device");
        bt[i].map = *v.map;
        bt[i].td = *v.td;
        bt[i].rv = v.sd->rv;
        bt[i].rv2 = v.sd->rv2;
        bt[i].vox3 = (double)v.voxel_m * (double)v.voxel_m * (double)v.voxel_m;
        bt[i].out_off = P->total;
        bt[i].gain = gain + P->total;
        bt[i].yaw = yaw + P->total;
        bt[i].depth = depth ? depth + (size_t)P->total * v.sd->H * v.sd->WB : nullptr;
        if ((uint64_t)P->total + (uint64_t)v.n >= (1ull << 31))
            return mgb::set_error(MG_E_UNSUPPORTED, "batch has 2^31 nodes or more");
        P->total += (uint32_t)v.n;
        P->max_nodes = std::max(P->max_nodes, (uint32_t)v.n);
        P->mask_bricks = std::max(P->mask_bricks, v.map->build_slots);
        levels = std::max(levels, v.levels);
    }
    P->sd = *v0.sd;
    P->device = v0.device;
    int32_t max_tiles = 0;                 // workgroups per node of the narrowest launch shape
    for (int k = 0; k < shape_count(); ++k) max_tiles = std::max(max_tiles, tiles_per_node(P->sd, k));
    // Split: with at least kGroups trees the units of work are whole trees;
    // otherwise the levels above depth s (the first depth holding at least
    // kGroups nodes) form a shared prefix and the units are the subtrees
    // rooted at depth s.
    int32_t split = 0;
    if (nt < kGroups) {
        split = levels;
        for (int32_t d = 1; d < levels; ++d) {
            int64_t cnt = 0;
            for (int32_t i = 0; i < nt; ++i) {
                const std::vector<int32_t>& lp = *views[i].level_ptr;
                if (d + 1 < (int32_t)lp.size()) cnt += lp[d + 1] - lp[d];
            }
            if (cnt >= kGroups) {
                split = d;
                break;
            }
        }
    }
    // unit of every node at depth >= split: (tree, ancestor at depth split)
    std::vector<std::vector<int32_t>> unit_of(nt);
    std::vector<int64_t> unit_size;
    for (int32_t i = 0; i < nt; ++i) {
        const std::vector<int32_t>& par = *views[i].parent;
        const std::vector<int32_t>& dep = *views[i].depth;
        const int32_t n = views[i].n;
        unit_of[i].assign(n, -1);
        if (nt >= kGroups) {
            for (int32_t k = 0; k < n; ++k) unit_of[i][k] = i;
            unit_size.push_back(n);
            continue;
        }
        for (int32_t k = 0; k < n; ++k) {            // parents precede children
            if (dep[k] < split) continue;
            if (dep[k] == split) {
                unit_of[i][k] = (int32_t)unit_size.size();
                unit_size.push_back(0);
            } else {
                unit_of[i][k] = unit_of[i][par[k]];
            }
            ++unit_size[unit_of[i][k]];
        }
    }
    // units to groups, largest first onto the least loaded group
    const int32_t G = (int32_t)std::min<size_t>(kGroups, unit_size.size());
    std::vector<int32_t> group_of_unit(unit_size.size(), 0);
    {
        std::vector<int32_t> order(unit_size.size());
        for (size_t u = 0; u < order.size(); ++u) order[u] = (int32_t)u;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return unit_size[a] > unit_size[b]; });
        std::vector<int64_t> load(G, 0);
        for (int32_t u : order) {
            const int32_t g = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
            group_of_unit[u] = g;
            load[g] += unit_size[u];
        }
    }
    P->groups = G;
    // items: the prefix level by level (trees in order), then every group's
    // levels; one launch record per non-empty (stream, level); mitems: the
    // same launches' nodes with children
    std::vector<unsigned long long> items, mitems;
    items.reserve(P->total);
    auto add_launch = [&](int32_t stream, int32_t begin, int32_t mbegin, int32_t d) -> int {
        const int32_t count = (int32_t)items.size() - begin;
        if (count == 0) return MG_OK;
        if ((uint64_t)count * (uint64_t)max_tiles >= (1ull << 31))
            return mgb::set_error(MG_E_UNSUPPORTED, "a depth level of the batch has 2^31 workgroups or more");
        P->launches.push_back({stream, begin, count, mbegin, (int32_t)mitems.size() - mbegin, d});
        return MG_OK;
    };
    auto add_level = [&](int32_t d, int32_t g) {    // g < 0: every node of the level
        for (int32_t i = 0; i < nt; ++i) {
            const std::vector<int32_t>& lp = *views[i].level_ptr;
            const std::vector<int32_t>& ln = *views[i].level_nodes;
            const std::vector<int32_t>& mp = *views[i].mask_level_ptr;
            const std::vector<int32_t>& mn = *views[i].mask_nodes;
            if (d + 1 >= (int32_t)lp.size()) continue;
            for (int32_t k = lp[d]; k < lp[d + 1]; ++k)
                if (g < 0 || group_of_unit[unit_of[i][ln[k]]] == g)
                    items.push_back(((unsigned long long)(uint32_t)i << 32) | (uint32_t)ln[k]);
            for (int32_t k = mp[d]; k < mp[d + 1]; ++k)
                if (g < 0 || group_of_unit[unit_of[i][mn[k]]] == g)
                    mitems.push_back(((unsigned long long)(uint32_t)i << 32) | (uint32_t)mn[k]);
        }
    };
    for (int32_t d = 0; d < split; ++d) {
        const int32_t begin = (int32_t)items.size(), mbegin = (int32_t)mitems.size();
        add_level(d, -1);
        int rc = add_launch(0, begin, mbegin, d);
        if (rc != MG_OK) return rc;
    }
    for (int32_t d = split; d < levels; ++d) {
        for (int32_t g = 0; g < G; ++g) {
            const int32_t begin = (int32_t)items.size(), mbegin = (int32_t)mitems.size();
            add_level(d, g);
            int rc = add_launch(g + 1, begin, mbegin, d);
            if (rc != MG_OK) return rc;
        }
    }
    P->levels = levels;
    // the persistent form's lists: every tree's level d, for d = 0, 1, ...
    std::vector<unsigned long long> pitems, pmitems;
    std::vector<int32_t> plevel(1, 0), pmlevel(1, 0);
    pitems.reserve(P->total);
    for (int32_t d = 0; d < levels; ++d) {
        for (int32_t i = 0; i < nt; ++i) {
            const std::vector<int32_t>& lp = *views[i].level_ptr;
            const std::vector<int32_t>& ln = *views[i].level_nodes;
            const std::vector<int32_t>& mp = *views[i].mask_level_ptr;
            const std::vector<int32_t>& mn = *views[i].mask_nodes;
            if (d + 1 >= (int32_t)lp.size()) continue;
            for (int32_t k = lp[d]; k < lp[d + 1]; ++k) pitems.push_back(((unsigned long long)(uint32_t)i << 32) | (uint32_t)ln[k]);
            for (int32_t k = mp[d]; k < mp[d + 1]; ++k) pmitems.push_back(((unsigned long long)(uint32_t)i << 32) | (uint32_t)mn[k]);
        }
        if ((uint64_t)(pitems.size() - plevel.back()) * (uint64_t)max_tiles >= (1ull << 31))
            return mgb::set_error(MG_E_UNSUPPORTED, "a depth level of the batch has 2^31 workgroups or more");
        plevel.push_back((int32_t)pitems.size());
        pmlevel.push_back((int32_t)pmitems.size());
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_trees = take(sizeof(BatchTree) * nt);
    const size_t o_items = take(sizeof(unsigned long long) * items.size());
    const size_t o_mitems = take(sizeof(unsigned long long) * std::max<size_t>(mitems.size(), 1));
    const size_t o_pitems = take(sizeof(unsigned long long) * pitems.size());
    const size_t o_pmitems = take(sizeof(unsigned long long) * std::max<size_t>(pmitems.size(), 1));
    const size_t o_plevel = take(sizeof(int32_t) * plevel.size());
    const size_t o_pmlevel = take(sizeof(int32_t) * pmlevel.size());
    const size_t o_psync = take(sizeof(uint32_t) * 2);
    hipError_t e = hipMalloc(&P->block, off);
    if (e != hipSuccess) return hip_fail(e, "batch plan allocation");
    char* base = (char*)P->block;
    e = hipMemcpyAsync(base + o_trees, bt.data(), sizeof(BatchTree) * nt, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_items, items.data(), sizeof(unsigned long long) * items.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !mitems.empty())
        e = hipMemcpyAsync(base + o_mitems, mitems.data(), sizeof(unsigned long long) * mitems.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_pitems, pitems.data(), sizeof(unsigned long long) * pitems.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !pmitems.empty())
        e = hipMemcpyAsync(base + o_pmitems, pmitems.data(), sizeof(unsigned long long) * pmitems.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_plevel, plevel.data(), sizeof(int32_t) * plevel.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_pmlevel, pmlevel.data(), sizeof(int32_t) * pmlevel.size(), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "batch plan upload");
    P->dtrees = (const BatchTree*)(base + o_trees);
    P->gain = gain;
    P->yaw = yaw;
    P->depth = depth;
    P->ditems = (const unsigned long long*)(base + o_items);
    P->dmitems = (const unsigned long long*)(base + o_mitems);
    P->pitems = (const unsigned long long*)(base + o_pitems);
    P->pmitems = (const unsigned long long*)(base + o_pmitems);
    P->plevel = (const int32_t*)(base + o_plevel);
    P->pmlevel = (const int32_t*)(base + o_pmlevel);
    P->psync = (uint32_t*)(base + o_psync);
    *out = std::move(P);
    return MG_OK;
}

// Optional per-launch timing of the trace kernel: each timed launch carries a
// start/stop event pair that its own dispatch records.
struct Timing {
    std::mutex mu;
    bool on = false;
    int device = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    int64_t units = 0;                     // workgroups (node tiles) launched while timed
};
Timing g_timing;
constexpr size_t kMaxTimedLaunches = 1u << 16;

// Next event pair for a timed launch on `device`, or {null, null} when timing is off.
int next_events(int device, hipEvent_t* t0, hipEvent_t* t1) {
    *t0 = *t1 = nullptr;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.on) return MG_OK;
    if (g_timing.device != device)
        return mgb::set_error(MG_E_INVALID, "kernel timing was enabled on another device");
    if (g_timing.used == kMaxTimedLaunches)
        return mgb::set_error(MG_E_BUSY, "too many timed launches since the last mg_timing_read");
    if (g_timing.used == g_timing.ev.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            return hip_fail(e, "timing event");
        }
        g_timing.ev.emplace_back(a, b);
    }
    *t0 = g_timing.ev[g_timing.used].first;
    *t1 = g_timing.ev[g_timing.used].second;
    ++g_timing.used;
    return MG_OK;
}

bool timing_on() {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    return g_timing.on;
}

// Per-device streams of the groups, with the events that fork them from and
// join them back to the caller's stream (all default priority, non-blocking).
struct GroupStreams {
    hipStream_t stream[kGroups] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kGroups] = {};
};
std::map<int, GroupStreams> g_group_streams;

int group_streams(int device, GroupStreams** out) {
    GroupStreams& G = g_group_streams[device];
    if (!G.fork) {
        hipError_t e = hipEventCreateWithFlags(&G.fork, hipEventDisableTiming);
        for (int32_t g = 0; g < kGroups && e == hipSuccess; ++g) {
            e = hipStreamCreateWithFlags(&G.stream[g], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&G.join[g], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            for (int32_t g = 0; g < kGroups; ++g) {
                if (G.stream[g]) (void)hipStreamDestroy(G.stream[g]);
                if (G.join[g]) (void)hipEventDestroy(G.join[g]);
            }
            if (G.fork) (void)hipEventDestroy(G.fork);
            G = GroupStreams();
            return hip_fail(e, "group streams");
        }
    }
    *out = &G;
    return MG_OK;
}

// Enqueues the plan's launches: the shared prefix on s, then each group on its
// own stream, forked from s and joined back to it. `timed` lets the kernel
// timer attach events.
int run_plan(const Plan& P, hipStream_t s, bool timed) {
    hipError_t e = launch_batch_zero(P.dtrees, (int32_t)P.trees.size(), P.max_nodes, P.sd, s);
    if (e != hipSuccess) return hip_fail(e, "batch zero");
    GroupStreams* GS = nullptr;
    if (P.groups > 0) {
        int rc = group_streams(P.device, &GS);
        if (rc != MG_OK) return rc;
    }
    bool forked = false;
    for (const Plan::Launch& L : P.launches) {
        if (L.stream > 0 && !forked) {
            e = hipEventRecord(GS->fork, s);
            for (int32_t g = 0; g < P.groups && e == hipSuccess; ++g) e = hipStreamWaitEvent(GS->stream[g], GS->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "group fork");
            forked = true;
        }
        hipEvent_t t0 = nullptr, t1 = nullptr, b0 = nullptr, b1 = nullptr;
        if (timed) {
            int rc = next_events(P.device, &t0, &t1);
            if (rc == MG_OK && L.mcount > 0) rc = next_events(P.device, &b0, &b1);
            if (rc != MG_OK) return rc;
        }
        hipStream_t ls = L.stream == 0 ? s : GS->stream[L.stream - 1];
        e = launch_batch_level(P.dtrees, P.ditems + L.begin, L.count, P.dmitems + L.mbegin, L.mcount, P.mask_bricks,
                               P.sd, ls, P.shape, t0, t1, b0, b1);
        if (e != hipSuccess) return hip_fail(e, "batch level");
        if (t0) {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            g_timing.units += (int64_t)L.count * tiles_per_node(P.sd, P.shape);
        }
    }
    if (forked) {
        for (int32_t g = 0; g < P.groups && e == hipSuccess; ++g) {
            e = hipEventRecord(GS->join[g], GS->stream[g]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, GS->join[g], 0);
        }
        if (e != hipSuccess) return hip_fail(e, "group join");
    }
    return MG_OK;
}

// The persistent form: bins cleared, one cooperative launch, then the barrier's
// give-up flag read back. Blocks on s (the flag decides the return code).
int run_persistent(const Plan& P, hipStream_t s, bool timed) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timed) {
        int rc = next_events(P.device, &t0, &t1);
        if (rc != MG_OK) return rc;
    }
    hipError_t e = launch_batch_zero(P.dtrees, (int32_t)P.trees.size(), P.max_nodes, P.sd, s);
    if (e == hipSuccess && t0) e = hipEventRecord(t0, s);
    if (e == hipSuccess)
        e = launch_batch_persistent(P.dtrees, P.pitems, P.plevel, P.pmitems, P.pmlevel, P.levels, P.mask_bricks, P.sd,
                                    P.psync, g_barrier_polls, s);
    if (e == hipSuccess && t1) e = hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.h_abort, P.psync + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "persistent batch");
    if (t0) {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.units += (int64_t)P.total * tiles_per_node(P.sd, 0);
    }
    if (*P.h_abort != 0)
        return mgb::set_error(MG_E_DEVICE, "persistent batch: a grid barrier wait gave up (its poll limit ran out)");
    return MG_OK;
}

std::vector<int64_t> tune_key(const Plan& P) {
    mgb::TreeView v;
    mgb::tree_view(P.trees[0], &v);
    auto bits = [](float f) { int32_t i; memcpy(&i, &f, 4); return (int64_t)i; };
    int64_t lg = 0;
    while ((1ull << (lg + 1)) <= P.total) ++lg;
    return {v.params.n_az, v.params.n_el, v.params.yaw_bins, bits(v.params.fov_h_deg), bits(v.params.fov_v_deg),
            bits(P.sd.rv), v.map->nx, v.map->ny, v.map->nz, (int64_t)P.trees.size(),
            (int64_t)P.levels, lg, P.device};
}

// Times every launch shape on the plan itself (second of two runs each) and
// keeps the fastest. Blocks on s.
int autotune(Plan& P, hipStream_t s) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int best = 0;
    float best_ms = 0.f;
    bool any = false;
    for (int k = 0; k < shape_count() && e == hipSuccess; ++k) {
        P.shape = k;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = hipEventRecord(a, s);
            if (e != hipSuccess) break;
            int rc = run_plan(P, s, false);
            if (rc != MG_OK) {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                return rc;
            }
            e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        }
        if (e == hipSuccess && (!any || ms < best_ms)) {
            best = k;
            best_ms = ms;
            any = true;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    P.shape = best;
    return MG_OK;
}

// Records the plan's launches into a graph on a private stream.
int capture(Plan& P) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = MG_OK;
    if (e == hipSuccess) {
        rc = run_plan(P, cs, false);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (rc == MG_OK && e2 == hipSuccess) {
            P.graph = g;
            e = hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0);
        } else {
            if (g) (void)hipGraphDestroy(g);
            if (rc == MG_OK) e = e2;
        }
    }
    (void)hipStreamDestroy(cs);
    if (rc != MG_OK) return rc;
    if (e != hipSuccess) {
        P.exec = nullptr;
        return hip_fail(e, "graph capture");
    }
    return MG_OK;
}

// Replays the plan's graph ordered after the work already on s, and makes
// later work on s wait for it.
int replay(const Plan& P, hipStream_t s) {
    Replay& R = g_replay[P.device];
    hipError_t e = hipSuccess;
    if (!R.stream) {
        e = hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&R.in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&R.out, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "replay stream");
    }
    e = hipEventRecord(R.in, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(R.stream, R.in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(P.exec, R.stream);
    if (e == hipSuccess) e = hipEventRecord(R.out, R.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, R.out, 0);
    if (e != hipSuccess) return hip_fail(e, "graph replay");
    return MG_OK;
}

// Launch shape (configured, cached or tuned now) and graph of a new plan.
int configure(Plan& P, hipStream_t s) {
    if (g_cfg_persistent) {
        int32_t grid = 0;
        hipError_t e = persistent_grid(P.sd, &grid);
        if (e == hipErrorNotSupported) return mgb::set_error(MG_E_UNSUPPORTED, "the device has no cooperative launch");
        if (e == hipSuccess) e = hipHostMalloc(&P.h_abort, sizeof(uint32_t), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "persistent batch set-up");
        P.persistent = true;
        P.shape = 0;
        return MG_OK;
    }
    if (g_cfg_shape >= 0) {
        P.shape = g_cfg_shape;
    } else {
        const std::vector<int64_t> key = tune_key(P);
        auto t = g_tuned.find(key);
        if (t != g_tuned.end()) {
            P.shape = t->second;
        } else {
            int rc = autotune(P, s);
            if (rc != MG_OK) return rc;
            g_tuned[key] = P.shape;
        }
    }
    if (g_cfg_graph) return capture(P);
    return MG_OK;
}

}  // namespace

namespace mgb {
void forget_tree(mg_tree t) {
    std::lock_guard<std::mutex> lk(g_mu);
    bool any = false;
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find(it->first.begin(), it->first.end(), t) != it->first.end()) {
            if (!any) (void)hipDeviceSynchronize();      // launches of the plan may still be queued
            any = true;
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}
}  // namespace mgb

extern "C" int mg_eval_marginal_batch(const mg_tree* trees, int32_t n_trees, void* hip_stream, uint32_t* gain,
                                      int32_t* yaw_bin, float* depth) {
    if (!trees || n_trees < 1 || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "bad batch arguments");
    if (n_trees > 65535) return mgb::set_error(MG_E_UNSUPPORTED, "more than 65535 trees in one batch");
    for (int32_t i = 0; i < n_trees; ++i)
        if (!trees[i]) return mgb::set_error(MG_E_INVALID, "NULL tree in batch");
    {
        // a tree listed twice would have two descriptors writing its bins and buffers
        std::vector<mg_tree> sorted(trees, trees + n_trees);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return mgb::set_error(MG_E_INVALID, "a tree appears twice in the batch");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::vector<mg_tree> key(trees, trees + n_trees);
    hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end() && (it->second->gain != gain || it->second->yaw != yaw_bin || it->second->depth != depth)) {
        (void)hipStreamSynchronize(s);          // the old descriptors may still be read
        g_plans.erase(it);
        it = g_plans.end();
    }
    if (it == g_plans.end()) {
        if (g_plans.size() >= kMaxPlans) {
            (void)hipDeviceSynchronize();
            g_plans.clear();
        }
        std::unique_ptr<Plan> P;
        int rc = build_plan(key, gain, yaw_bin, depth, s, &P);
        if (rc != MG_OK) return rc;
        if (P->device != dev) return mgb::set_error(MG_E_INVALID, "batch trees live on another device");
        rc = configure(*P, s);
        if (rc != MG_OK) return rc;
        it = g_plans.emplace(key, std::move(P)).first;
    }
    const Plan& P = *it->second;
    if (P.device != dev) return mgb::set_error(MG_E_INVALID, "batch trees live on another device");
    if (P.persistent) return run_persistent(P, s, timing_on());
    // the kernel timer needs the launches made one by one
    if (!P.exec || timing_on()) return run_plan(P, s, true);
    return replay(P, s);
}

extern "C" int mg_score_branches(const mg_tree* trees, int32_t n_trees, void* hip_stream, const uint32_t* gain,
                                 double lambda, double* cost, double* objective, int32_t* best, int32_t* branch) {
    if (!trees || n_trees < 1 || !gain || !objective || !best)
        return mgb::set_error(MG_E_INVALID, "bad scoring arguments");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return mgb::set_error(MG_E_INVALID, "lambda must be >= 0");
    std::vector<mg_tree> key(trees, trees + n_trees);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it == g_plans.end())
        return mgb::set_error(MG_E_INVALID, "no plan for this tree list (evaluate it with mg_eval_marginal_batch first)");
    const Plan& P = *it->second;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (P.device != dev) return mgb::set_error(MG_E_INVALID, "batch trees live on another device");
    e = launch_score(P.dtrees, n_trees, P.max_nodes, gain, lambda, cost, objective, best, branch,
                     (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "path score");
    return MG_OK;
}

extern "C" int mg_batch_config(int32_t shape, int32_t launch) {
    if (shape < -1 || shape >= shape_count() || launch < 0 || launch > 2)
        return mgb::set_error(MG_E_INVALID, "shape must be -1 or a shape index, launch 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_plans.empty()) {
        (void)hipDeviceSynchronize();          // launches of cached plans may still be queued
        g_plans.clear();
    }
    g_cfg_shape = shape;
    g_cfg_graph = launch == 1;
    g_cfg_persistent = launch == 2;
    return MG_OK;
}

extern "C" int mg_batch_barrier_polls(int64_t polls) {
    if (polls < 0 || polls > (int64_t)INT32_MAX) return mgb::set_error(MG_E_INVALID, "polls must be in [0, 2^31)");
    std::lock_guard<std::mutex> lk(g_mu);
    g_barrier_polls = (uint32_t)polls;
    return MG_OK;
}

extern "C" int mg_trace_shapes(int32_t* count, int32_t* threads, int32_t* bricks, int32_t capacity) {
    if (!count || capacity < 0 || (capacity > 0 && (!threads || !bricks)))
        return mgb::set_error(MG_E_INVALID, "bad shape query");
    *count = shape_count();
    for (int k = 0; k < shape_count() && k < capacity; ++k) {
        int th = 0, b = 0;
        shape_of(k, &th, &b);
        threads[k] = th;
        bricks[k] = b;
    }
    return MG_OK;
}

extern "C" int mg_batch_plan_info(const mg_tree* trees, int32_t n_trees, int32_t* shape, int32_t* graphed) {
    if (!trees || n_trees < 1) return mgb::set_error(MG_E_INVALID, "bad batch arguments");
    std::vector<mg_tree> key(trees, trees + n_trees);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) return mgb::set_error(MG_E_INVALID, "no plan for this tree list (evaluate it first)");
    if (shape) *shape = it->second->shape;
    if (graphed) *graphed = it->second->persistent ? 2 : (it->second->exec ? 1 : 0);
    return MG_OK;
}

extern "C" int mg_timing_enable(int32_t on) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (on && g_timing.device != dev) {
        if (g_timing.used != 0) return mgb::set_error(MG_E_BUSY, "timed launches on another device are unread");
        for (auto& p : g_timing.ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        g_timing.ev.clear();
        g_timing.device = dev;
    }
    g_timing.on = on != 0;
    return MG_OK;
}

extern "C" int mg_timing_read(double* total_ms, double* busy_ms, int64_t* launches, int64_t* workgroups) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double sum = 0.0;
    std::vector<std::pair<double, double>> iv;     // launch intervals relative to the first start
    for (size_t i = 0; i < g_timing.used; ++i) {
        hipError_t e = hipEventSynchronize(g_timing.ev[i].second);
        float ms = 0.f, a = 0.f, b = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_timing.ev[i].first, g_timing.ev[i].second);
        if (e == hipSuccess) e = hipEventElapsedTime(&a, g_timing.ev[0].first, g_timing.ev[i].first);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, g_timing.ev[0].first, g_timing.ev[i].second);
        if (e != hipSuccess) {
            g_timing.used = 0;
            g_timing.units = 0;
            return hip_fail(e, "timing readout");
        }
        sum += ms;
        iv.emplace_back(a, b);
    }
    // union of the intervals: time during which at least one timed launch ran
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, lo = 0.0, hi = 0.0;
    for (size_t i = 0; i < iv.size(); ++i) {
        if (i == 0 || iv[i].first > hi) {
            busy += hi - lo;
            lo = iv[i].first;
            hi = iv[i].second;
        } else {
            hi = std::max(hi, iv[i].second);
        }
    }
    busy += hi - lo;
    if (total_ms) *total_ms = sum;
    if (busy_ms) *busy_ms = busy;
    if (launches) *launches = (int64_t)g_timing.used;
    if (workgroups) *workgroups = g_timing.units;
    g_timing.used = 0;
    g_timing.units = 0;
    return MG_OK;
}
