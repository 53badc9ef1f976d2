// Exact marginal gain with hash sets on the device (eq. 2 at given yaw
// windows; the comparison the paper runs with voxel hash maps on the CPU,
// Sec. IV-E and V-A).
//
// For node n at window k_n, I(n) is the set of unknown voxels its window's
// rays meet. With the windows fixed, every I(n) is known up front, so there is
// no level order: one launch builds every node's set (open addressing, linear
// probing, 32-bit voxel ids, compare-and-swap inserts), a second walks every
// window ray again and counts the unknown incidences whose voxel lies in none
// of the ancestors' sets (X_ray), a third counts each set's members outside
// the ancestors' sets (X_set); |I(n)| is A_set. A first walk counts each
// node's unknown incidences, which bounds |I(n)| and sizes its table (a power
// of two at least twice that), so the call synchronises once to size the pool.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "mg_batch.h"

using namespace mgk;

namespace mgx {

constexpr int kXThreads = 256;
constexpr uint32_t kEmpty = 0xffffffffu;     // never a voxel id (grids hold < 2^32 voxels)

struct Tables {
    uint32_t* slots;           // all nodes' tables
    const uint64_t* off;       // [n] first slot of node n's table
    const uint32_t* mask;      // [n] capacity - 1 (capacity a power of two)
};

__device__ __forceinline__ uint32_t mix(uint32_t x) {      // 32-bit finaliser (xorshift-multiply)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ bool contains(const Tables& T, int32_t node, uint32_t id) {
    const uint32_t* t = T.slots + T.off[node];
    const uint32_t m = T.mask[node];
    for (uint32_t h = mix(id) & m;; h = (h + 1) & m) {
        const uint32_t v = t[h];
        if (v == id) return true;
        if (v == kEmpty) return false;
    }
}

// Inserts id; true when it was not there yet.
__device__ __forceinline__ bool insert(const Tables& T, int32_t node, uint32_t id) {
    uint32_t* t = T.slots + T.off[node];
    const uint32_t m = T.mask[node];
    for (uint32_t h = mix(id) & m;; h = (h + 1) & m) {
        const uint32_t prev = atomicCAS(&t[h], kEmpty, id);
        if (prev == kEmpty) return true;
        if (prev == id) return false;
    }
}

// The DDA of the depth-buffer path (same operations and tie rules), calling
// f(id) for every unknown voxel visited before the ray stops.
template <class F>
__device__ void walk_unknown(const MapDev& M, float rv, float4 p, float4 d, float4 inv, F& f) {
    int32_t i[3] = {(int32_t)floorf(p.x), (int32_t)floorf(p.y), (int32_t)floorf(p.z)};
    const float q[3] = {p.x, p.y, p.z}, dd[3] = {d.x, d.y, d.z}, iv[3] = {inv.x, inv.y, inv.z};
    const int32_t n[3] = {M.nx, M.ny, M.nz};
    int32_t st[3], nb[3];
    float tn[3];
    const float infv = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st[a] = dd[a] > 0.0f ? 1 : (dd[a] < 0.0f ? -1 : 0);
        nb[a] = st[a] > 0 ? i[a] + 1 : i[a];
        tn[a] = st[a] ? ((float)nb[a] - q[a]) * iv[a] : infv;
    }
    float t = 0.0f;
    for (;;) {
        if (i[0] < 0 || i[0] >= n[0] || i[1] < 0 || i[1] >= n[1] || i[2] < 0 || i[2] >= n[2]) break;
        if (!(t < rv)) break;
        const uint8_t s = M.bricks[voxel_addr(i[0], i[1], i[2], M)];
        if (s == kOccupied) break;
        if (is_unknown(s)) f((uint32_t)i[0] + (uint32_t)n[0] * ((uint32_t)i[1] + (uint32_t)n[1] * (uint32_t)i[2]));
        const int ax = (tn[0] <= tn[1] && tn[0] <= tn[2]) ? 0 : (tn[1] <= tn[2] ? 1 : 2);
        t = tn[ax];
        i[ax] += st[ax];
        nb[ax] += st[ax];
        tn[ax] = ((float)nb[ax] - q[ax]) * iv[ax];
    }
}

// Work item = (node, window ray): blockIdx.x / tiles is the node, the rest the
// ray among the W_buf * H rays of its window (column-major like the panorama).
struct RayOf {
    int32_t node, r;
    bool ok;
};

__device__ __forceinline__ RayOf window_ray(const SensorDev& S, const int32_t* yaw, int32_t tiles,
                                            const int32_t* nodes) {
    RayOf o;
    const int32_t item = (int32_t)(blockIdx.x / (uint32_t)tiles);
    o.node = nodes ? nodes[item] : item;
    const int32_t k = (int32_t)(blockIdx.x % (uint32_t)tiles) * kXThreads + (int32_t)threadIdx.x;
    o.ok = k < S.WB * S.H;
    const int32_t ci = k / S.H, j = k % S.H;
    int32_t c = S.c0_of_win[yaw[o.node]] + ci;
    c = c >= S.W ? c - S.W : c;
    o.r = o.ok ? c * S.H + j : 0;
    return o;
}

struct CountF {
    uint32_t n = 0;
    __device__ void operator()(uint32_t) { ++n; }
};

__global__ __launch_bounds__(kXThreads) void k_exact_count(MapDev M, SensorDev S, TreeDev Tr,
                                                           const int32_t* __restrict__ yaw, int32_t tiles,
                                                           const int32_t* __restrict__ nodes,
                                                           uint32_t* __restrict__ inc) {
    const RayOf R = window_ray(S, yaw, tiles, nodes);
    CountF f;
    if (R.ok) walk_unknown(M, S.rv, Tr.q4[R.node], S.d4[R.r], S.iv4[R.r], f);
    if (f.n) atomicAdd(&inc[R.node], f.n);
}

struct InsertF {
    const Tables* T;
    int32_t node;
    uint32_t added = 0;
    __device__ void operator()(uint32_t id) { added += insert(*T, node, id) ? 1u : 0u; }
};

__global__ __launch_bounds__(kXThreads) void k_exact_insert(MapDev M, SensorDev S, TreeDev Tr, Tables T,
                                                            const int32_t* __restrict__ yaw, int32_t tiles,
                                                            const int32_t* __restrict__ nodes,
                                                            uint32_t* __restrict__ a_set) {
    const RayOf R = window_ray(S, yaw, tiles, nodes);
    InsertF f{&T, R.node};
    if (R.ok) walk_unknown(M, S.rv, Tr.q4[R.node], S.d4[R.r], S.iv4[R.r], f);
    if (f.added && a_set) atomicAdd(&a_set[R.node], f.added);
}

__device__ __forceinline__ bool seen_by_ancestors(const Tables& T, const TreeDev& Tr, int32_t node, uint32_t id) {
    const int32_t a0 = Tr.anc_ptr[node], a1 = Tr.anc_ptr[node + 1];
    for (int32_t k = a0; k < a1; ++k)
        if (contains(T, Tr.anc_ids[k], id)) return true;
    return false;
}

struct MarginalF {
    const Tables* T;
    const TreeDev* Tr;
    int32_t node;
    uint32_t n = 0;
    __device__ void operator()(uint32_t id) { n += seen_by_ancestors(*T, *Tr, node, id) ? 0u : 1u; }
};

__global__ __launch_bounds__(kXThreads) void k_exact_xray(MapDev M, SensorDev S, TreeDev Tr, Tables T,
                                                          const int32_t* __restrict__ yaw, int32_t tiles,
                                                          const int32_t* __restrict__ nodes,
                                                          uint32_t* __restrict__ x_ray) {
    const RayOf R = window_ray(S, yaw, tiles, nodes);
    MarginalF f{&T, &Tr, R.node};
    if (R.ok) walk_unknown(M, S.rv, Tr.q4[R.node], S.d4[R.r], S.iv4[R.r], f);
    if (f.n) atomicAdd(&x_ray[R.node], f.n);
}

// Own-yaw exact gain, one level: work item = (level node, panorama ray); each
// unknown incidence whose voxel is in no ancestor's set counts towards the bin
// of the ray's column (the node's marginal bins).
__global__ __launch_bounds__(kXThreads) void k_exact_bins(MapDev M, SensorDev S, TreeDev Tr, Tables T,
                                                          const int32_t* __restrict__ nodes, int32_t tiles) {
    __shared__ uint32_t s_bins[kMaxBins];
    const int32_t node = nodes[blockIdx.x / (uint32_t)tiles];
    const int32_t r = (int32_t)(blockIdx.x % (uint32_t)tiles) * kXThreads + (int32_t)threadIdx.x;
    for (int32_t i = threadIdx.x; i < S.B; i += kXThreads) s_bins[i] = 0u;
    __syncthreads();
    if (r < S.R) {
        MarginalF f{&T, &Tr, node};
        walk_unknown(M, S.rv, Tr.q4[node], S.d4[r], S.iv4[r], f);
        if (f.n) atomicAdd(&s_bins[S.bin_of_col[r / S.H]], f.n);
    }
    __syncthreads();
    uint32_t* gb = Tr.bins + (size_t)node * 2 * S.B + S.B;
    for (int32_t i = threadIdx.x; i < S.B; i += kXThreads)
        if (s_bins[i]) atomicAdd(&gb[i], s_bins[i]);
}

// Grid: (slot blocks, nodes); every occupied slot of node n's table not in an
// ancestor's table adds one to X_set(n).
__global__ __launch_bounds__(kXThreads) void k_exact_xset(TreeDev Tr, Tables T, int32_t n_nodes,
                                                          uint32_t* __restrict__ x_set) {
    for (int32_t node = (int32_t)blockIdx.y; node < n_nodes; node += (int32_t)gridDim.y) {
        const uint64_t cap = (uint64_t)T.mask[node] + 1u;
        const uint32_t* t = T.slots + T.off[node];
        uint32_t n = 0;
        for (uint64_t h = blockIdx.x * (uint64_t)kXThreads + threadIdx.x; h < cap;
             h += (uint64_t)gridDim.x * kXThreads) {
            const uint32_t id = t[h];
            if (id != kEmpty && !seen_by_ancestors(T, Tr, node, id)) ++n;
        }
        if (n) atomicAdd(&x_set[node], n);
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Per-tree device state: incidence counts, table offsets and masks, the pool.
struct State {
    uint32_t* inc = nullptr;       // [n]
    uint64_t* off = nullptr;       // [n]
    uint32_t* mask = nullptr;      // [n]
    uint32_t* pool = nullptr;
    size_t pool_slots = 0;
    std::vector<uint32_t> inc_h, mask_h;
    std::vector<uint64_t> off_h;
};

std::mutex g_mu;
std::map<mg_tree, State> g_state;

unsigned blocks_for(size_t n) {
    size_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

int fail_hip(hipError_t e, const char* what) {
    return mgb::set_error(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, what);
}

// Lays out one table per node, a power of two at least twice bound[i] slots
// (bound[i] >= |I(i)|), grows the pool when needed, uploads the layout and
// marks every slot empty. The host layout must outlive the enqueued copies
// (the caller synchronises before returning).
int setup_tables(State& st, int32_t n, const uint32_t* bound, hipStream_t s, Tables* T) {
    hipError_t e = hipSuccess;
    if (!st.inc) {
        e = hipMalloc(&st.inc, sizeof(uint32_t) * n);
        if (e == hipSuccess) e = hipMalloc(&st.off, sizeof(uint64_t) * n);
        if (e == hipSuccess) e = hipMalloc(&st.mask, sizeof(uint32_t) * n);
        if (e != hipSuccess) return fail_hip(e, "exact-gain state");
        st.inc_h.resize(n);
        st.off_h.resize(n);
        st.mask_h.resize(n);
    }
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        uint64_t cap = 64;
        while (cap < 2ull * bound[i]) cap *= 2;
        if (cap > (1ull << 32)) return mgb::set_error(MG_E_UNSUPPORTED, "a node's set needs more than 2^32 slots");
        st.off_h[i] = total;
        st.mask_h[i] = (uint32_t)(cap - 1);
        total += cap;
    }
    if (total > st.pool_slots) {
        (void)hipFree(st.pool);
        st.pool = nullptr;
        st.pool_slots = 0;
        e = hipMalloc(&st.pool, sizeof(uint32_t) * total);
        if (e != hipSuccess) return fail_hip(e, "exact-gain tables");
        st.pool_slots = total;
    }
    e = hipMemcpyAsync(st.off, st.off_h.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st.mask, st.mask_h.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e, "exact-gain table layout");
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(total)), dim3(256), 0, s, st.pool, total, kEmpty);
    *T = Tables{st.pool, st.off, st.mask};
    return MG_OK;
}

}  // namespace mgx

namespace mgb {
void forget_exact(mg_tree t) {
    std::lock_guard<std::mutex> lk(mgx::g_mu);
    auto it = mgx::g_state.find(t);
    if (it == mgx::g_state.end()) return;
    (void)hipFree(it->second.inc);
    (void)hipFree(it->second.off);
    (void)hipFree(it->second.mask);
    (void)hipFree(it->second.pool);
    mgx::g_state.erase(it);
}
}  // namespace mgb

extern "C" int mg_eval_exact(mg_tree t, void* hip_stream, const int32_t* yaw_bin, uint32_t* x_ray, uint32_t* x_set,
                             uint32_t* a_set) {
    using namespace mgx;
    if (!t || !yaw_bin || !x_ray) return mgb::set_error(MG_E_INVALID, "tree/yaw_bin/x_ray is NULL");
    mgb::TreeView v;
    int rc = mgb::tree_view(t, &v);
    if (rc != MG_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != v.device) return mgb::set_error(MG_E_INVALID, "the tree lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    const SensorDev& S = *v.sd;
    const TreeDev& Tr = *v.td;
    const int32_t n = v.n;
    const int32_t tiles = (S.WB * S.H + kXThreads - 1) / kXThreads;
    const dim3 grid((unsigned)n * (unsigned)tiles);
    {
        // windows are indices into the sensor's tables: check them on the host
        std::vector<int32_t> k(n);
        e = hipMemcpyAsync(k.data(), yaw_bin, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail_hip(e, "exact-gain windows");
        for (int32_t i = 0; i < n; ++i)
            if (k[i] < 0 || k[i] >= S.B) return mgb::set_error(MG_E_INVALID, "a window index is outside [0, yaw_bins)");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    State& st = g_state[t];
    if (!st.inc) {
        e = hipMalloc(&st.inc, sizeof(uint32_t) * n);
        if (e == hipSuccess) e = hipMalloc(&st.off, sizeof(uint64_t) * n);
        if (e == hipSuccess) e = hipMalloc(&st.mask, sizeof(uint32_t) * n);
        if (e != hipSuccess) return fail_hip(e, "exact-gain state");
        st.inc_h.resize(n);
        st.off_h.resize(n);
        st.mask_h.resize(n);
    }
    // 1. unknown incidences per node bound |I(n)|: size the tables
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, s, st.inc, (size_t)n, 0u);
    hipLaunchKernelGGL(k_exact_count, grid, dim3(kXThreads), 0, s, *v.map, S, Tr, yaw_bin, tiles, nullptr, st.inc);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(st.inc_h.data(), st.inc, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "exact-gain sizing");
    Tables T{};
    rc = setup_tables(st, n, st.inc_h.data(), s, &T);
    if (rc != MG_OK) return rc;
    // 2. sets, 3. X_ray, 4. X_set
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, s, x_ray, (size_t)n, 0u);
    if (x_set) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, s, x_set, (size_t)n, 0u);
    if (a_set) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, s, a_set, (size_t)n, 0u);
    hipLaunchKernelGGL(k_exact_insert, grid, dim3(kXThreads), 0, s, *v.map, S, Tr, T, yaw_bin, tiles, nullptr, a_set);
    hipLaunchKernelGGL(k_exact_xray, grid, dim3(kXThreads), 0, s, *v.map, S, Tr, T, yaw_bin, tiles, nullptr, x_ray);
    if (x_set) {
        uint64_t maxcap = 0;
        for (int32_t i = 0; i < n; ++i) maxcap = std::max<uint64_t>(maxcap, (uint64_t)st.mask_h[i] + 1u);
        const unsigned bx = (unsigned)std::min<uint64_t>((maxcap + kXThreads - 1) / kXThreads, 1024);
        hipLaunchKernelGGL(k_exact_xset, dim3(bx, (unsigned)std::min(n, 65535)), dim3(kXThreads), 0, s, Tr, T, n,
                           x_set);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "exact-gain kernels");
    // the host copies of the layout must outlive the copies enqueued above
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "exact-gain kernels");
    return MG_OK;
}

extern "C" int mg_eval_exact_marginal(mg_tree t, void* hip_stream, uint32_t* gain, int32_t* yaw_bin) {
    using namespace mgx;
    if (!t || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "tree/gain/yaw_bin is NULL");
    mgb::TreeView v;
    int rc = mgb::tree_view(t, &v);
    if (rc != MG_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != v.device) return mgb::set_error(MG_E_INVALID, "the tree lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    const SensorDev& S = *v.sd;
    const TreeDev& Tr = *v.td;
    const int32_t n = v.n;
    std::lock_guard<std::mutex> lk(g_mu);
    State& st = g_state[t];
    // 1. bound |I(n)| by the absolute gain (the largest window's unknown incidences)
    e = launch_zero_u32(Tr.bins, (size_t)2 * S.B * n, s);
    if (e == hipSuccess) e = launch_trace(*v.map, S, Tr, Tr.level_nodes, n, false, s);
    if (e == hipSuccess) e = launch_finish(S, Tr, Tr.level_nodes, n, false, v.scratch_gain, v.scratch_yaw, s);
    std::vector<uint32_t> bound(n);
    if (e == hipSuccess) e = hipMemcpyAsync(bound.data(), v.scratch_gain, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "exact-gain sizing");
    Tables T{};
    rc = setup_tables(st, n, bound.data(), s, &T);
    if (rc != MG_OK) return rc;
    // 2. level by level: new incidences per bin, window, then the node's set at that window
    e = launch_zero_u32(Tr.bins, (size_t)2 * S.B * n, s);
    const int32_t tiles_all = (S.R + kXThreads - 1) / kXThreads;
    const int32_t tiles_win = (S.WB * S.H + kXThreads - 1) / kXThreads;
    for (int32_t d = 0; d < v.levels && e == hipSuccess; ++d) {
        const int32_t b = (*v.level_ptr)[d], cnt = (*v.level_ptr)[d + 1] - b;
        if (cnt <= 0) continue;
        const int32_t* nodes = Tr.level_nodes + b;
        hipLaunchKernelGGL(k_exact_bins, dim3((unsigned)cnt * (unsigned)tiles_all), dim3(kXThreads), 0, s, *v.map, S,
                           Tr, T, nodes, tiles_all);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_finish(S, Tr, nodes, cnt, true, gain, yaw_bin, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_exact_insert, dim3((unsigned)cnt * (unsigned)tiles_win), dim3(kXThreads), 0, s,
                               *v.map, S, Tr, T, (const int32_t*)yaw_bin, tiles_win, nodes, nullptr);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "exact marginal gain");
    return MG_OK;
}
