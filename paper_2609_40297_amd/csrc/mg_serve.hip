// Serving loop: replanning requests from many robots, continuously batched.
//
// A worker thread runs steps. A step advances every in-flight request by one
// depth level (Sec. IV-C's order inside each request) with one trace launch and
// one window launch over the union of their current-level nodes, so requests
// at different depths, on different maps, share the GPU. Requests are admitted
// between steps, first come first served, when a slot is free and their tree
// fits in the server's device arena (admission by device-memory footprint);
// a finished request's results are copied to the caller's host arrays and its
// arena block is released. Nothing on the request path allocates device memory.
//
// Map updates between replans are queued with the requests. An update is
// applied once every request on its map submitted before it has finished and
// no in-flight request uses the map: requests submitted before it see the old
// map, requests on that map submitted after it wait for it and see the new
// one, and requests on other maps are not held back by it.
//
// Failure isolation: every in-flight request has a device status word that its
// kernels check first; a nonzero word (set by mg_server_fail_request, as a
// kernel that finds an error in the request's data would) makes them skip the
// request, and the step that reads it back retires the request with that
// status while the others continue. A cancelled request is dropped from the
// queue at once, or at the next step boundary when it is in flight. While
// paused, requests are still admitted but no step runs.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mg_batch.h"

using namespace mgk;
using Clock = std::chrono::steady_clock;

namespace {

// First-fit allocator over [0, size) with 256-byte granules and coalescing.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
        size_ = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0;
};

struct Request {
    int64_t ticket = 0;
    int kind = 0;                    // 0 a tree to evaluate, 1 a map update
    mg_map map = nullptr;
    std::vector<uint32_t> upd_ids;   // map update: voxel ids and new states (host copies)
    std::vector<uint8_t> upd_states;
    mgb::HostTree* host = nullptr;
    int32_t n = 0;
    uint32_t* out_gain = nullptr;    // caller's host arrays
    int32_t* out_yaw = nullptr;
    Clock::time_point t_submit, t_done;
    size_t bytes = 0, arena_off = 0;
    mg_tree tree = nullptr;
    const std::vector<int32_t>* level_ptr = nullptr;
    const std::vector<int32_t>* level_nodes = nullptr;
    const std::vector<int32_t>* mask_level_ptr = nullptr;   // nodes with children, by level
    const std::vector<int32_t>* mask_nodes = nullptr;
    int32_t level = 0, levels = 0;
    int rc = MG_OK;
    int state = 0;                   // 0 queued, 1 in flight, 2 done (rc tells success)
    int32_t slot = -1;               // in flight: index of the request's device status word
    int32_t inject = 0;              // status set by mg_server_fail_request (0: none)
    bool inject_sent = false;        // ... and written to the device
    bool cancel = false;             // cancelled while in flight (dropped at the next step boundary)
    bool holds_map = false;          // a reference on `map` (mg_map_destroy answers MG_E_BUSY meanwhile)
    void hold_map(mg_map m) {
        map = m;
        mgb::map_ref(m, 1);
        holds_map = true;
    }
    // Done (rc tells success): the map is no longer used by this request.
    void finish(int code) {
        rc = code;
        state = 2;
        t_done = Clock::now();
        if (holds_map) mgb::map_ref(map, -1);
        holds_map = false;
    }
    ~Request() {
        if (host) mgb::free_host_tree(host);
        if (holds_map) mgb::map_ref(map, -1);
    }
};

int hip_fail(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return mgb::set_error(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, m.c_str());
}

}  // namespace

struct mg_server_s {
    mg_server_config cfg{};
    int device = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::vector<Request*> inflight;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    int64_t next_ticket = 1;
    bool stop = false;
    bool paused = false;
    uint64_t wake_seq = 0;              // bumped by every call that may give a paused worker work
    int fatal = MG_OK;
    std::string fatal_msg;
    hipStream_t compute = nullptr, upload = nullptr;
    void* arena_mem = nullptr;
    Arena arena;
    // per-step launch descriptors: device arrays and pinned host staging
    BatchTree* d_trees = nullptr;
    unsigned long long* d_items = nullptr;
    BatchTree* h_trees = nullptr;
    unsigned long long* h_items = nullptr;
    size_t cap_trees = 0, cap_items = 0;
    uint32_t* h_stage = nullptr;        // pinned: gain then yaw of finished requests
    size_t cap_stage = 0;
    uint32_t* d_upd = nullptr;          // map updates: ids, then states (device), grown on demand
    size_t cap_upd = 0;
    int32_t* d_status = nullptr;        // [max_inflight] device status word per in-flight slot
    int32_t* h_status = nullptr;        // pinned [2 * max_inflight]: read-back, then injection staging
    std::vector<int32_t> free_slots;
    // statistics
    int64_t steps = 0, completed = 0;
    double rays_done = 0.0;

    int grow(size_t trees, size_t items, size_t stage_words);
    int apply_update(Request* r);
    int send_status(Request* r);
    void retire(Request* r, int code);
    void run();
    int step();
};

// Applies a queued map update on the compute stream (after every earlier
// launch on it) and waits for it, so the host copies can be released.
int mg_server_s::apply_update(Request* r) {
    const size_t n = r->upd_ids.size();
    if (n == 0) return MG_OK;
    const size_t words = n + (n + 3) / 4;
    hipError_t e = hipSuccess;
    if (words > cap_upd) {
        (void)hipFree(d_upd);
        d_upd = nullptr;
        cap_upd = 0;
        e = hipMalloc(&d_upd, sizeof(uint32_t) * std::max(words, (size_t)1024));
        if (e != hipSuccess) return hip_fail(e, "server map update staging");
        cap_upd = std::max(words, (size_t)1024);
    }
    uint8_t* d_states = (uint8_t*)(d_upd + n);
    e = hipMemcpyAsync(d_upd, r->upd_ids.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, compute);
    if (e == hipSuccess) e = hipMemcpyAsync(d_states, r->upd_states.data(), n, hipMemcpyHostToDevice, compute);
    if (e == hipSuccess) e = launch_map_scatter(d_upd, d_states, (uint32_t)n, *mgb::map_dev(r->map), nullptr, compute);
    if (e == hipSuccess) e = launch_brick_flags(*mgb::map_dev(r->map), compute);
    if (e == hipSuccess) e = hipStreamSynchronize(compute);
    if (e != hipSuccess) return hip_fail(e, "server map update");
    return MG_OK;
}

// Writes a request's injected status to its device status word (compute
// stream; the pinned staging word is not reused before the step's end).
int mg_server_s::send_status(Request* r) {
    const int32_t m = cfg.max_inflight;
    h_status[m + r->slot] = r->inject;
    const hipError_t e =
        hipMemcpyAsync(d_status + r->slot, h_status + m + r->slot, sizeof(int32_t), hipMemcpyHostToDevice, compute);
    if (e != hipSuccess) return hip_fail(e, "server status word");
    r->inject_sent = true;
    return MG_OK;
}

// Ends an in-flight request that will not complete (failed or cancelled):
// its tree, arena block and status slot are released. The caller holds mu and
// no work of the request is pending on the compute stream.
void mg_server_s::retire(Request* r, int code) {
    if (r->tree) mg_tree_destroy(r->tree);
    r->tree = nullptr;
    arena.release(r->arena_off, r->bytes);
    free_slots.push_back(r->slot);
    r->slot = -1;
    r->finish(code);
    inflight.erase(std::find(inflight.begin(), inflight.end(), r));
}

int mg_server_s::grow(size_t trees, size_t items, size_t stage_words) {
    hipError_t e = hipSuccess;
    if (trees > cap_trees) {
        const size_t c = std::max(trees, cap_trees * 2);
        (void)hipFree(d_trees);
        (void)hipHostFree(h_trees);
        d_trees = nullptr;
        h_trees = nullptr;
        e = hipMalloc(&d_trees, sizeof(BatchTree) * c);
        if (e == hipSuccess) e = hipHostMalloc(&h_trees, sizeof(BatchTree) * c, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "server descriptors");
        cap_trees = c;
    }
    if (items > cap_items) {
        const size_t c = std::max(items, cap_items * 2);
        (void)hipFree(d_items);
        (void)hipHostFree(h_items);
        d_items = nullptr;
        h_items = nullptr;
        e = hipMalloc(&d_items, sizeof(unsigned long long) * c);
        if (e == hipSuccess) e = hipHostMalloc(&h_items, sizeof(unsigned long long) * c, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "server work lists");
        cap_items = c;
    }
    if (stage_words > cap_stage) {
        const size_t c = std::max(stage_words, cap_stage * 2);
        (void)hipHostFree(h_stage);
        h_stage = nullptr;
        e = hipHostMalloc(&h_stage, sizeof(uint32_t) * c, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "server staging");
        cap_stage = c;
    }
    return MG_OK;
}

// One step: admit, launch one level of every in-flight request, retire finished ones.
int mg_server_s::step() {
    // Admission, in queue order. A map update is applied once no in-flight
    // request uses its map (and not while paused); until then every later
    // entry on that map stays queued behind it, while entries on other maps go
    // ahead. Requests are admitted first come first served: the first that
    // finds no free slot or arena block ends the admission (and so holds back
    // what is queued behind it).
    for (;;) {
        Request* r = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            std::vector<mg_map> held;              // maps with an update still queued
            for (auto it = queue.begin(); it != queue.end(); ++it) {
                Request* q = *it;
                const bool behind = std::find(held.begin(), held.end(), q->map) != held.end();
                if (q->kind == 1) {
                    if (!behind && !paused &&
                        std::none_of(inflight.begin(), inflight.end(), [&](Request* f) { return f->map == q->map; })) {
                        r = q;
                        queue.erase(it);
                        break;
                    }
                    if (!behind) held.push_back(q->map);
                    continue;
                }
                if (behind) continue;                  // it must see the update queued before it
                if ((int32_t)inflight.size() >= cfg.max_inflight) break;
                size_t off = 0;
                if (!arena.alloc(q->bytes, &off)) break;
                q->arena_off = off;
                q->slot = free_slots.back();
                free_slots.pop_back();
                r = q;
                queue.erase(it);
                break;
            }
            if (r == nullptr) break;
        }
        if (r->kind == 1) {
            const int urc = apply_update(r);
            std::lock_guard<std::mutex> lk(mu);
            r->upd_ids = std::vector<uint32_t>();
            r->upd_states = std::vector<uint8_t>();
            r->finish(urc);
            cv_done.notify_all();
            if (urc != MG_OK) return urc;
            continue;
        }
        int rc = mgb::upload_into(r->map, *r->host, &cfg.sensor, upload, (char*)arena_mem + r->arena_off, &r->tree);
        std::lock_guard<std::mutex> lk(mu);
        if (rc != MG_OK) {
            arena.release(r->arena_off, r->bytes);
            free_slots.push_back(r->slot);
            r->slot = -1;
            r->finish(rc);
            cv_done.notify_all();
            continue;
        }
        mgb::TreeView v;
        mgb::tree_view(r->tree, &v);
        r->level_ptr = v.level_ptr;
        r->level_nodes = v.level_nodes;
        r->mask_level_ptr = v.mask_level_ptr;
        r->mask_nodes = v.mask_nodes;
        r->level = 0;
        r->levels = v.levels;
        r->state = 1;
        hipError_t e = launch_zero_u32(v.td->bins, (size_t)2 * v.sd->B * v.n, compute);
        if (e == hipSuccess) e = launch_zero_u32((uint32_t*)(d_status + r->slot), 1, compute);
        if (e != hipSuccess) return hip_fail(e, "server bins");
        if (r->inject != 0) {            // failed (mg_server_fail_request) while queued
            rc = send_status(r);
            if (rc != MG_OK) return rc;
        }
        inflight.push_back(r);
    }
    std::vector<Request*> active;
    {
        // cancelled requests leave (the previous step has drained the stream);
        // statuses injected since the last step go to the device
        std::lock_guard<std::mutex> lk(mu);
        std::vector<Request*> gone;
        for (Request* r : inflight) {
            if (r->cancel) {
                gone.push_back(r);
            } else if (r->inject != 0 && !r->inject_sent) {
                const int rc = send_status(r);
                if (rc != MG_OK) return rc;
            }
        }
        for (Request* r : gone) retire(r, MG_E_CANCELLED);
        if (!gone.empty()) cv_done.notify_all();
        if (paused) return MG_OK;
        active = inflight;
    }
    if (active.empty()) return MG_OK;

    // descriptors and the work lists of this step: every node of the current
    // levels, and those of them with children (their path masks are built)
    size_t n_items = 0, n_mitems = 0, stage = 0;
    uint32_t mask_bricks = 0;
    for (Request* r : active) {
        n_items += (size_t)((*r->level_ptr)[r->level + 1] - (*r->level_ptr)[r->level]);
        n_mitems += (size_t)((*r->mask_level_ptr)[r->level + 1] - (*r->mask_level_ptr)[r->level]);
        mask_bricks = std::max(mask_bricks, mgb::map_dev(r->map)->build_slots);
        if (r->level + 1 == r->levels) stage += 2 * (size_t)r->n;
    }
    int rc = grow(active.size(), n_items + n_mitems, stage);
    if (rc != MG_OK) return rc;
    SensorDev sd{};
    size_t k = 0, km = n_items;
    for (size_t i = 0; i < active.size(); ++i) {
        Request* r = active[i];
        mgb::TreeView v;
        mgb::tree_view(r->tree, &v);
        if (i == 0) sd = *v.sd;
        BatchTree& bt = h_trees[i];
        bt.map = *v.map;
        bt.td = *v.td;
        bt.rv = v.sd->rv;
        bt.rv2 = v.sd->rv2;
        bt.gain = v.scratch_gain;
        bt.yaw = v.scratch_yaw;
        bt.depth = nullptr;
        bt.status = d_status + r->slot;
        for (int32_t j = (*r->level_ptr)[r->level]; j < (*r->level_ptr)[r->level + 1]; ++j)
            h_items[k++] = ((unsigned long long)i << 32) | (uint32_t)(*r->level_nodes)[j];
        for (int32_t j = (*r->mask_level_ptr)[r->level]; j < (*r->mask_level_ptr)[r->level + 1]; ++j)
            h_items[km++] = ((unsigned long long)i << 32) | (uint32_t)(*r->mask_nodes)[j];
    }
    hipError_t e = hipMemcpyAsync(d_trees, h_trees, sizeof(BatchTree) * active.size(), hipMemcpyHostToDevice, compute);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_items, h_items, sizeof(unsigned long long) * (n_items + n_mitems), hipMemcpyHostToDevice,
                           compute);
    if (e == hipSuccess)
        e = launch_batch_level(d_trees, d_items, (int32_t)n_items, d_items + n_items, (int32_t)n_mitems, mask_bricks, sd,
                               compute, serve_shape());
    size_t so = 0;
    std::vector<std::pair<Request*, size_t>> finishing;
    for (Request* r : active) {
        if (r->level + 1 != r->levels || e != hipSuccess) continue;
        mgb::TreeView v;
        mgb::tree_view(r->tree, &v);
        e = hipMemcpyAsync(h_stage + so, v.scratch_gain, sizeof(uint32_t) * r->n, hipMemcpyDeviceToHost, compute);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_stage + so + r->n, v.scratch_yaw, sizeof(int32_t) * r->n, hipMemcpyDeviceToHost,
                               compute);
        finishing.emplace_back(r, so);
        so += 2 * (size_t)r->n;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_status, d_status, sizeof(int32_t) * cfg.max_inflight, hipMemcpyDeviceToHost, compute);
    if (e == hipSuccess) e = hipStreamSynchronize(compute);
    if (e != hipSuccess) return hip_fail(e, "server step");
    ++steps;
    std::lock_guard<std::mutex> lk(mu);
    bool any = false;
    for (Request* r : active) {
        r->level++;
        const int32_t st = h_status[r->slot];
        if (st != 0) {              // failed on the device: its results are not copied
            retire(r, st < 0 ? st : (int)MG_E_DEVICE);
            any = true;
        }
    }
    for (auto& f : finishing) {
        Request* r = f.first;
        if (r->state == 2) continue;
        std::memcpy(r->out_gain, h_stage + f.second, sizeof(uint32_t) * r->n);
        std::memcpy(r->out_yaw, h_stage + f.second + r->n, sizeof(int32_t) * r->n);
        rays_done += (double)r->n * cfg.sensor.n_az * cfg.sensor.n_el;
        ++completed;
        retire(r, MG_OK);
        any = true;
    }
    if (any) cv_done.notify_all();
    return MG_OK;
}

void mg_server_s::run() {
    (void)hipSetDevice(device);
    uint64_t seen = ~0ull;
    for (;;) {
        {
            // running: work while anything is queued or in flight; paused: one
            // admission pass per call that may have changed something
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || (paused ? wake_seq != seen : (!queue.empty() || !inflight.empty()));
            });
            if (stop && queue.empty() && inflight.empty()) return;
            seen = wake_seq;
        }
        const int rc = step();
        if (rc != MG_OK) {
            // a device error ends the server: every pending request fails with it
            std::lock_guard<std::mutex> lk(mu);
            fatal = rc;
            fatal_msg = mg_last_error();
            for (Request* r : inflight) r->finish(rc);
            for (Request* r : queue) r->finish(rc);
            inflight.clear();
            queue.clear();
            cv_done.notify_all();
            return;
        }
    }
}

extern "C" int mg_server_create(const mg_server_config* cfg, mg_server* out) {
    if (!out) return mgb::set_error(MG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->max_inflight < 1 || cfg->arena_bytes < 1)
        return mgb::set_error(MG_E_INVALID, "server needs max_inflight >= 1 and arena_bytes >= 1");
    float tab[1];
    (void)tab;
    int rc = mg_sensor_tables(&cfg->sensor, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (rc != MG_OK) return rc;
    std::unique_ptr<mg_server_s> S(new (std::nothrow) mg_server_s());
    if (!S) return mgb::set_error(MG_E_NOMEM, "host allocation failed");
    S->cfg = *cfg;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&S->arena_mem, (size_t)cfg->arena_bytes);
    if (e == hipSuccess) e = hipMalloc(&S->d_status, sizeof(int32_t) * (size_t)cfg->max_inflight);
    if (e == hipSuccess)
        e = hipHostMalloc(&S->h_status, sizeof(int32_t) * 2 * (size_t)cfg->max_inflight, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(S->arena_mem);
        (void)hipFree(S->d_status);
        if (S->compute) (void)hipStreamDestroy(S->compute);
        if (S->upload) (void)hipStreamDestroy(S->upload);
        return hip_fail(e, "server setup");
    }
    for (int32_t i = cfg->max_inflight - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->arena.reset((size_t)cfg->arena_bytes);
    mg_server_s* raw = S.get();
    S->worker = std::thread([raw] { raw->run(); });
    *out = S.release();
    return MG_OK;
}

extern "C" int mg_server_submit(mg_server s, mg_map map, const float* pos_m, const int32_t* parent, int32_t n,
                                uint32_t* gain, int32_t* yaw_bin, int64_t* ticket) {
    if (!s || !ticket || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "server/ticket/outputs is NULL");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return mgb::set_error(MG_E_NOMEM, "host allocation failed");
    r->host = mgb::new_host_tree();
    if (!r->host) return mgb::set_error(MG_E_NOMEM, "host allocation failed");
    const int rc = mgb::prepare(map, pos_m, parent, n, &s->cfg.sensor, r->host);
    if (rc != MG_OK) return rc;
    r->bytes = mgb::block_bytes(*r->host);
    if (r->bytes > s->arena.size())
        return mgb::set_error(MG_E_NOMEM, "the tree needs more device memory than the server's whole arena");
    r->n = n;
    r->out_gain = gain;
    r->out_yaw = yaw_bin;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != MG_OK) return mgb::set_error(s->fatal, s->fatal_msg.c_str());
    if (s->stop) return mgb::set_error(MG_E_BUSY, "server is shutting down");
    r->hold_map(map);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->all.emplace(r->ticket, std::move(r));
    s->wake_seq++;
    s->cv_work.notify_one();
    return MG_OK;
}

// Retires a finished ticket (the caller holds s->mu). MG_E_INVALID when the
// ticket is unknown, e.g. retired meanwhile by another caller.
static int finish_ticket(mg_server s, std::unique_lock<std::mutex>& lk, int64_t ticket, int32_t* status,
                         double* latency_us) {
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return mgb::set_error(MG_E_INVALID, "unknown ticket (retired by another caller)");
    Request* r = it->second.get();
    if (latency_us) latency_us[0] = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    const int rc = r->rc;
    if (status) *status = rc == MG_OK ? 1 : rc;
    s->all.erase(it);
    (void)lk;
    return rc;
}

extern "C" int mg_server_map_update(mg_server s, mg_map map, const uint32_t* voxel_ids, const uint8_t* states,
                                    int32_t count, int64_t* ticket) {
    if (!s || !map || !ticket || count < 0 || (count > 0 && (!voxel_ids || !states)))
        return mgb::set_error(MG_E_INVALID, "bad map update arguments");
    const size_t nvox = mgb::map_voxel_count(map);
    for (int32_t i = 0; i < count; ++i)
        if (voxel_ids[i] >= nvox || states[i] > 2)
            return mgb::set_error(MG_E_INVALID, "map update lists a voxel outside the grid or a state above 2");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return mgb::set_error(MG_E_NOMEM, "host allocation failed");
    r->kind = 1;
    r->upd_ids.assign(voxel_ids, voxel_ids + count);
    r->upd_states.assign(states, states + count);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != MG_OK) return mgb::set_error(s->fatal, s->fatal_msg.c_str());
    if (s->stop) return mgb::set_error(MG_E_BUSY, "server is shutting down");
    r->hold_map(map);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->all.emplace(r->ticket, std::move(r));
    s->wake_seq++;
    s->cv_work.notify_one();
    return MG_OK;
}

extern "C" int mg_server_poll(mg_server s, int64_t ticket, int32_t* status, double* latency_us) {
    if (!s || !status) return mgb::set_error(MG_E_INVALID, "server/status is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return mgb::set_error(MG_E_INVALID, "unknown ticket");
    if (it->second->state != 2) {
        *status = 0;
        return MG_OK;
    }
    const int rc = finish_ticket(s, lk, ticket, status, latency_us);
    return rc == MG_E_INVALID ? rc : MG_OK;
}

extern "C" int mg_server_wait(mg_server s, int64_t ticket, double* latency_us) {
    if (!s) return mgb::set_error(MG_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->all.find(ticket) == s->all.end()) return mgb::set_error(MG_E_INVALID, "unknown ticket");
    // the ticket is looked up again on every wake-up: another caller may retire it meanwhile
    s->cv_done.wait(lk, [&] {
        auto it = s->all.find(ticket);
        return it == s->all.end() || it->second->state == 2;
    });
    const int rc = finish_ticket(s, lk, ticket, nullptr, latency_us);
    if (rc == MG_E_INVALID) return rc;
    if (rc != MG_OK) return mgb::set_error(rc, "request failed");
    return MG_OK;
}

extern "C" int mg_server_cancel(mg_server s, int64_t ticket) {
    if (!s) return mgb::set_error(MG_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return mgb::set_error(MG_E_INVALID, "unknown ticket");
    Request* r = it->second.get();
    if (r->state == 2) return mgb::set_error(MG_E_BUSY, "the request has already finished");
    if (r->state == 0) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
        r->finish(MG_E_CANCELLED);
        s->cv_done.notify_all();
    } else {
        r->cancel = true;            // the worker drops it at the next step boundary
    }
    s->wake_seq++;
    s->cv_work.notify_one();
    return MG_OK;
}

extern "C" int mg_server_fail_request(mg_server s, int64_t ticket, int32_t code) {
    if (!s) return mgb::set_error(MG_E_INVALID, "server is NULL");
    if (code >= 0) return mgb::set_error(MG_E_INVALID, "the status must be a negative error code");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return mgb::set_error(MG_E_INVALID, "unknown ticket");
    Request* r = it->second.get();
    if (r->kind != 0) return mgb::set_error(MG_E_INVALID, "a map update has no device status word");
    if (r->state == 2) return mgb::set_error(MG_E_BUSY, "the request has already finished");
    if (r->inject == 0) r->inject = code;
    s->wake_seq++;
    s->cv_work.notify_one();
    return MG_OK;
}

extern "C" int mg_server_pause(mg_server s, int32_t paused) {
    if (!s || (paused != 0 && paused != 1)) return mgb::set_error(MG_E_INVALID, "server is NULL or paused is not 0/1");
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
    s->wake_seq++;
    s->cv_work.notify_one();
    return MG_OK;
}

extern "C" int mg_server_stats(mg_server s, int64_t* steps, int64_t* completed, double* rays, int32_t* in_flight,
                               int32_t* queued) {
    if (!s) return mgb::set_error(MG_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (steps) *steps = s->steps;
    if (completed) *completed = s->completed;
    if (rays) *rays = s->rays_done;
    if (in_flight) *in_flight = (int32_t)s->inflight.size();
    if (queued) *queued = (int32_t)s->queue.size();
    return s->fatal;
}

extern "C" int mg_server_destroy(mg_server s) {
    if (!s) return mgb::set_error(MG_E_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->paused = false;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->all)
        if (kv.second->tree) mg_tree_destroy(kv.second->tree);
    (void)hipStreamSynchronize(s->compute);
    (void)hipFree(s->d_trees);
    (void)hipFree(s->d_items);
    (void)hipHostFree(s->h_trees);
    (void)hipHostFree(s->h_items);
    (void)hipHostFree(s->h_stage);
    (void)hipFree(s->d_upd);
    (void)hipFree(s->d_status);
    (void)hipHostFree(s->h_status);
    (void)hipFree(s->arena_mem);
    (void)hipStreamDestroy(s->compute);
    (void)hipStreamDestroy(s->upload);
    delete s;
    return MG_OK;
}
