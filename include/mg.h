/*
 * mg.h — C ABI of the MI355X (gfx950) path-dependent marginal information
 * gain library (paper: "GPU-Accelerated Path-Dependent Marginal Information
 * Gain for Autonomous Exploration").
 *
 * The library evaluates, for every node of an RRT of candidate viewpoints,
 * the number of unknown voxels its sensor rays meet (absolute gain, eq. 1)
 * and the number left after dropping those its ancestors' depth buffers
 * already see (path-dependent marginal gain, eq. 2, approximated with depth
 * buffers as in Sec. IV-A/IV-B), together with the best yaw window. Nodes are
 * evaluated after all their ancestors (Sec. IV-C); each node's first-hit depth
 * buffer stays on the device for its descendants (Sec. IV-A).
 *
 * Conventions
 *   - Every call returns MG_OK (0) or a negative MG_E_* code; the message of
 *     the last failure on the calling thread is returned by mg_last_error().
 *     No C++ exception crosses this interface.
 *   - Host-side validation happens before any device work: a call that
 *     returns MG_E_INVALID has enqueued nothing.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream). Evaluation
 *     calls are asynchronous on that stream; their outputs are valid once the
 *     caller has synchronised it. A device fault surfaces as MG_E_DEVICE.
 *   - Handles are opaque and owned by the library until destroyed. One handle
 *     must not be used from two streams at the same time; different handles
 *     may be used concurrently from different threads.
 *   - Units: positions in metres; depths in voxel units (multiply by the voxel
 *     size for metres); gains are integer counts of ray-voxel incidences
 *     (multiply by voxel_m^3 for the volume of eq. 1 and 2).
 */
#ifndef MG_H
#define MG_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
    MG_OK = 0,
    MG_E_INVALID = -1,      /* bad argument or input; nothing was enqueued      */
    MG_E_NOMEM = -2,        /* device or host allocation failed                 */
    MG_E_DEVICE = -3,       /* a HIP call or a kernel failed                    */
    MG_E_BUSY = -4,         /* the handle is still referenced                   */
    MG_E_UNSUPPORTED = -5,  /* valid input outside the sizes this library handles */
    MG_E_CANCELLED = -6     /* a server request was cancelled (mg_server_cancel) */
};

/* Longest root path of a tree (depth <= 64): the row length of the branch
 * output of mg_score_branches. */
#define MG_BRANCH_LEN 65

typedef struct mg_map_s* mg_map;
typedef struct mg_tree_s* mg_tree;

/* Candidate-ray sensor (Sec. III-B yaw set, Sec. IV-A depth buffers).
 * n_az columns cover 360 degrees, column c's centre at
 * az_offset_deg + (c + 1/2) * 360 / n_az; n_el rows cover fov_v_deg,
 * row j's centre at -fov_v_deg/2 + (j + 1/2) * fov_v_deg / n_el. The yaw set
 * is yaw_bins azimuth bins; a yaw window of w = yaw_bins * fov_h_deg / 360
 * bins holds w_buf = n_az * w / yaw_bins columns and defines a depth buffer of
 * n_el x w_buf pixels. Requires w and w_buf integral, 2*w < yaw_bins,
 * yaw_bins <= 256, n_az*n_el <= 2^22, 0 < fov_v_deg < 180 and range_m > 0;
 * otherwise MG_E_INVALID. */
typedef struct {
    int32_t n_az;
    int32_t n_el;
    float fov_h_deg;
    float fov_v_deg;
    float range_m;
    int32_t yaw_bins;
    float az_offset_deg;
} mg_sensor;

/* Occupancy map (Sec. III-A: voxels of edge voxel_m labelled free, occupied
 * or unknown; Sec. IV: converted to a contiguous grid and moved to the GPU).
 *   states: HOST array [nz][ny][nx], x fastest, values 0 unknown, 1 free,
 *           2 occupied (any other value: MG_E_INVALID). The library copies it
 *           into its device layout before returning; the caller may free it
 *           on return.
 *   origin_m: world position of the grid's minimum corner.
 * Sizes: 1 <= nx, ny, nz <= 8192 and nx*ny*nz < 2^32. The device copy is
 * padded per axis to a power of two of 8-voxel bricks holding at least n + 1
 * voxels (at most 8x the grid, e.g. 256 MiB for 512 x 512 x 128);
 * MG_E_UNSUPPORTED when that exceeds 2^32 - 256 bytes. */
int mg_map_create(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                  const float origin_m[3], void* hip_stream, mg_map* out);

/* Frees the map. MG_E_BUSY while trees created on it still exist, or while
 * server requests or map updates submitted on it (mg_server_submit,
 * mg_server_map_update) have not finished. */
int mg_map_destroy(mg_map map);

/* Map from a truncated signed distance field (the planners' volumetric map,
 * which Sec. IV converts into a contiguous grid on the GPU). distance (metres)
 * and weight: DEVICE float [nz][ny][nx], x fastest, read on hip_stream. A
 * voxel is unknown unless weight >= min_weight, occupied when
 * distance <= surface_m, free otherwise (comparisons with NaN are false: a
 * NaN weight is unknown, a NaN distance free). One pass reads 8 B and writes
 * the bricked byte per voxel; the call returns after it finished. Same
 * geometry rules and errors as mg_map_create; MG_E_INVALID for a non-finite
 * surface_m or min_weight. */
int mg_map_create_tsdf(const float* distance, const float* weight, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                       const float origin_m[3], float surface_m, float min_weight, void* hip_stream, mg_map* out);

/* Replaces the states of a box of voxels [lo, lo + size) (HOST int32[3]
 * each) by the conversion above of its TSDF, distance and weight DEVICE float
 * [size_z][size_y][size_x], x fastest. Enqueued on hip_stream; evaluations
 * that must see the update go on the same stream (or are ordered after it).
 * MG_E_INVALID when the box leaves the grid. */
int mg_map_update_tsdf(mg_map map, void* hip_stream, const float* distance, const float* weight, const int32_t lo[3],
                       const int32_t size[3], float surface_m, float min_weight);

/* New states for listed voxels between replans: voxel_ids DEVICE uint32
 * [count] (linear ids x + nx (y + ny z), distinct; for repeated ids the
 * state written is one of theirs), states DEVICE uint8 [count] in {0, 1, 2}.
 * An id outside the grid or a larger state is skipped and counted into
 * *rejected (DEVICE uint32, zeroed first; may be NULL). Enqueued on
 * hip_stream. */
int mg_map_update(mg_map map, void* hip_stream, const uint32_t* voxel_ids, const uint8_t* states, int32_t count,
                  uint32_t* rejected);

/* Dense copy of the map's states: DEVICE uint8 [nz][ny][nx], x fastest,
 * enqueued on hip_stream. */
int mg_map_read(mg_map map, void* hip_stream, uint8_t* states);

/* Diagnostic: the map's bytes as the traversal reads them, in the layout of
 * mg_map_read: bits 0-1 the state, bits 2-4 of an unknown or free voxel the
 * level of the largest aligned block around it that holds its state only and
 * lies inside the grid (1: 16x16x16; 2: its 8x8x8 brick;
 * 3: its 4x4x4 quarter brick; 4: its 2x2x2 block, free voxels only; 0: none).
 * The marks let the traversal cross such a block in one step; they are kept
 * current by every write of the states. */
int mg_map_read_marked(mg_map map, void* hip_stream, uint8_t* bytes);

/* Candidate tree (Sec. III-A: nodes with positions; Sec. IV-D: the whole tree
 * is built first, then evaluated).
 *   pos_m: HOST array [n][3] in metres; parent: HOST array [n] with
 *   parent[0] = -1 and 0 <= parent[i] < i. Depth <= 64, every node inside the
 *   map, n >= 1; otherwise MG_E_INVALID. Both arrays are copied. Device
 *   buffers for all later evaluations (depth buffers, bins, ancestor lists,
 *   and one path mask of one bit per map voxel for every node with children)
 *   are allocated here, so evaluation calls allocate nothing. */
int mg_tree_upload(mg_map map, const float* pos_m, const int32_t* parent, int32_t n,
                   const mg_sensor* sensor, void* hip_stream, mg_tree* out);

int mg_tree_destroy(mg_tree tree);

/* Number of nodes and depth-buffer size (n_el * w_buf) of a tree; -1 on a NULL handle. */
int32_t mg_tree_nodes(mg_tree tree);
int32_t mg_tree_buffer_pixels(mg_tree tree);

/* Device bytes held by the tree (node data, depth buffers, bins): what an
 * admission controller must reserve for it. */
int64_t mg_tree_footprint_bytes(mg_tree tree);

/* Path-dependent marginal gain of every node (eq. 2 with depth buffers,
 * Sec. IV-B), nodes in depth order (Sec. IV-C). Per depth level: one trace
 * launch, one window selection, then one launch that records, for every node
 * of the level with children, which voxels the node or an ancestor observes
 * (its path mask, what conditions its children).
 *   gain    DEVICE uint32[n]: marginal gain at the chosen window (incidences).
 *   yaw_bin DEVICE int32[n]: chosen window k (bins k..k+w-1); the yaw angle
 *           of the window centre is az_offset + k*360/B + fov_h/2.
 *   depth   DEVICE float[n][n_el][w_buf] or NULL: each node's depth buffer at
 *           its chosen window (first-hit parameter t in voxel units).
 * All three are caller-owned device memory. */
int mg_eval_marginal(mg_tree tree, void* hip_stream, uint32_t* gain, int32_t* yaw_bin, float* depth);

/* Paper-style evaluation (Sec. IV-C: results return to the CPU after every
 * level): as mg_eval_marginal, but after each level the stream is
 * synchronised and that level's gains and yaw bins are copied into the HOST
 * arrays host_gain / host_yaw_bin ([n], required). Blocks until done. */
int mg_eval_marginal_levelsync(mg_tree tree, void* hip_stream, uint32_t* gain, int32_t* yaw_bin,
                               float* depth, uint32_t* host_gain, int32_t* host_yaw_bin);

/* Many trees at once (on one or several maps, same sensor geometry: equal
 * n_az, n_el, yaw_bins, fov and azimuth offset): all trees advance one depth
 * level at a time (Sec. IV-C), each level being one trace launch over every
 * node of that depth in every tree plus one window-selection launch, so small
 * levels of one tree share the GPU with those of the others. Outputs are
 * concatenated in tree order (tree t's nodes start at the sum of the node
 * counts of trees < t). Results equal per-tree mg_eval_marginal calls. The
 * launch plan (tree descriptors, per-level work lists) is built on the first
 * call with a given tree list and reused. MG_E_INVALID when a tree appears
 * twice in the list; MG_E_UNSUPPORTED for more than 65535 trees. */
int mg_eval_marginal_batch(const mg_tree* trees, int32_t n_trees, void* hip_stream, uint32_t* gain,
                           int32_t* yaw_bin, float* depth);

/* For callers that cannot allocate device memory (code under HIP graph capture
 * planning, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of mg_eval_marginal_batch with the same outputs and results, but
 * no allocation of any kind. The launch descriptors and per-level work lists
 * (8 bytes per node and per node with children, plus about 0.3 KB per tree)
 * go into a fixed 16 MiB device array that the library holds on every device
 * it runs on until the process ends, written from a fixed host array on
 * hip_stream. Every depth level runs on hip_stream (no stream groups, launch
 * shape 0, no graph). The call waits until the previous call's copies have
 * left the host array. Calls that overlap on one device (other streams or
 * threads) share the array and race: serialise them. MG_E_UNSUPPORTED for more
 * than 4096 trees or descriptors and lists above 16 MiB; other errors as
 * mg_eval_marginal_batch. */
int mg_eval_marginal_batch_noalloc(const mg_tree* trees, int32_t n_trees, void* hip_stream, uint32_t* gain,
                                   int32_t* yaw_bin, float* depth);

/* Path score of every node of a batch (Sec. III-C): traversal cost
 * c(n) = c(Pa(n)) + |p_n - p_Pa(n)| in metres (eq. 3) and exponential
 * objective o(n) = o(Pa(n)) + g(n) exp(-lambda c(n)) (eq. 4), with g(n) the
 * gain count times the voxel volume (m^3) and c(root) = 0, o(root) = g(root);
 * float64 on the float32 positions. best[t] is tree t's node of largest o
 * (smallest id on ties): the end of its best branch. branch (may be NULL):
 * DEVICE int32 [n_trees][MG_BRANCH_LEN], row t the node ids of that branch
 * from the root to best[t], then -1 to the end of the row; the first node
 * after the root is the segment a planner executes. The tree list must have a
 * plan (a prior
 * mg_eval_marginal_batch call); gain is the DEVICE uint32 array of gains in
 * the batch's concatenated order (usually that call's output), enqueued on
 * hip_stream after it. cost (may be NULL) and objective: DEVICE double [sum of
 * n]; best: DEVICE int32 [n_trees]. MG_E_INVALID for lambda < 0 or no plan. */
int mg_score_branches(const mg_tree* trees, int32_t n_trees, void* hip_stream, const uint32_t* gain, double lambda,
                      double* cost, double* objective, int32_t* best, int32_t* branch);

/* Launch configuration of mg_eval_marginal_batch for plans built after this
 * call (cached plans are dropped, after the device has finished their work).
 *   shape: -1 (default) = autotune: the first call with a tree list whose
 *          workload shape (sensor, range, map dims, tree count, depth, node
 *          count to a power of two) has not been seen times every compiled
 *          launch shape (trace and mask-builder workgroup sizes) on that
 *          call's own trees, twice each, keeps the fastest for that workload
 *          shape, and blocks until done; 0 .. count-1 = that shape
 *          (mg_trace_shapes).
 *   launch: 0 (default) = per depth level a trace, a window and a mask-builder
 *          launch, on three stream groups; 1 = those launches recorded once
 *          into a HIP graph that each call replays (on a library stream joined
 *          to hip_stream by events before and after); 2 = one persistent
 *          cooperative launch per call (Sec. IV-C's level order over all trees:
 *          as many workgroups as the device holds at once, each phase of each
 *          level dealt out to them, grid barriers between the phases; shape 0;
 *          the call waits for it and returns MG_E_DEVICE if a barrier wait gave
 *          up, see mg_batch_barrier_polls; MG_E_UNSUPPORTED at the first call
 *          when the device has no cooperative launch).
 * Results do not depend on either setting. MG_E_INVALID for other values. */
int mg_batch_config(int32_t shape, int32_t launch);

/* Polls (each about 0.2 us) of one grid-barrier wait of the persistent batch
 * launch before it gives up and every workgroup leaves (default 2^25, several
 * seconds, far beyond any phase); 0 .. 2^31 - 1, else MG_E_INVALID. For
 * callers that bound how long a stalled launch may hold the device. */
int mg_batch_barrier_polls(int64_t polls);

/* The compiled launch shapes: *count, and for the first `capacity` shapes the
 * rays per workgroup of the trace kernel and the 8x8x8-voxel bricks per
 * workgroup of the path-mask builder. Host only. */
int mg_trace_shapes(int32_t* count, int32_t* threads, int32_t* bricks, int32_t capacity);

/* Launch shape index and launch form (0 one by one, 1 graph replay, 2
 * persistent) of the cached plan of this tree list. MG_E_INVALID when the list
 * has no plan yet. */
int mg_batch_plan_info(const mg_tree* trees, int32_t n_trees, int32_t* shape, int32_t* graphed);

/* Single-parent gain g_sp (the comparison gain of Sec. V-A, Fig. 4): as
 * mg_eval_marginal, but each node is conditioned on its parent's depth buffer
 * only; the parent's window and buffer are its own single-parent results.
 * Same outputs and errors as mg_eval_marginal; it overwrites the tree's
 * buffers, so a later path score or descendant evaluation sees these. */
int mg_eval_single_parent(mg_tree tree, void* hip_stream, uint32_t* gain, int32_t* yaw_bin, float* depth);

/* Marginal gain with the paper's own ancestor test (Sec. IV-A, IV-B,
 * eq. 5-7), "interval mode". Each node keeps a pinhole depth buffer of
 * wd x hd pixels at its chosen yaw (wd, hd <= 0: the resolution rule of
 * Sec. IV-A, ceil(2 d_max tan(fov/2) / v) per axis), holding the camera-frame
 * z (voxel units) of the first occupied voxel through each pixel centre, or
 * of the ray's end at the range limit. A candidate ray is moved into every
 * ancestor's camera frame, clipped to z in [1/64, Rv], projected (eq. 5),
 * clipped to the buffer (Liang-Barsky) and walked pixel by pixel (2D DDA)
 * with inverse depth linear in screen space (eq. 6); where z <= the stored
 * depth it is observed, which gives each ancestor's overlap intervals in t
 * (eq. 7); the intervals of all ancestors are merged. An unknown voxel counts
 * unless the midpoint of its chord [t_enter, min(t_exit, Rv)] lies in a
 * merged interval. Camera frame of yaw psi: x = (sin, -cos, 0), y = (0, 0, -1),
 * z = (cos, sin, 0); window k's yaw is az_offset + (k + w/2) * 360 / B.
 * Candidate rays, bins and windows are those of mg_eval_marginal.
 *   gain DEVICE uint32[n], yaw_bin DEVICE int32[n], depth DEVICE float
 *   [n][hd][wd] or NULL. The first call on a tree (or a call with another
 *   buffer size) allocates the tree's buffers and copies the camera tables
 *   synchronously; later calls allocate nothing and run on hip_stream.
 *   MG_E_UNSUPPORTED for a side above 4096 pixels. It overwrites the tree's
 *   bins and windows (not its panorama buffers). */
int mg_eval_interval(mg_tree tree, void* hip_stream, int32_t wd, int32_t hd, uint32_t* gain, int32_t* yaw_bin,
                     float* depth);

/* Merged overlap intervals the interval mode holds per ray (1..16; -1
 * restores the default 16). A ray whose union has more components is
 * evaluated in windows of that many (the ancestors' intervals are regenerated
 * for each window), so results do not depend on it; small values exercise
 * that path. Host only. */
int mg_interval_config(int32_t cap);

/* Host copy of the interval-mode camera for a sensor and voxel size (for
 * tests): wh[2] = (wd, hd) after the resolution rule, intr[6] = (fx, fy, cx,
 * cy, z_near, Rv), pdir [hd][wd][3] unit camera-frame pixel-centre
 * directions, cs [yaw_bins][2] cos and sin of each window's yaw. Pointers
 * other than wh may be NULL. */
int mg_interval_tables(const mg_sensor* sensor, float voxel_m, int32_t wd, int32_t hd, int32_t* wh, float* intr,
                       float* pdir, float* cs);

/* Exact marginal gain with voxel hash sets (eq. 2; the exact comparison of
 * Sec. V-A, there computed with hash maps on the CPU) at given windows:
 * yaw_bin DEVICE int32[n] (e.g. from mg_eval_marginal). I(n) is the set of
 * unknown voxels met by the rays of node n's window; outputs DEVICE
 * uint32[n]: x_ray = unknown incidences of those rays whose voxel is in no
 * ancestor's I (the per-incidence counterpart of the depth-buffer gain),
 * x_set = |I(n) minus the ancestors' I| (may be NULL), a_set = |I(n)| (may be
 * NULL). Synchronises hip_stream twice (windows checked on the host, tables
 * sized from a first pass) and may grow the tree's table pool (about 8 bytes
 * per unknown incidence of the windows). MG_E_INVALID for a window outside
 * [0, yaw_bins). */
int mg_eval_exact(mg_tree tree, void* hip_stream, const int32_t* yaw_bin, uint32_t* x_ray, uint32_t* x_set,
                  uint32_t* a_set);

/* Exact marginal gain with its own yaw choice (eq. 2 with the yaw choice of
 * Sec. III-B; the paper's exact planner gain, there computed with hash maps on
 * the CPU): nodes in depth order; node n's bin counts are the unknown
 * incidences of its panorama rays whose voxel lies in no ancestor's set I(a)
 * (each I(a) at a's own chosen window); the best window is chosen as for the
 * other evaluations and I(n) is then built at it. gain DEVICE uint32[n],
 * yaw_bin DEVICE int32[n]. Tables are sized from an absolute pass (one host
 * synchronisation; the pool may grow, about 8 bytes per unknown incidence of
 * each node's best absolute window); the call returns after the work. It
 * overwrites the tree's bins and window starts. */
int mg_eval_exact_marginal(mg_tree tree, void* hip_stream, uint32_t* gain, int32_t* yaw_bin);

/* Absolute gain of every node (eq. 1 maximised over the yaw windows), no
 * conditioning and no level order: one flat launch over all nodes.
 *   gain DEVICE uint32[n], yaw_bin DEVICE int32[n]. */
int mg_eval_absolute(mg_tree tree, void* hip_stream, uint32_t* gain, int32_t* yaw_bin);

/* ---------------------------------------------------------------- serving
 * Replanning requests from many robots (maps stay resident; each request is a
 * whole tree, Sec. IV-D), evaluated by a worker thread with continuous
 * batching: every step advances all in-flight requests by one depth level
 * (Sec. IV-C inside each request) in one trace launch plus one window launch,
 * so requests at different depths and on different maps share the GPU.
 * Requests are admitted between steps, first come first served, when fewer
 * than max_inflight are in flight and their tree fits in the server's device
 * arena (admission by device-memory footprint, mg_tree_footprint_bytes).
 * Results equal mg_eval_marginal on the same tree, alone or in any mix.
 * Each in-flight request has a device status word that its kernels check
 * first: a request marked failed (mg_server_fail_request) is skipped by them and
 * retired with its status at the end of the step, and a cancelled one
 * (mg_server_cancel) is dropped, while the other requests complete unchanged. */
typedef struct mg_server_s* mg_server;

typedef struct {
    mg_sensor sensor;          /* geometry and range of every request          */
    int32_t max_inflight;      /* requests advanced together, at most (>= 1)   */
    int64_t arena_bytes;       /* device memory for in-flight trees (>= 1)     */
} mg_server_config;

/* Allocates the arena (the only device allocation of the server) and starts
 * the worker thread on the current device. */
int mg_server_create(const mg_server_config* cfg, mg_server* out);

/* Queues a request: the marginal gain of the tree (pos_m [n][3] metres,
 * parent [n], HOST arrays, copied and validated here as in mg_tree_upload) on
 * `map`. Results go to the HOST arrays gain [n] and yaw_bin [n], which must
 * stay valid until the request is reported done. MG_E_INVALID for a bad tree,
 * MG_E_NOMEM when the tree can never fit in the arena. *ticket identifies the
 * request. Thread-safe. */
int mg_server_submit(mg_server server, mg_map map, const float* pos_m, const int32_t* parent, int32_t n,
                     uint32_t* gain, int32_t* yaw_bin, int64_t* ticket);

/* Queues a map update between replans: voxel_ids HOST uint32 [count] (linear
 * ids x + nx (y + ny z), distinct), states HOST uint8 [count] in {0, 1, 2};
 * both copied. The update is applied once every request on `map` submitted
 * before it has finished (none is queued ahead of it or in flight), so those
 * requests see the old map; requests on `map` submitted after it wait for it
 * and see the new one, while requests on other maps are not held back by it.
 * *ticket works with
 * mg_server_poll / mg_server_wait like a request's. MG_E_INVALID for an id
 * outside the grid or a larger state. Thread-safe. */
int mg_server_map_update(mg_server server, mg_map map, const uint32_t* voxel_ids, const uint8_t* states,
                         int32_t count, int64_t* ticket);

/* Non-blocking: *status = 0 while pending, 1 when done, or the request's
 * negative error code. Once reported done (or failed) the ticket is retired;
 * latency_us (may be NULL) receives submit-to-result time in microseconds. */
int mg_server_poll(mg_server server, int64_t ticket, int32_t* status, double* latency_us);

/* Blocks until the request is done; returns its status and retires the ticket. */
int mg_server_wait(mg_server server, int64_t ticket, double* latency_us);

/* Cancels a request or a queued map update. A queued one is dropped at once;
 * an in-flight request at the next step boundary (the device work done for it
 * is discarded and its arena block released). It then reports
 * MG_E_CANCELLED through mg_server_poll / mg_server_wait and its output arrays
 * are not written. MG_E_INVALID for an unknown ticket, MG_E_BUSY when the
 * request has already finished or the update is being applied. Thread-safe. */
int mg_server_cancel(mg_server server, int64_t ticket);

/* Marks a request failed with `code` (a negative MG_E_* value) through its
 * device status word, as a kernel that detects an error in that request's
 * data does: the request's remaining kernels skip it, and at the end of the
 * step that reads the word the request is retired with `code` (its outputs not
 * written) while every other request continues and completes unchanged. A
 * queued request is marked when it is admitted. For callers and tests that
 * need a request to fail in isolation. MG_E_INVALID for an unknown ticket, a
 * map update or code >= 0; MG_E_BUSY when the request has already finished.
 * Thread-safe. */
int mg_server_fail_request(mg_server server, int64_t ticket, int32_t code);

/* paused = 1: no step runs after the current one; requests are still admitted
 * into flight (up to max_inflight and the arena), map updates wait. paused = 0
 * resumes. MG_E_INVALID for another value. Thread-safe. */
int mg_server_pause(mg_server server, int32_t paused);

/* Counters: steps run, requests completed, rays evaluated, requests in flight and queued. */
int mg_server_stats(mg_server server, int64_t* steps, int64_t* completed, double* rays, int32_t* in_flight,
                    int32_t* queued);

/* Finishes every queued and in-flight request, stops the worker, frees the arena. */
int mg_server_destroy(mg_server server);

/* ---------------------------------------------------------------- timing
 * Measurement of the dominant kernels (the trace kernel and the path-mask
 * builder of mg_eval_marginal_batch). While enabled (on != 0), every trace
 * and builder launch that mg_eval_marginal_batch makes on the current device
 * carries a pair of HIP events recorded by the kernel dispatch itself, so the
 * interval is the kernel's own execution (while enabled, batch plans are
 * launched one by one instead of replaying their graph). Enabling binds the
 * timer to the current device; MG_E_BUSY if unread launches of another device
 * remain. Process-wide. */
int mg_timing_enable(int32_t on);

/* Waits for the timed launches since the last read, returns the sum of their
 * durations (ms), the union of their intervals (ms during which at least one
 * ran: launches of different groups of a batch plan overlap), their number
 * and the workgroups the trace launches ran (any pointer may be NULL), and
 * resets the sums.
 * At most 65536 launches may be timed between two reads (MG_E_BUSY from the
 * launch call beyond that). */
int mg_timing_read(double* total_ms, double* busy_ms, int64_t* launches, int64_t* workgroups);

/* Host-only diagnostics: the sensor tables the library builds (no device
 * work). dir and inv [n_az*n_el][3] (ray r = c*n_el + j), bv [n_az][2]
 * (column left-boundary unit vectors), ts [n_el+1] (tan(e)|tan(e)| at row
 * boundaries), bins [n_az], c0 [yaw_bins]. Any pointer may be NULL. */
int mg_sensor_tables(const mg_sensor* sensor, float* dir, float* inv, float* bv, float* ts,
                     int32_t* bins, int32_t* c0);

/* Message of the last failed call on this thread ("" if none). */
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
