/*
 * mgref — the ORACLE for path-dependent marginal information gain.
 *
 * TEST INFRASTRUCTURE ONLY. Plain, serial, deliberately slow C that computes
 * what the GPU library must reproduce. Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it. It shares no source,
 * header, table generator or helper with the GPU library.
 *
 * What it computes (paper: "GPU-Accelerated Path-Dependent Marginal
 * Information Gain for Autonomous Exploration"):
 *   - absolute gain per candidate yaw window, eq. (1), maximised over yaw
 *     (Sec. III-B);
 *   - the depth-buffer marginal gain: each unknown voxel met by a node's rays
 *     is dropped when an ancestor's first-hit depth buffer already sees it
 *     (Sec. IV-A, IV-B, with the per-voxel, equiangular reading below), the
 *     yaw window is maximised and the node's own buffer is stored
 *     (Sec. IV-A, last sentence) for its descendants, level by level
 *     (Sec. IV-C);
 *   - the exact set-difference marginal gain of eq. (2) with per-node sorted
 *     voxel sets (the paper's hash-map baseline, Sec. IV-E).
 *
 * Precision: all geometry is IEEE binary32 in the operation order written
 * here (build with -ffp-contract=off, no fast-math). The paper does not fix a
 * precision; float is the precision the GPU path decides in, so the integer
 * results (counts, yaw bins) are decided in the same precision on both sides.
 * Trigonometry happens only in the sensor tables, in double, rounded once.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - gains count ray incidences (a voxel crossed by k rays counts k);
 *   - yaw candidates are B azimuth bins; a window of w = B*fov_h/360 bins
 *     covers the W_buf panorama columns whose centres fall in it;
 *   - a depth buffer stores the DDA parameter t of the first occupied voxel
 *     (or the range limit) for the window's rays, and a voxel is "observed"
 *     by ancestor a when its centre falls in one of a's pixel cells and its
 *     squared range from a is <= the squared stored depth (comparison "<=",
 *     Sec. IV-B).
 */
#ifndef MGREF_H
#define MGREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_az;          /* panorama columns over 360 degrees            */
    int32_t n_el;          /* rows over fov_v_deg                          */
    float fov_h_deg;       /* horizontal field of view of one yaw window   */
    float fov_v_deg;       /* vertical field of view                       */
    float range_m;         /* maximum sensing range                        */
    int32_t yaw_bins;      /* B azimuth bins                               */
    float az_offset_deg;   /* azimuth of column 0's left boundary          */
} mgref_sensor_params;

typedef struct {
    uint64_t visits;       /* V: voxels visited by the DDA                 */
    uint64_t unk_visits;   /* U: unknown voxels visited                    */
    uint64_t anc_tests;    /* T: ancestor tests, parent first, early exit  */
} mgref_counters;

/* Host sensor tables. Ray index r = c*n_el + j (column c, row j). */
typedef struct {
    mgref_sensor_params p;
    int32_t win_bins, w_buf;
    float *dir;     /* [n_az*n_el*3]  unit directions                  */
    float *inv;     /* [n_az*n_el*3]  1.0f/dir (0 where dir == 0)      */
    float *bvx;     /* [n_az] column left-boundary unit vectors        */
    float *bvy;
    float *ts;      /* [n_el+1] tan(e)*|tan(e)| at row boundaries      */
    int32_t *bin_of_col;  /* [n_az]    */
    int32_t *c0_of_win;   /* [yaw_bins] */
} mgref_sensor;

/* Returns 0, or -1 when the sensor is not representable (see mgref.c). */
int mgref_sensor_init(const mgref_sensor_params* p, mgref_sensor* out);
void mgref_sensor_free(mgref_sensor* s);

/* Copy of the tables, for tests: dir/inv [n_az*n_el*3], bv [n_az*2], ts [n_el+1],
 * bins [n_az], c0 [yaw_bins]. Any pointer may be NULL. */
int mgref_sensor_tables(const mgref_sensor_params* p, float* dir, float* inv, float* bv,
                        float* ts, int32_t* bins, int32_t* c0);

/* One ray: lists the visited voxels (linear ids x + nx*(y + ny*z)) with their
 * states and entry parameters t, in traversal order; returns the visit count
 * (or -1 if cap is too small). *h receives the first-hit t (or Rv). */
int mgref_trace_ray(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                    const float q[3], const float d[3], const float inv[3], float rv,
                    int32_t cap, uint32_t* ids, uint8_t* st, float* tenter, float* h);

/* The same traversal; texit[v] (if not NULL) also receives the parameter at
 * which visit v's voxel is left: the next voxel's entry, which may lie at or
 * beyond Rv or outside the grid (for an occupied voxel, its own entry). */
int mgref_trace_ray_exit(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                         const float q[3], const float d[3], const float inv[3], float rv,
                         int32_t cap, uint32_t* ids, uint8_t* st, float* tenter, float* texit, float* h);

/* obs(a, x) for the voxel (ix,iy,iz): 1 when ancestor a (position qa in
 * voxel units, window start column c0a, buffer Da[n_el][w_buf]) observes it. */
int mgref_obs(const mgref_sensor* s, const float qa[3], int32_t c0a, const float* Da,
              int32_t ix, int32_t iy, int32_t iz, int32_t* row, int32_t* col);

/* One node on its own: traverses all panorama rays from q (voxel units) and
 * accumulates abs_bins / marg_bins [B] (not cleared), conditioning on n_anc
 * ancestors given explicitly, nearest first: anc_q [n_anc][3], anc_c0
 * [n_anc], anc_D [n_anc][n_el][w_buf]. h [n_az*n_el] receives first hits.
 * Returns 0 or -1. */
int mgref_eval_node(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                    const mgref_sensor_params* sp, float rv, const float q[3], int32_t n_anc,
                    const float* anc_q, const int32_t* anc_c0, const float* anc_D,
                    uint32_t* abs_bins, uint32_t* marg_bins, float* h, mgref_counters* cnt);

/* I(n) for a node at window k: sorted distinct ids of the unknown voxels met by
 * the window's rays. Returns the count, or -1 when cap is too small. */
int64_t mgref_node_set(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                       const mgref_sensor_params* sp, float rv, const float q[3], int32_t k,
                       int64_t cap, uint32_t* ids_out);

/* Window selection over B bins: returns the maximum window sum, *k = smallest maximiser. */
uint32_t mgref_best_window(const uint32_t* bins, int32_t B, int32_t w, int32_t* k);

/* Whole-tree evaluation in depth order.
 *   max_anc: -1 all ancestors (marginal), 0 none (absolute), m>0 the m nearest.
 *   mask: NULL, or an ancestor-closed subset of nodes to evaluate (others are
 *         left untouched in the outputs).
 *   abs_bins / marg_bins: [n][B] or NULL; D: [n][n_el][w_buf] (required).
 *   n_threads: worker threads over the nodes of one level (results do not
 *   depend on it). Returns 0, or -1 on invalid input. */
int mgref_eval_tree(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                    const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                    const mgref_sensor_params* sp, int32_t max_anc, const uint8_t* mask,
                    uint32_t* g_abs, int32_t* k_abs, uint32_t* g_db, int32_t* k_db, float* D,
                    uint32_t* abs_bins, uint32_t* marg_bins, mgref_counters* cnt,
                    int32_t n_threads);

/* Exact quantities at the yaw windows k_db (eq. 2; fixed-yaw protocol of Sec. V-A):
 *   A_set = |I(n)|, X_set = |I(n) \ U_a I(a)|,
 *   X_ray = sum over window rays of #{incidences not in U_a I(a)},
 *   G_db_set = #{x in I(n) : not observed through the ancestors' buffers D}.
 * mask as above. Returns 0 or -1. */
int mgref_exact(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                const mgref_sensor_params* sp, const int32_t* k_db, const float* D,
                const uint8_t* mask, uint32_t* A_set, uint32_t* X_set, uint32_t* X_ray,
                uint32_t* G_db_set);

/* Exact marginal gain with its own yaw choice (eq. 2, Sec. III-B): depth
 * order; a node's per-bin counts are the incidences of its panorama rays whose
 * unknown voxel lies in no ancestor's I (each taken at that ancestor's chosen
 * window); gain/k as for the other evaluations; I(n) is then built at the
 * chosen window. mask as above. Returns 0 or -1. */
int mgref_exact_marginal(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                         const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                         const mgref_sensor_params* sp, const uint8_t* mask, uint32_t* gain, int32_t* k_out);

#ifdef __cplusplus
}
#endif
#endif
