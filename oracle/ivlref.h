/*
 * ivlref — the ORACLE of the interval mode (test infrastructure only).
 *
 * TEST INFRASTRUCTURE ONLY, like mgref.h: plain serial C that computes what
 * the GPU library's interval mode must reproduce bit for bit. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * The interval mode follows the paper's own conditioning (Sec. IV-A, IV-B):
 *   - every node keeps a pinhole depth buffer of W_D x H_D pixels at its
 *     chosen yaw, sized so that one pixel at the maximum range spans one
 *     voxel, W_D = ceil(2 d_max tan(fov_h/2) / v), H_D likewise with fov_v;
 *     a pixel holds the camera-frame z of the first occupied voxel on the ray
 *     through its centre, or of the ray's end at the range limit;
 *   - a candidate ray r(t) = q_n + t d, 0 <= t <= Rv (the maximum range in
 *     voxel units), is moved into each ancestor's camera frame, clipped to
 *     the valid depth range z_near <= z <= Rv, projected with eq. (5),
 *     clipped to the buffer with the Liang-Barsky algorithm and walked pixel
 *     by pixel with a 2D DDA; inverse depth is interpolated linearly in
 *     screen space (eq. 6), and the part of each pixel's span where z <= the
 *     stored depth is observed: its two ends, mapped back to t, are an
 *     overlap interval (eq. 7), joined to the previous one of the same
 *     ancestor when it starts at or before that one's end;
 *   - the ancestors' intervals are merged one ancestor after another, and the
 *     3D DDA counts an unknown voxel unless the midpoint of its chord lies in
 *     a merged interval.
 * Candidate rays, yaw windows, counting and window selection are those of
 * mgref.h (panorama rays, B bins, ray incidences).
 *
 * Camera frame of yaw psi: x right = (sin psi, -cos psi, 0), y down =
 * (0, 0, -1), z forward = (cos psi, sin psi, 0); world axes in voxel units.
 * The yaw of window k is az_offset + (k + w/2) * 360 / B degrees (the centre
 * of the window's azimuth span).
 */
#ifndef IVLREF_H
#define IVLREF_H
#include <stdint.h>

#include "mgref.h"
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t wd, hd;        /* buffer width and height in pixels                */
    int32_t B, w;          /* yaw bins, window bins                            */
    float fx, fy, cx, cy;  /* intrinsics of eq. (5), pixels                   */
    float znear;           /* near end of the valid depth range (voxel units) */
    float rv;              /* range limit (voxel units)                        */
    float* pdir;           /* [hd*wd*3] unit camera-frame direction of pixel centres, index j*wd + i */
    float* cs;             /* [B*2] cos, sin of the yaw of window k            */
} ivlref_camera;

typedef struct {
    uint64_t visits;       /* voxels visited by the 3D DDA                     */
    uint64_t unk_visits;   /* unknown voxels visited                           */
    uint64_t pixel_steps;  /* pixels visited by the 2D DDAs                    */
    uint64_t intervals;    /* merged intervals, summed over rays               */
    uint64_t max_merged;   /* most merged intervals on one ray                 */
} ivlref_counters;

/* Buffer size by the resolution rule (wd, hd <= 0) or as given; tables in
 * double, rounded once. Returns 0, or -1 for an invalid sensor or a size
 * outside 1..4096 per side. */
int ivlref_camera_init(const mgref_sensor_params* sp, float voxel_m, int32_t wd, int32_t hd, ivlref_camera* cam);
void ivlref_camera_free(ivlref_camera* cam);

/* Copy of the camera: wh[2] = (wd, hd), intr[6] = (fx, fy, cx, cy, znear, rv),
 * pdir [hd*wd*3], cs [B*2]. Pointers other than wh may be NULL. */
int ivlref_camera_tables(const mgref_sensor_params* sp, float voxel_m, int32_t wd, int32_t hd, int32_t* wh,
                         float* intr, float* pdir, float* cs);

/* Depth buffer D [hd*wd] of a viewpoint at q (voxel units) with window k. */
int ivlref_render(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, const ivlref_camera* cam,
                  const float q[3], int32_t k, float* D);

/* Overlap intervals of one ancestor (position qa, window ka, buffer Da) on
 * the candidate ray from qn along the unit direction d, 0 <= t <= Rv: up to
 * cap intervals [lo, hi] in t (voxel units), in the order found, touching
 * ones joined, written to out[2*i], out[2*i+1]. Returns their number (which
 * may exceed cap: only the first cap are written). *steps (may be NULL)
 * receives the pixels visited. */
int32_t ivlref_intervals(const ivlref_camera* cam, const float qn[3], const float d[3], const float qa[3],
                         int32_t ka, const float* Da, float* out, int32_t cap, uint64_t* steps);

/* Union of two sorted lists of disjoint intervals M [m][2] and S [ns][2] into
 * out [m + ns][2], sorted, overlapping or touching intervals joined. Returns
 * the count. */
int32_t ivlref_merge(const float* M, int32_t m, const float* S, int32_t ns, float* out);

/* Whole tree, depth order, marginal gain in the interval mode. Outputs as
 * mgref_eval_tree (g_abs/k_abs/abs_bins/marg_bins may be NULL), D [n][hd][wd].
 * Returns 0 or -1. */
int ivlref_eval_tree(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                     const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                     const mgref_sensor_params* sp, int32_t wd, int32_t hd, const uint8_t* mask,
                     uint32_t* g_abs, int32_t* k_abs, uint32_t* g_db, int32_t* k_db, float* D,
                     uint32_t* abs_bins, uint32_t* marg_bins, ivlref_counters* cnt, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
