/*
 * ivlref.c — the ORACLE of the interval mode (test infrastructure only; see
 * ivlref.h). Built into libmgref.so with mgref.c (same flags: -O2
 * -ffp-contract=off, no fast-math). Geometry is IEEE binary32 in the order
 * written; the camera tables are computed in double and rounded once.
 */
#define _GNU_SOURCE
#include "ivlref.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

enum { S_UNK = 0, S_FREE = 1, S_OCC = 2 };

static double snap(double x) { return fabs(x) < 1e-9 ? 0.0 : x; }

/* ------------------------------------------------------------------ camera (Sec. IV-A, eq. 5) */

/* The buffer resolution rule of Sec. IV-A: one pixel at the maximum range
 * spans one voxel, W_D = ceil(2 d_max tan(fov_h/2) / v) and
 * H_D = ceil(2 d_max tan(fov_v/2) / v). The pinhole has its principal point
 * at the buffer centre and focal lengths that make the buffer span the field
 * of view: f_x = (W_D/2) / tan(fov_h/2), f_y = (H_D/2) / tan(fov_v/2). */
int ivlref_camera_init(const mgref_sensor_params* sp, float voxel_m, int32_t wd, int32_t hd, ivlref_camera* cam) {
    memset(cam, 0, sizeof(*cam));
    mgref_sensor s;
    if (!(voxel_m > 0.0f) || mgref_sensor_init(sp, &s) != 0) return -1;
    const int32_t w = s.win_bins;
    mgref_sensor_free(&s);
    const double deg = M_PI / 180.0;
    const double th = tan((double)sp->fov_h_deg * 0.5 * deg);
    const double tv = tan((double)sp->fov_v_deg * 0.5 * deg);
    if (wd <= 0) {
        double x = ceil(2.0 * (double)sp->range_m * th / (double)voxel_m);
        if (!(x >= 1.0 && x <= 4096.0)) return -1;
        wd = (int32_t)x;
    }
    if (hd <= 0) {
        double x = ceil(2.0 * (double)sp->range_m * tv / (double)voxel_m);
        if (!(x >= 1.0 && x <= 4096.0)) return -1;
        hd = (int32_t)x;
    }
    if (wd < 1 || wd > 4096 || hd < 1 || hd > 4096) return -1;
    const double cxd = (double)wd * 0.5, cyd = (double)hd * 0.5;
    const double fxd = cxd / th, fyd = cyd / tv;
    cam->wd = wd;
    cam->hd = hd;
    cam->B = sp->yaw_bins;
    cam->w = w;
    cam->fx = (float)fxd;
    cam->fy = (float)fyd;
    cam->cx = (float)cxd;
    cam->cy = (float)cyd;
    cam->znear = 1.0f / 64.0f;
    cam->rv = sp->range_m / voxel_m;
    cam->pdir = (float*)malloc(sizeof(float) * 3 * (size_t)wd * (size_t)hd);
    cam->cs = (float*)malloc(sizeof(float) * 2 * (size_t)cam->B);
    if (!cam->pdir || !cam->cs) {
        ivlref_camera_free(cam);
        return -1;
    }
    for (int32_t j = 0; j < hd; ++j)
        for (int32_t i = 0; i < wd; ++i) {
            double x = ((double)i + 0.5 - cxd) / fxd, y = ((double)j + 0.5 - cyd) / fyd;
            double nrm = sqrt(x * x + y * y + 1.0);
            float* p = cam->pdir + 3 * ((size_t)j * wd + i);
            p[0] = (float)snap(x / nrm);
            p[1] = (float)snap(y / nrm);
            p[2] = (float)(1.0 / nrm);
        }
    for (int32_t k = 0; k < cam->B; ++k) {
        double psi = ((double)sp->az_offset_deg + ((double)k + 0.5 * (double)w) * 360.0 / (double)cam->B) * deg;
        cam->cs[2 * k] = (float)snap(cos(psi));
        cam->cs[2 * k + 1] = (float)snap(sin(psi));
    }
    return 0;
}

void ivlref_camera_free(ivlref_camera* cam) {
    free(cam->pdir);
    free(cam->cs);
    memset(cam, 0, sizeof(*cam));
}

int ivlref_camera_tables(const mgref_sensor_params* sp, float voxel_m, int32_t wd, int32_t hd, int32_t* wh,
                         float* intr, float* pdir, float* cs) {
    ivlref_camera cam;
    if (ivlref_camera_init(sp, voxel_m, wd, hd, &cam) != 0) return -1;
    wh[0] = cam.wd;
    wh[1] = cam.hd;
    if (intr) {
        intr[0] = cam.fx; intr[1] = cam.fy; intr[2] = cam.cx; intr[3] = cam.cy;
        intr[4] = cam.znear; intr[5] = cam.rv;
    }
    if (pdir) memcpy(pdir, cam.pdir, sizeof(float) * 3 * (size_t)cam.wd * cam.hd);
    if (cs) memcpy(cs, cam.cs, sizeof(float) * 2 * (size_t)cam.B);
    ivlref_camera_free(&cam);
    return 0;
}

/* ------------------------------------------------------------------ depth buffer (Sec. IV-A) */

/* Pixel (i, j) looks along its centre's camera direction p, which in the
 * world is p_x * right + p_y * down + p_z * forward for the window's yaw.
 * The 3D DDA gives the first occupied voxel's entry t (or Rv); the pixel
 * stores the camera-frame z of that point, t * p_z. */
int ivlref_render(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, const ivlref_camera* cam,
                  const float q[3], int32_t k, float* D) {
    const float c = cam->cs[2 * k], s = cam->cs[2 * k + 1];
    const int32_t cap = 3 * (int32_t)ceilf(cam->rv) + 16;
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    int rc = (ids && st && te) ? 0 : -1;
    for (int32_t px = 0; px < cam->wd * cam->hd && rc == 0; ++px) {
        const float* p = cam->pdir + 3 * (size_t)px;
        float wdir[3] = {s * p[0] + c * p[2], s * p[2] - c * p[0], -p[1]};
        float inv[3];
        for (int a = 0; a < 3; ++a) inv[a] = wdir[a] != 0.0f ? 1.0f / wdir[a] : 0.0f;
        float h;
        if (mgref_trace_ray(states, nx, ny, nz, q, wdir, inv, cam->rv, cap, ids, st, te, &h) < 0) rc = -1;
        D[px] = h * p[2];
    }
    free(ids); free(st); free(te);
    return rc;
}

/* ------------------------------------------------------------------ overlap intervals (eq. 5-7) */

typedef struct {
    float tlo, thi, wa, wb;
} segment;

/* Ray parameter t of screen parameter s on the projected segment: the point
 * at s has inverse depth w(s) = (1 - s) w_A + s w_B (eq. 6); its fraction of
 * the 3D segment is s w_B / w(s) (perspective-correct), so
 * t = t_lo + (s w_B / w(s)) (t_hi - t_lo). */
static float t_of_s(const segment* g, float s) {
    float lam = (s * g->wb) / ((1.0f - s) * g->wa + s * g->wb);
    return g->tlo + lam * (g->thi - g->tlo);
}

/* One ancestor's overlap intervals in t, in the order the 2D DDA finds them:
 * an interval that starts at or before the end of the open one is joined to
 * it, otherwise the open one is written out and the new one opened. */
typedef struct {
    float* out;
    int32_t cap, n;
    float lo, hi;            /* the open interval, in t */
} ivl_list;

static void ivl_emit(ivl_list* L) {
    if (L->n > 0 && L->n - 1 < L->cap) {
        L->out[2 * (L->n - 1)] = L->lo;
        L->out[2 * (L->n - 1) + 1] = L->hi;
    }
}

static void ivl_push(ivl_list* L, float lo, float hi) {
    if (L->n > 0 && lo <= L->hi) {
        if (hi > L->hi) L->hi = hi;
        return;
    }
    ivl_emit(L);
    L->lo = lo;
    L->hi = hi;
    L->n++;
}

int32_t ivlref_intervals(const ivlref_camera* cam, const float qn[3], const float d[3], const float qa[3],
                         int32_t ka, const float* Da, float* out, int32_t cap, uint64_t* steps) {
    const float c = cam->cs[2 * ka], s = cam->cs[2 * ka + 1];
    const int32_t wd = cam->wd, hd = cam->hd;
    segment g;
    ivl_list L = {out, cap, 0, 0.0f, 0.0f};
    if (steps) *steps = 0;
    /* the ray's origin and direction in the ancestor's camera frame */
    const float o[3] = {qn[0] - qa[0], qn[1] - qa[1], qn[2] - qa[2]};
    const float P0[3] = {s * o[0] - c * o[1], -o[2], c * o[0] + s * o[1]};
    const float Dc[3] = {s * d[0] - c * d[1], -d[2], c * d[0] + s * d[1]};
    /* the ray r(t), 0 <= t <= Rv (Sec. IV-B), clipped to the valid depth range
     * znear <= z <= Rv; z is linear in t */
    if (Dc[2] == 0.0f) {
        if (!(P0[2] >= cam->znear && P0[2] <= cam->rv)) return 0;
        g.tlo = 0.0f;
        g.thi = cam->rv;
    } else {
        float t1 = (cam->znear - P0[2]) / Dc[2], t2 = (cam->rv - P0[2]) / Dc[2];
        float a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
        g.tlo = a > 0.0f ? a : 0.0f;
        g.thi = b < cam->rv ? b : cam->rv;
    }
    if (!(g.tlo < g.thi)) return 0;
    float A[3], Bp[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = P0[k] + g.tlo * Dc[k];
        Bp[k] = P0[k] + g.thi * Dc[k];
    }
    if (!(A[2] > 0.0f && Bp[2] > 0.0f)) return 0;
    /* eq. (5) at both ends; inverse depths for eq. (6) */
    const float uA = cam->fx * A[0] / A[2] + cam->cx, vA = cam->fy * A[1] / A[2] + cam->cy;
    const float uB = cam->fx * Bp[0] / Bp[2] + cam->cx, vB = cam->fy * Bp[1] / Bp[2] + cam->cy;
    g.wa = 1.0f / A[2];
    g.wb = 1.0f / Bp[2];
    /* Liang-Barsky: clip the screen segment to 0 <= u <= W_D, 0 <= v <= H_D */
    const float du = uB - uA, dv = vB - vA;
    const float pp[4] = {-du, du, -dv, dv};
    const float qq[4] = {uA, (float)wd - uA, vA, (float)hd - vA};
    float s0 = 0.0f, s1 = 1.0f;
    for (int e = 0; e < 4; ++e) {
        if (pp[e] == 0.0f) {
            if (qq[e] < 0.0f) return 0;
            continue;
        }
        float r = qq[e] / pp[e];
        if (pp[e] < 0.0f) {
            if (r > s0) s0 = r;
        } else {
            if (r < s1) s1 = r;
        }
    }
    if (!(s0 < s1)) return 0;
    /* 2D DDA over the pixels of the clipped segment; boundary crossings are
     * recomputed from the integer boundary, s = (b - u_A) * (1/du); ties step u first */
    const float u0 = uA + s0 * du, v0 = vA + s0 * dv;
    int32_t i = (int32_t)floorf(u0), j = (int32_t)floorf(v0);
    i = i < 0 ? 0 : (i > wd - 1 ? wd - 1 : i);
    j = j < 0 ? 0 : (j > hd - 1 ? hd - 1 : j);
    const int32_t si = du > 0.0f ? 1 : (du < 0.0f ? -1 : 0);
    const int32_t sj = dv > 0.0f ? 1 : (dv < 0.0f ? -1 : 0);
    const float iu = si ? 1.0f / du : 0.0f, iv = sj ? 1.0f / dv : 0.0f;
    int32_t bu = si > 0 ? i + 1 : i, bv = sj > 0 ? j + 1 : j;
    float su = si ? ((float)bu - uA) * iu : INFINITY;
    float sv = sj ? ((float)bv - vA) * iv : INFINITY;
    float sa = s0;
    uint64_t n_steps = 0;
    for (int32_t it = 0; it < wd + hd + 2; ++it) {
        float e = su < sv ? su : sv;
        e = e < s1 ? e : s1;
        ++n_steps;
        /* the part of [sa, e] where z(s) <= D, i.e. w(s) >= 1/D (w is linear in s) */
        const float Dp = Da[(size_t)j * wd + i];
        if (Dp > 0.0f) {
            const float wD = 1.0f / Dp;
            float lo = sa, hi = e;
            int ok = 1;
            if (g.wb == g.wa) {
                ok = g.wa >= wD;
            } else {
                const float ss = (wD - g.wa) / (g.wb - g.wa);
                if (g.wb > g.wa) lo = sa > ss ? sa : ss;
                else hi = e < ss ? e : ss;
            }
            if (ok && lo <= hi) ivl_push(&L, t_of_s(&g, lo), t_of_s(&g, hi));
        }
        if (!(e < s1)) break;
        if (su <= sv) {
            i += si;
            bu += si;
            su = ((float)bu - uA) * iu;
        } else {
            j += sj;
            bv += sj;
            sv = ((float)bv - vA) * iv;
        }
        sa = e;
        if (i < 0 || i >= wd || j < 0 || j >= hd) break;
    }
    ivl_emit(&L);
    if (steps) *steps = n_steps;
    return L.n;
}

/* ------------------------------------------------------------------ merging (eq. 7, last sentence) */

/* Union of the sorted, disjoint lists M [m] and S [ns] into out, in order of
 * the lower ends; an interval starting at or before the end of the previous
 * one is joined to it. Returns the merged count. */
int32_t ivlref_merge(const float* M, int32_t m, const float* S, int32_t ns, float* out) {
    int32_t a = 0, b = 0, n = 0;
    while (a < m || b < ns) {
        const float* x;
        if (b >= ns || (a < m && M[2 * a] <= S[2 * b])) x = M + 2 * a++;
        else x = S + 2 * b++;
        if (n > 0 && x[0] <= out[2 * n - 1]) {
            if (x[1] > out[2 * n - 1]) out[2 * n - 1] = x[1];
        } else {
            out[2 * n] = x[0];
            out[2 * n + 1] = x[1];
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ tree driver (Sec. IV-B, IV-C) */

typedef struct {
    const uint8_t* states;
    int32_t nx, ny, nz;
    const mgref_sensor* s;
    const ivlref_camera* cam;
    const float* q;
    const int32_t* parent;
    int32_t *k_db, *k_abs;
    uint32_t *g_db, *g_abs;
    uint32_t *abs_bins, *marg_bins;
    float* D;
    const int32_t* nodes;
    int32_t count, next;
    pthread_mutex_t lock;
    ivlref_counters total;
    int failed;
} ivl_job;

typedef struct {
    float *M, *tmp, *S;
    int32_t cap;             /* capacity of M, tmp and S in intervals */
} ivl_work;

static int grow(ivl_work* W, int32_t need) {
    if (need <= W->cap) return 0;
    int32_t cap = W->cap;
    while (cap < need) cap *= 2;
    float* a = (float*)realloc(W->M, sizeof(float) * 2 * cap);
    if (!a) return -1;
    W->M = a;
    a = (float*)realloc(W->tmp, sizeof(float) * 2 * cap);
    if (!a) return -1;
    W->tmp = a;
    a = (float*)realloc(W->S, sizeof(float) * 2 * cap);
    if (!a) return -1;
    W->S = a;
    W->cap = cap;
    return 0;
}

/* One node: for every panorama ray, the merged overlap intervals of its
 * ancestors (nearest first), then the 3D DDA: each unknown voxel counts
 * towards the absolute bin of the ray's column and, unless the midpoint of
 * its chord [t_enter, min(t_exit, Rv)] lies in a merged interval, towards the
 * marginal bin. Then both windows are chosen and the node's buffer is
 * rendered at the marginal window's yaw. */
static int eval_node(ivl_job* J, int32_t n, ivl_work* W, uint32_t* ids, uint8_t* st, float* te, float* tx,
                     int32_t cap, ivlref_counters* cnt) {
    const mgref_sensor* s = J->s;
    const ivlref_camera* cam = J->cam;
    const int Wp = s->p.n_az, H = s->p.n_el, B = s->p.yaw_bins;
    const size_t npx = (size_t)cam->wd * cam->hd;
    uint32_t* ab = (uint32_t*)calloc(B, sizeof(uint32_t));
    uint32_t* mb = (uint32_t*)calloc(B, sizeof(uint32_t));
    int32_t anc[65];
    int32_t na = 0;
    int rc = (ab && mb) ? 0 : -1;
    for (int32_t a = J->parent[n]; a >= 0 && na < 65; a = J->parent[a]) anc[na++] = a;
    const float* qn = J->q + 3 * n;
    for (int c = 0; c < Wp && rc == 0; ++c) {
        const int b = s->bin_of_col[c];
        for (int j = 0; j < H && rc == 0; ++j) {
            const int r = c * H + j;
            const float* d = s->dir + 3 * r;
            int32_t m = 0;
            for (int32_t k = 0; k < na && rc == 0; ++k) {
                const int32_t a = anc[k];
                uint64_t steps = 0;
                int32_t ns = ivlref_intervals(cam, qn, d, J->q + 3 * a, J->k_db[a], J->D + (size_t)a * npx, W->S,
                                              W->cap, &steps);
                if (ns > W->cap) {
                    if (grow(W, ns) != 0) { rc = -1; break; }
                    ns = ivlref_intervals(cam, qn, d, J->q + 3 * a, J->k_db[a], J->D + (size_t)a * npx, W->S,
                                          W->cap, &steps);
                }
                cnt->pixel_steps += steps;
                if (grow(W, m + ns) != 0) { rc = -1; break; }
                m = ivlref_merge(W->M, m, W->S, ns, W->tmp);
                float* t = W->M; W->M = W->tmp; W->tmp = t;
            }
            if (rc != 0) break;
            cnt->intervals += (uint64_t)m;
            if ((uint64_t)m > cnt->max_merged) cnt->max_merged = (uint64_t)m;
            float h;
            int nv = mgref_trace_ray_exit(J->states, J->nx, J->ny, J->nz, qn, d, s->inv + 3 * r, cam->rv, cap, ids,
                                          st, te, tx, &h);
            if (nv < 0) { rc = -1; break; }
            cnt->visits += (uint64_t)nv;
            for (int v = 0; v < nv; ++v) {
                if (st[v] != S_UNK) continue;
                cnt->unk_visits++;
                ab[b]++;
                const float tex = tx[v] < cam->rv ? tx[v] : cam->rv;
                const float tm = 0.5f * (te[v] + tex);
                int covered = 0;
                for (int32_t k = 0; k < m && !covered; ++k) covered = W->M[2 * k] <= tm && tm <= W->M[2 * k + 1];
                if (!covered) mb[b]++;
            }
        }
    }
    if (rc == 0) {
        int32_t ka, km;
        uint32_t ga = mgref_best_window(ab, B, s->win_bins, &ka);
        uint32_t gm = mgref_best_window(mb, B, s->win_bins, &km);
        if (J->g_abs) J->g_abs[n] = ga;
        if (J->k_abs) J->k_abs[n] = ka;
        J->g_db[n] = gm;
        J->k_db[n] = km;
        if (J->abs_bins) memcpy(J->abs_bins + (size_t)n * B, ab, sizeof(uint32_t) * B);
        if (J->marg_bins) memcpy(J->marg_bins + (size_t)n * B, mb, sizeof(uint32_t) * B);
        rc = ivlref_render(J->states, J->nx, J->ny, J->nz, cam, qn, km, J->D + (size_t)n * npx);
    }
    free(ab);
    free(mb);
    return rc;
}

static void* level_worker(void* arg) {
    ivl_job* J = (ivl_job*)arg;
    const int32_t cap = 3 * (int32_t)ceilf(J->cam->rv) + 16;
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    float* tx = (float*)malloc(sizeof(float) * cap);
    ivl_work W = {NULL, NULL, NULL, 0};
    ivlref_counters cnt;
    memset(&cnt, 0, sizeof(cnt));
    W.cap = 16;
    W.M = (float*)malloc(sizeof(float) * 2 * W.cap);
    W.tmp = (float*)malloc(sizeof(float) * 2 * W.cap);
    W.S = (float*)malloc(sizeof(float) * 2 * W.cap);
    int bad = !ids || !st || !te || !tx || !W.M || !W.tmp || !W.S;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int32_t k = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (k >= J->count || bad) break;
        if (eval_node(J, J->nodes[k], &W, ids, st, te, tx, cap, &cnt) != 0) bad = 1;
    }
    pthread_mutex_lock(&J->lock);
    J->total.visits += cnt.visits;
    J->total.unk_visits += cnt.unk_visits;
    J->total.pixel_steps += cnt.pixel_steps;
    J->total.intervals += cnt.intervals;
    if (cnt.max_merged > J->total.max_merged) J->total.max_merged = cnt.max_merged;
    if (bad) J->failed = 1;
    pthread_mutex_unlock(&J->lock);
    free(ids); free(st); free(te); free(tx);
    free(W.M); free(W.tmp); free(W.S);
    return NULL;
}

int ivlref_eval_tree(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                     const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                     const mgref_sensor_params* sp, int32_t wd, int32_t hd, const uint8_t* mask,
                     uint32_t* g_abs, int32_t* k_abs, uint32_t* g_db, int32_t* k_db, float* D,
                     uint32_t* abs_bins, uint32_t* marg_bins, ivlref_counters* cnt, int32_t n_threads) {
    if (n < 1 || nx < 1 || ny < 1 || nz < 1 || !(voxel_m > 0.0f) || parent[0] != -1) return -1;
    mgref_sensor s;
    if (mgref_sensor_init(sp, &s) != 0) return -1;
    ivlref_camera cam;
    if (ivlref_camera_init(sp, voxel_m, wd, hd, &cam) != 0) {
        mgref_sensor_free(&s);
        return -1;
    }
    float* q = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int rc = -1;
    if (!q || !depth || !order) goto done;
    /* validation and q = (p - o) / v as in mgref_eval_tree */
    depth[0] = 0;
    for (int32_t i = 1; i < n; ++i) {
        if (parent[i] < 0 || parent[i] >= i) goto done;
        depth[i] = depth[parent[i]] + 1;
        if (depth[i] > 64) goto done;
    }
    {
        const int32_t dims[3] = {nx, ny, nz};
        for (int32_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                float v = (pos_m[3 * i + a] - origin_m[a]) / voxel_m;
                if (!(v >= 0.0f) || !(v < (float)dims[a]) || (int32_t)floorf(v) >= dims[a]) goto done;
                q[3 * i + a] = v;
            }
    }
    if (mask)
        for (int32_t i = 1; i < n; ++i)
            if (mask[i] && !mask[parent[i]]) goto done;
    {
        ivl_job J;
        memset(&J, 0, sizeof(J));
        J.states = states; J.nx = nx; J.ny = ny; J.nz = nz; J.s = &s; J.cam = &cam;
        J.q = q; J.parent = parent; J.k_db = k_db; J.k_abs = k_abs; J.g_db = g_db; J.g_abs = g_abs; J.D = D;
        J.abs_bins = abs_bins; J.marg_bins = marg_bins;
        pthread_mutex_init(&J.lock, NULL);
        if (n_threads < 1) n_threads = 1;
        if (n_threads > 256) n_threads = 256;
        int32_t maxd = 0;
        for (int32_t i = 0; i < n; ++i) if (depth[i] > maxd) maxd = depth[i];
        for (int32_t d = 0; d <= maxd && !J.failed; ++d) {
            int32_t cntd = 0;
            for (int32_t i = 0; i < n; ++i)
                if (depth[i] == d && (!mask || mask[i])) order[cntd++] = i;
            J.nodes = order; J.count = cntd; J.next = 0;
            if (cntd == 0) continue;
            int nt = n_threads < cntd ? n_threads : cntd;
            if (nt == 1) {
                level_worker(&J);
            } else {
                pthread_t th[256];
                for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, level_worker, &J);
                for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
            }
        }
        pthread_mutex_destroy(&J.lock);
        if (!J.failed) rc = 0;
        if (cnt) *cnt = J.total;
    }
done:
    free(q); free(depth); free(order);
    ivlref_camera_free(&cam);
    mgref_sensor_free(&s);
    return rc;
}
