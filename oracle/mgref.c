/*
 * mgref.c — the ORACLE (test infrastructure only; see mgref.h).
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math -pthread
 * Every function follows the paper section named in its comment. Nothing here
 * is blocked, fused or reordered beyond what that section states.
 */
#define _GNU_SOURCE
#include "mgref.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

enum { S_UNK = 0, S_FREE = 1, S_OCC = 2 };

/* ------------------------------------------------------------------ sensor */

static double snap(double x) { return fabs(x) < 1e-9 ? 0.0 : x; }

/* Yaw candidates (Sec. III-B: the yaw maximising the gain over a candidate
 * set). The candidate set is B azimuth bins; a window of w bins spans the
 * horizontal field of view. Column c's centre azimuth is
 * az_offset + (c + 1/2)*360/n_az; bin(c) is the bin holding that centre; the
 * window starting at bin k holds the columns whose centres lie in
 * [k*n_az/B, (k+w)*n_az/B), which are exactly w_buf = n_az*w/B consecutive
 * columns starting at c0(k) = ceil((2k*n_az - B) / (2B)) mod n_az. */
int mgref_sensor_init(const mgref_sensor_params* p, mgref_sensor* s) {
    memset(s, 0, sizeof(*s));
    if (!p || p->n_az < 1 || p->n_el < 1 || p->yaw_bins < 1) return -1;
    if (!(p->fov_h_deg > 0.0f) || !(p->fov_v_deg > 0.0f) || !(p->fov_v_deg < 180.0f)) return -1;
    if (!(p->range_m > 0.0f)) return -1;
    double wd = (double)p->yaw_bins * (double)p->fov_h_deg / 360.0;
    long w = lround(wd);
    if (w < 1 || fabs(wd - (double)w) > 1e-6) return -1;
    if (2 * w >= p->yaw_bins) return -1;               /* window must span < 180 degrees */
    if (((long)p->n_az * w) % p->yaw_bins != 0) return -1;
    s->p = *p;
    s->win_bins = (int32_t)w;
    s->w_buf = (int32_t)((long)p->n_az * w / p->yaw_bins);

    const int W = p->n_az, H = p->n_el, B = p->yaw_bins;
    s->dir = (float*)malloc(sizeof(float) * 3 * W * H);
    s->inv = (float*)malloc(sizeof(float) * 3 * W * H);
    s->bvx = (float*)malloc(sizeof(float) * W);
    s->bvy = (float*)malloc(sizeof(float) * W);
    s->ts = (float*)malloc(sizeof(float) * (H + 1));
    s->bin_of_col = (int32_t*)malloc(sizeof(int32_t) * W);
    s->c0_of_win = (int32_t*)malloc(sizeof(int32_t) * B);
    if (!s->dir || !s->inv || !s->bvx || !s->bvy || !s->ts || !s->bin_of_col || !s->c0_of_win) {
        mgref_sensor_free(s);
        return -1;
    }
    const double deg = M_PI / 180.0;
    const double daz = 360.0 / (double)W;
    const double del = (double)p->fov_v_deg / (double)H;
    for (int c = 0; c < W; ++c) {
        double az = ((double)p->az_offset_deg + ((double)c + 0.5) * daz) * deg;
        for (int j = 0; j < H; ++j) {
            double el = (-(double)p->fov_v_deg / 2.0 + ((double)j + 0.5) * del) * deg;
            double dd[3] = {cos(el) * cos(az), cos(el) * sin(az), sin(el)};
            int r = c * H + j;
            for (int a = 0; a < 3; ++a) {
                float f = (float)snap(dd[a]);
                s->dir[3 * r + a] = f;
                s->inv[3 * r + a] = (f != 0.0f) ? 1.0f / f : 0.0f;
            }
        }
        double beta = ((double)p->az_offset_deg + (double)c * daz) * deg;
        s->bvx[c] = (float)snap(cos(beta));
        s->bvy[c] = (float)snap(sin(beta));
        s->bin_of_col[c] = (int32_t)(((long)(2 * c + 1) * B) / (2L * W));
    }
    for (int j = 0; j <= H; ++j) {
        double e = (-(double)p->fov_v_deg / 2.0 + (double)j * del) * deg;
        double t = snap(tan(e));
        s->ts[j] = (float)(t * fabs(t));
    }
    for (int k = 0; k < B; ++k) {
        long num = 2L * k * W - B, den = 2L * B;
        long c0 = num >= 0 ? (num + den - 1) / den : 0; /* ceil; num > -den here */
        s->c0_of_win[k] = (int32_t)(c0 % W);
    }
    return 0;
}

void mgref_sensor_free(mgref_sensor* s) {
    free(s->dir); free(s->inv); free(s->bvx); free(s->bvy); free(s->ts);
    free(s->bin_of_col); free(s->c0_of_win);
    memset(s, 0, sizeof(*s));
}

int mgref_sensor_tables(const mgref_sensor_params* p, float* dir, float* inv, float* bv,
                        float* ts, int32_t* bins, int32_t* c0) {
    mgref_sensor s;
    if (mgref_sensor_init(p, &s) != 0) return -1;
    int W = p->n_az, H = p->n_el;
    if (dir) memcpy(dir, s.dir, sizeof(float) * 3 * W * H);
    if (inv) memcpy(inv, s.inv, sizeof(float) * 3 * W * H);
    if (bv) for (int c = 0; c < W; ++c) { bv[2 * c] = s.bvx[c]; bv[2 * c + 1] = s.bvy[c]; }
    if (ts) memcpy(ts, s.ts, sizeof(float) * (H + 1));
    if (bins) memcpy(bins, s.bin_of_col, sizeof(int32_t) * W);
    if (c0) memcpy(c0, s.c0_of_win, sizeof(int32_t) * p->yaw_bins);
    mgref_sensor_free(&s);
    return 0;
}

/* ------------------------------------------------------------------ ray traversal */

/* 3D DDA of Amanatides and Woo (the voxel traversal the paper cites for
 * raycasting, Sec. I and IV-B): start in the voxel holding q, step to the
 * neighbour across whichever voxel face the ray meets first. Face crossing
 * parameters are recomputed from the integer boundary each time,
 * t = (boundary - q) * (1/d), so no error accumulates. Ties between axes step
 * x before y before z. A voxel is visited iff its entry parameter t is below
 * the range limit Rv and the ray is still inside the grid. Unknown and free
 * voxels let the ray through; the first occupied voxel ends it and its entry
 * t is the first-hit depth; without a hit the depth is Rv (Sec. IV-A). */
int mgref_trace_ray_exit(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                         const float q[3], const float d[3], const float inv[3], float rv,
                         int32_t cap, uint32_t* ids, uint8_t* st, float* tenter, float* texit, float* h) {
    int32_t n[3] = {nx, ny, nz};
    int32_t i[3], step[3], nb[3];
    float tn[3];
    for (int a = 0; a < 3; ++a) {
        i[a] = (int32_t)floorf(q[a]);
        if (d[a] > 0.0f) { step[a] = 1; nb[a] = i[a] + 1; tn[a] = ((float)nb[a] - q[a]) * inv[a]; }
        else if (d[a] < 0.0f) { step[a] = -1; nb[a] = i[a]; tn[a] = ((float)nb[a] - q[a]) * inv[a]; }
        else { step[a] = 0; nb[a] = 0; tn[a] = INFINITY; }
    }
    float t = 0.0f;
    int count = 0;
    *h = rv;
    for (;;) {
        if (i[0] < 0 || i[0] >= n[0] || i[1] < 0 || i[1] >= n[1] || i[2] < 0 || i[2] >= n[2]) break;
        if (!(t < rv)) break;
        uint32_t id = (uint32_t)i[0] + (uint32_t)nx * ((uint32_t)i[1] + (uint32_t)ny * (uint32_t)i[2]);
        uint8_t s = states[id];
        if (count >= cap) return -1;
        ids[count] = id;
        st[count] = s;
        tenter[count] = t;
        ++count;
        if (s == S_OCC) { *h = t; if (texit) texit[count - 1] = t; break; }
        int a;
        if (tn[0] <= tn[1] && tn[0] <= tn[2]) a = 0;
        else if (tn[1] <= tn[2]) a = 1;
        else a = 2;
        if (texit) texit[count - 1] = tn[a];      /* the voxel is left where the next one is entered */
        t = tn[a];
        i[a] += step[a];
        nb[a] += step[a];
        tn[a] = ((float)nb[a] - q[a]) * inv[a];
    }
    return count;
}

int mgref_trace_ray(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                    const float q[3], const float d[3], const float inv[3], float rv,
                    int32_t cap, uint32_t* ids, uint8_t* st, float* tenter, float* h) {
    return mgref_trace_ray_exit(states, nx, ny, nz, q, d, inv, rv, cap, ids, st, tenter, NULL, h);
}

/* ------------------------------------------------------------------ ancestor test */

/* Is voxel x already observed by ancestor a? (Sec. IV-B, per-voxel reading.)
 * The ancestor's buffer holds first-hit depths of the panorama rays in its
 * chosen window: pixel (row, col) is the ray of column (c0a + col) mod n_az
 * and row `row`. A pixel's cell is the solid angle between its column's two
 * azimuth boundaries and its row's two elevation boundaries. With r the
 * vector from the ancestor to the voxel centre:
 *   - elevation cell: tan(elev) = r_z / rho, rho^2 = r_x^2 + r_y^2; compared
 *     through the monotone map t -> t|t| as r_z|r_z| >= rho^2 * T_j with
 *     T_j = tan(e_j)|tan(e_j)| at boundary elevation e_j (no square root);
 *   - azimuth cell: r is at or left of boundary b when
 *     b_x r_y - b_y r_x >= 0 (the window spans < 180 degrees);
 *   - row = number of inner elevation boundaries at or below r, col = number
 *     of inner azimuth boundaries at or right of r (counted one by one);
 *   - observed iff inside the window and the band, and
 *     |r|^2 <= D[row][col]^2 (the comparison "<=" of Sec. IV-B).
 * No near plane is applied; a voxel outside the grid is never tested. */
int mgref_obs(const mgref_sensor* s, const float qa[3], int32_t c0a, const float* Da,
              int32_t ix, int32_t iy, int32_t iz, int32_t* row_out, int32_t* col_out) {
    const int W = s->p.n_az, H = s->p.n_el, WB = s->w_buf;
    float rx = ((float)ix + 0.5f) - qa[0];
    float ry = ((float)iy + 0.5f) - qa[1];
    float rz = ((float)iz + 0.5f) - qa[2];
    float rho2 = rx * rx + ry * ry;
    float range2 = rho2 + rz * rz;
    float sz = rz * fabsf(rz);
    if (row_out) *row_out = -1;
    if (col_out) *col_out = -1;
    /* elevation band */
    if (!(sz >= rho2 * s->ts[0])) return 0;
    if (!(sz < rho2 * s->ts[H])) return 0;
    /* azimuth wedge */
    int cb = c0a, ce = (c0a + WB) % W;
    if (!(s->bvx[cb] * ry - s->bvy[cb] * rx >= 0.0f)) return 0;
    if (!(s->bvx[ce] * ry - s->bvy[ce] * rx < 0.0f)) return 0;
    int col = 0;
    for (int i = 1; i < WB; ++i) {
        int c = (c0a + i) % W;
        if (s->bvx[c] * ry - s->bvy[c] * rx >= 0.0f) ++col;
    }
    int row = 0;
    for (int j = 1; j < H; ++j)
        if (sz >= rho2 * s->ts[j]) ++row;
    if (row_out) *row_out = row;
    if (col_out) *col_out = col;
    float D = Da[row * WB + col];
    return range2 <= D * D;
}

/* ------------------------------------------------------------------ windows */

/* Yaw selection (Sec. III-B): the window sum S(k) = sum_{i<w} bins[(k+i) mod B]
 * is maximised over k; the smallest maximising k wins ties. */
uint32_t mgref_best_window(const uint32_t* bins, int32_t B, int32_t w, int32_t* k_out) {
    uint32_t best = 0;
    int32_t bk = 0;
    for (int32_t k = 0; k < B; ++k) {
        uint32_t sum = 0;
        for (int32_t i = 0; i < w; ++i) sum += bins[(k + i) % B];
        if (k == 0 || sum > best) { best = sum; bk = k; }
    }
    *k_out = bk;
    return best;
}

/* ------------------------------------------------------------------ tree driver */

typedef struct {
    const uint8_t* states;
    int32_t nx, ny, nz;
    const mgref_sensor* s;
    float rv;
    const float* q;          /* [n][3] voxel units */
    const int32_t* parent;
    int32_t max_anc;
    int32_t* k_db;           /* window chosen by each evaluated node */
    float* D;
    uint32_t *g_abs, *g_db;
    int32_t* k_abs;
    uint32_t *abs_bins, *marg_bins;
    /* level work list */
    const int32_t* nodes;
    int32_t count;
    int32_t next;
    pthread_mutex_t lock;
    mgref_counters total;
    int failed;
} tree_job;

/* The per-node pass: every panorama ray is traversed; each unknown voxel
 * counts towards the absolute bin of the ray's column and, unless an ancestor
 * observes it (nearest ancestor first, stopping at the first that does),
 * towards the marginal bin (eq. 1 and 2 in the per-ray-incidence reading).
 * h receives the first-hit depth of every ray. */
static int node_pass(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, const mgref_sensor* s,
                     float rv, const float* qn, int32_t na, const float* anc_q, const int32_t* anc_c0,
                     const float* const* anc_D, uint32_t* ab, uint32_t* mb, float* h,
                     uint32_t* ids, uint8_t* st, float* te, int32_t cap, mgref_counters* cnt) {
    const int W = s->p.n_az, H = s->p.n_el;
    for (int c = 0; c < W; ++c) {
        int b = s->bin_of_col[c];
        for (int j = 0; j < H; ++j) {
            int r = c * H + j;
            int nv = mgref_trace_ray(states, nx, ny, nz, qn, s->dir + 3 * r, s->inv + 3 * r, rv, cap, ids,
                                     st, te, &h[r]);
            if (nv < 0) return -1;
            cnt->visits += (uint64_t)nv;
            for (int v = 0; v < nv; ++v) {
                if (st[v] != S_UNK) continue;
                cnt->unk_visits++;
                ab[b]++;
                int32_t ix = (int32_t)(ids[v] % (uint32_t)nx);
                int32_t iy = (int32_t)((ids[v] / (uint32_t)nx) % (uint32_t)ny);
                int32_t iz = (int32_t)(ids[v] / ((uint32_t)nx * (uint32_t)ny));
                int seen = 0;
                for (int k = 0; k < na && !seen; ++k) {
                    cnt->anc_tests++;
                    seen = mgref_obs(s, anc_q + 3 * k, anc_c0[k], anc_D[k], ix, iy, iz, NULL, NULL);
                }
                if (!seen) mb[b]++;
            }
        }
    }
    return 0;
}

int mgref_eval_node(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                    const mgref_sensor_params* sp, float rv, const float q[3], int32_t n_anc,
                    const float* anc_q, const int32_t* anc_c0, const float* anc_D,
                    uint32_t* abs_bins, uint32_t* marg_bins, float* h, mgref_counters* cnt) {
    mgref_sensor s;
    if (n_anc < 0 || n_anc > 128 || mgref_sensor_init(sp, &s) != 0) return -1;
    const float* Dp[128];
    for (int k = 0; k < n_anc; ++k) Dp[k] = anc_D + (size_t)k * s.p.n_el * s.w_buf;
    int32_t cap = 3 * (int32_t)ceilf(rv) + 16;
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    mgref_counters local = {0, 0, 0};
    int rc = -1;
    if (ids && st && te)
        rc = node_pass(states, nx, ny, nz, &s, rv, q, n_anc, anc_q, anc_c0, Dp, abs_bins, marg_bins, h,
                       ids, st, te, cap, &local);
    if (cnt) *cnt = local;
    free(ids); free(st); free(te);
    mgref_sensor_free(&s);
    return rc;
}

/* Evaluate node n of a tree: the per-node pass against its ancestors (parent
 * first), then both yaw windows are selected and the node's buffer is
 * written from the marginal window's columns (Sec. IV-A, IV-B). */
static int eval_node(tree_job* J, int32_t n, float* h, uint32_t* ids, uint8_t* st, float* te,
                     int32_t cap, mgref_counters* cnt) {
    const mgref_sensor* s = J->s;
    const int W = s->p.n_az, H = s->p.n_el, B = s->p.yaw_bins, WB = s->w_buf;
    uint32_t* ab = (uint32_t*)calloc(B, sizeof(uint32_t));
    uint32_t* mb = (uint32_t*)calloc(B, sizeof(uint32_t));
    float aq[3 * 128];
    int32_t ac0[128];
    const float* aD[128];
    int32_t na = 0;
    if (!ab || !mb) { free(ab); free(mb); return -1; }
    for (int32_t a = J->parent[n]; a >= 0 && (J->max_anc < 0 || na < J->max_anc); a = J->parent[a]) {
        aq[3 * na + 0] = J->q[3 * a + 0];
        aq[3 * na + 1] = J->q[3 * a + 1];
        aq[3 * na + 2] = J->q[3 * a + 2];
        ac0[na] = s->c0_of_win[J->k_db[a]];
        aD[na] = J->D + (size_t)a * H * WB;
        ++na;
    }
    if (node_pass(J->states, J->nx, J->ny, J->nz, s, J->rv, J->q + 3 * n, na, aq, ac0, aD, ab, mb, h,
                  ids, st, te, cap, cnt) != 0) {
        free(ab); free(mb);
        return -1;
    }
    int32_t ka, km;
    uint32_t ga = mgref_best_window(ab, B, s->win_bins, &ka);
    uint32_t gm = mgref_best_window(mb, B, s->win_bins, &km);
    if (J->g_abs) J->g_abs[n] = ga;
    if (J->k_abs) J->k_abs[n] = ka;
    J->g_db[n] = gm;
    J->k_db[n] = km;
    int c0 = s->c0_of_win[km];
    float* Dn = J->D + (size_t)n * H * WB;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < WB; ++i) Dn[j * WB + i] = h[((c0 + i) % W) * H + j];
    if (J->abs_bins) memcpy(J->abs_bins + (size_t)n * B, ab, sizeof(uint32_t) * B);
    if (J->marg_bins) memcpy(J->marg_bins + (size_t)n * B, mb, sizeof(uint32_t) * B);
    free(ab);
    free(mb);
    return 0;
}

static void* level_worker(void* arg) {
    tree_job* J = (tree_job*)arg;
    const mgref_sensor* s = J->s;
    int32_t cap = 3 * (int32_t)ceilf(J->rv) + 16;
    float* h = (float*)malloc(sizeof(float) * s->p.n_az * s->p.n_el);
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    mgref_counters cnt = {0, 0, 0};
    int bad = !h || !ids || !st || !te;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int32_t k = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (k >= J->count || bad) break;
        if (eval_node(J, J->nodes[k], h, ids, st, te, cap, &cnt) != 0) { bad = 1; break; }
    }
    pthread_mutex_lock(&J->lock);
    J->total.visits += cnt.visits;
    J->total.unk_visits += cnt.unk_visits;
    J->total.anc_tests += cnt.anc_tests;
    if (bad) J->failed = 1;
    pthread_mutex_unlock(&J->lock);
    free(h); free(ids); free(st); free(te);
    return NULL;
}

/* Validates the tree and converts positions to voxel units, q = (p - o) / v
 * in float (subtract, then divide). Requires parent[0] = -1,
 * 0 <= parent[i] < i, depth <= 64 and every node inside the grid. */
static int prepare_tree(int32_t nx, int32_t ny, int32_t nz, float voxel_m, const float origin_m[3],
                        const float* pos_m, const int32_t* parent, int32_t n, float* q, int32_t* depth) {
    if (n < 1 || nx < 1 || ny < 1 || nz < 1 || !(voxel_m > 0.0f)) return -1;
    if (parent[0] != -1) return -1;
    depth[0] = 0;
    for (int32_t i = 1; i < n; ++i) {
        if (parent[i] < 0 || parent[i] >= i) return -1;
        depth[i] = depth[parent[i]] + 1;
        if (depth[i] > 64) return -1;
    }
    int32_t dims[3] = {nx, ny, nz};
    for (int32_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = (pos_m[3 * i + a] - origin_m[a]) / voxel_m;
            if (!(v >= 0.0f) || !(v < (float)dims[a])) return -1;
            if ((int32_t)floorf(v) >= dims[a]) return -1;
            q[3 * i + a] = v;
        }
    return 0;
}

int mgref_eval_tree(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                    const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                    const mgref_sensor_params* sp, int32_t max_anc, const uint8_t* mask,
                    uint32_t* g_abs, int32_t* k_abs, uint32_t* g_db, int32_t* k_db, float* D,
                    uint32_t* abs_bins, uint32_t* marg_bins, mgref_counters* cnt,
                    int32_t n_threads) {
    mgref_sensor s;
    if (mgref_sensor_init(sp, &s) != 0) return -1;
    float* q = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int rc = -1;
    if (!q || !depth || !order) goto done;
    if (prepare_tree(nx, ny, nz, voxel_m, origin_m, pos_m, parent, n, q, depth) != 0) goto done;
    if (mask)
        for (int32_t i = 1; i < n; ++i)
            if (mask[i] && !mask[parent[i]]) goto done;   /* not ancestor-closed */

    tree_job J;
    memset(&J, 0, sizeof(J));
    J.states = states; J.nx = nx; J.ny = ny; J.nz = nz; J.s = &s;
    J.rv = sp->range_m / voxel_m;
    J.q = q; J.parent = parent; J.max_anc = max_anc;
    J.k_db = k_db; J.D = D; J.g_abs = g_abs; J.g_db = g_db; J.k_abs = k_abs;
    J.abs_bins = abs_bins; J.marg_bins = marg_bins;
    pthread_mutex_init(&J.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    int32_t maxd = 0;
    for (int32_t i = 0; i < n; ++i) if (depth[i] > maxd) maxd = depth[i];
    /* Depth order (Sec. IV-C): all nodes of depth d before any of depth d+1. */
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
done:
    free(q); free(depth); free(order);
    mgref_sensor_free(&s);
    return rc;
}

/* ------------------------------------------------------------------ exact sets */

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

static int contains(const uint32_t* set, uint32_t n, uint32_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (set[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < n && set[lo] == key;
}

/* I(n) at window k: the distinct unknown voxels met by the window's rays
 * (sorted ascending). */
int64_t mgref_node_set(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz,
                       const mgref_sensor_params* sp, float rv, const float q[3], int32_t k,
                       int64_t cap, uint32_t* ids_out) {
    mgref_sensor s;
    if (mgref_sensor_init(sp, &s) != 0) return -1;
    if (k < 0 || k >= sp->yaw_bins) { mgref_sensor_free(&s); return -1; }
    const int W = s.p.n_az, H = s.p.n_el, WB = s.w_buf;
    int32_t rcap = 3 * (int32_t)ceilf(rv) + 16;
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * rcap);
    uint8_t* st = (uint8_t*)malloc((size_t)rcap);
    float* te = (float*)malloc(sizeof(float) * rcap);
    int64_t cnt = 0;
    int c0 = s.c0_of_win[k];
    for (int ci = 0; ci < WB && cnt >= 0; ++ci) {
        int c = (c0 + ci) % W;
        for (int j = 0; j < H && cnt >= 0; ++j) {
            int r = c * H + j;
            float h;
            int nv = mgref_trace_ray(states, nx, ny, nz, q, s.dir + 3 * r, s.inv + 3 * r, rv, rcap, ids, st,
                                     te, &h);
            if (nv < 0) { cnt = -1; break; }
            for (int v = 0; v < nv; ++v) {
                if (st[v] != S_UNK) continue;
                if (cnt >= cap) { cnt = -1; break; }
                ids_out[cnt++] = ids[v];
            }
        }
    }
    if (cnt > 0) {
        qsort(ids_out, (size_t)cnt, sizeof(uint32_t), cmp_u32);
        int64_t u = 0;
        for (int64_t i = 0; i < cnt; ++i)
            if (u == 0 || ids_out[i] != ids_out[u - 1]) ids_out[u++] = ids_out[i];
        cnt = u;
    }
    free(ids); free(st); free(te);
    mgref_sensor_free(&s);
    return cnt;
}

/* Exact marginal gain, eq. (2): I(n) is the set of distinct unknown voxels
 * met by the rays of node n's chosen window (sorted array, the role the
 * paper's per-node hash map plays); a voxel is new when no ancestor's set
 * holds it. Each ancestor's set is probed separately instead of being merged
 * (Sec. IV-E keeps only local observations). */
int mgref_exact(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                const mgref_sensor_params* sp, const int32_t* k_db, const float* D,
                const uint8_t* mask, uint32_t* A_set, uint32_t* X_set, uint32_t* X_ray,
                uint32_t* G_db_set) {
    mgref_sensor s;
    if (mgref_sensor_init(sp, &s) != 0) return -1;
    const int W = s.p.n_az, H = s.p.n_el, WB = s.w_buf;
    float rv = sp->range_m / voxel_m;
    int32_t cap = 3 * (int32_t)ceilf(rv) + 16;
    float* q = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t** sets = (uint32_t**)calloc((size_t)n, sizeof(uint32_t*));
    uint32_t* setn = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    int rc = -1;
    if (!q || !depth || !sets || !setn || !ids || !st || !te) goto done;
    if (prepare_tree(nx, ny, nz, voxel_m, origin_m, pos_m, parent, n, q, depth) != 0) goto done;
    if (mask)
        for (int32_t i = 1; i < n; ++i)
            if (mask[i] && !mask[parent[i]]) goto done;

    /* I(n) for every node in the mask */
    for (int32_t i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        size_t capn = 1024, cnt = 0;
        uint32_t* buf = (uint32_t*)malloc(sizeof(uint32_t) * capn);
        if (!buf) goto done;
        int c0 = s.c0_of_win[k_db[i]];
        for (int ci = 0; ci < WB; ++ci) {
            int c = (c0 + ci) % W;
            for (int j = 0; j < H; ++j) {
                int r = c * H + j;
                float h;
                int nv = mgref_trace_ray(states, nx, ny, nz, q + 3 * i, s.dir + 3 * r, s.inv + 3 * r, rv,
                                         cap, ids, st, te, &h);
                if (nv < 0) { free(buf); goto done; }
                for (int v = 0; v < nv; ++v) {
                    if (st[v] != S_UNK) continue;
                    if (cnt == capn) {
                        capn *= 2;
                        uint32_t* nb2 = (uint32_t*)realloc(buf, sizeof(uint32_t) * capn);
                        if (!nb2) { free(buf); goto done; }
                        buf = nb2;
                    }
                    buf[cnt++] = ids[v];
                }
            }
        }
        qsort(buf, cnt, sizeof(uint32_t), cmp_u32);
        size_t u = 0;
        for (size_t k = 0; k < cnt; ++k)
            if (u == 0 || buf[k] != buf[u - 1]) buf[u++] = buf[k];
        sets[i] = buf;
        setn[i] = (uint32_t)u;
    }

    for (int32_t i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        int32_t anc[128];
        int na = 0;
        for (int32_t a = parent[i]; a >= 0; a = parent[a]) anc[na++] = a;
        uint32_t xs = 0, gds = 0;
        for (uint32_t k = 0; k < setn[i]; ++k) {
            uint32_t id = sets[i][k];
            int in_union = 0;
            for (int m = 0; m < na && !in_union; ++m)
                in_union = contains(sets[anc[m]], setn[anc[m]], id);
            if (!in_union) ++xs;
            int32_t ix = (int32_t)(id % (uint32_t)nx);
            int32_t iy = (int32_t)((id / (uint32_t)nx) % (uint32_t)ny);
            int32_t iz = (int32_t)(id / ((uint32_t)nx * (uint32_t)ny));
            int seen = 0;
            for (int m = 0; m < na && !seen; ++m) {
                int32_t a = anc[m];
                seen = mgref_obs(&s, q + 3 * a, s.c0_of_win[k_db[a]], D + (size_t)a * H * WB, ix, iy, iz,
                                 NULL, NULL);
            }
            if (!seen) ++gds;
        }
        /* incidences */
        uint32_t xr = 0;
        int c0 = s.c0_of_win[k_db[i]];
        for (int ci = 0; ci < WB; ++ci) {
            int c = (c0 + ci) % W;
            for (int j = 0; j < H; ++j) {
                int r = c * H + j;
                float h;
                int nv = mgref_trace_ray(states, nx, ny, nz, q + 3 * i, s.dir + 3 * r, s.inv + 3 * r, rv,
                                         cap, ids, st, te, &h);
                for (int v = 0; v < nv; ++v) {
                    if (st[v] != S_UNK) continue;
                    int in_union = 0;
                    for (int m = 0; m < na && !in_union; ++m)
                        in_union = contains(sets[anc[m]], setn[anc[m]], ids[v]);
                    if (!in_union) ++xr;
                }
            }
        }
        if (A_set) A_set[i] = setn[i];
        if (X_set) X_set[i] = xs;
        if (X_ray) X_ray[i] = xr;
        if (G_db_set) G_db_set[i] = gds;
    }
    rc = 0;
done:
    if (sets) for (int32_t i = 0; i < n; ++i) free(sets[i]);
    free(sets); free(setn); free(q); free(depth); free(ids); free(st); free(te);
    mgref_sensor_free(&s);
    return rc;
}

/* ------------------------------------------------------------------ exact marginal with its own yaw */

/* The exact marginal gain as a planner would use it (eq. 2 with the yaw
 * choice of Sec. III-B): nodes in depth order; for node n every panorama ray
 * is traversed and each unknown voxel it meets counts towards the bin of the
 * ray's column unless some ancestor's set I(a) holds it (I(a) taken at a's
 * own chosen window); the window with the largest sum wins (smallest k on
 * ties), and I(n) is then the set of distinct unknown voxels met by that
 * window's rays. Counts are ray incidences, as for the depth-buffer gain.
 * mask: NULL or an ancestor-closed subset. */
int mgref_exact_marginal(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                         const float origin_m[3], const float* pos_m, const int32_t* parent, int32_t n,
                         const mgref_sensor_params* sp, const uint8_t* mask, uint32_t* gain, int32_t* k_out) {
    mgref_sensor s;
    if (mgref_sensor_init(sp, &s) != 0) return -1;
    const int W = s.p.n_az, H = s.p.n_el, B = s.p.yaw_bins;
    const float rv = sp->range_m / voxel_m;
    const int32_t cap = 3 * (int32_t)ceilf(rv) + 16;
    float* q = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t** sets = (uint32_t**)calloc((size_t)n, sizeof(uint32_t*));
    uint32_t* setn = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    uint8_t* st = (uint8_t*)malloc((size_t)cap);
    float* te = (float*)malloc(sizeof(float) * cap);
    uint32_t* bins = (uint32_t*)malloc(sizeof(uint32_t) * B);
    int rc = -1;
    int32_t maxd = 0;
    if (!q || !depth || !sets || !setn || !ids || !st || !te || !bins) goto done;
    if (prepare_tree(nx, ny, nz, voxel_m, origin_m, pos_m, parent, n, q, depth) != 0) goto done;
    if (mask)
        for (int32_t i = 1; i < n; ++i)
            if (mask[i] && !mask[parent[i]]) goto done;
    for (int32_t i = 0; i < n; ++i) if (depth[i] > maxd) maxd = depth[i];
    for (int32_t d = 0; d <= maxd; ++d) {
        for (int32_t i = 0; i < n; ++i) {
            if (depth[i] != d || (mask && !mask[i])) continue;
            int32_t anc[65], na = 0;
            for (int32_t a = parent[i]; a >= 0 && na < 65; a = parent[a]) anc[na++] = a;
            memset(bins, 0, sizeof(uint32_t) * B);
            for (int c = 0; c < W; ++c) {
                const int b = s.bin_of_col[c];
                for (int j = 0; j < H; ++j) {
                    const int r = c * H + j;
                    float h;
                    int nv = mgref_trace_ray(states, nx, ny, nz, q + 3 * i, s.dir + 3 * r, s.inv + 3 * r, rv, cap,
                                             ids, st, te, &h);
                    if (nv < 0) goto done;
                    for (int v = 0; v < nv; ++v) {
                        if (st[v] != S_UNK) continue;
                        int in_union = 0;
                        for (int m = 0; m < na && !in_union; ++m)
                            in_union = contains(sets[anc[m]], setn[anc[m]], ids[v]);
                        if (!in_union) bins[b]++;
                    }
                }
            }
            int32_t k;
            gain[i] = mgref_best_window(bins, B, s.win_bins, &k);
            k_out[i] = k;
            /* I(i) at the chosen window: at most the window's unknown incidences, which the
             * absolute count of that window bounds; grow until the set fits */
            int64_t capn = 4096, cnt;
            uint32_t* buf = NULL;
            for (;;) {
                buf = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)capn);
                if (!buf) goto done;
                cnt = mgref_node_set(states, nx, ny, nz, sp, rv, q + 3 * i, k, capn, buf);
                if (cnt >= 0) break;
                free(buf);
                capn *= 4;
            }
            sets[i] = buf;
            setn[i] = (uint32_t)cnt;
        }
    }
    rc = 0;
done:
    if (sets) for (int32_t i = 0; i < n; ++i) free(sets[i]);
    free(sets); free(setn); free(q); free(depth); free(ids); free(st); free(te); free(bins);
    mgref_sensor_free(&s);
    return rc;
}
