// Interval mode: the paper's own ancestor test (Sec. IV-A, IV-B, eq. 5-7).
//
// Each node keeps a pinhole depth buffer of W_D x H_D pixels at its chosen
// yaw, by default sized so that one pixel spans one voxel at the maximum range
// (Sec. IV-A). A pixel holds the camera-frame z of the first occupied voxel on
// the ray through its centre, or of the ray's end at the range limit.
//
// A candidate ray r(t) = q + t d, 0 <= t <= Rv (one thread per panorama ray),
// is moved into every ancestor's camera frame, clipped to the valid depth
// range z_near <= z <= Rv (z is linear in t), projected with eq. (5), clipped
// to the buffer with the Liang-Barsky algorithm and walked pixel by pixel with
// a 2D DDA. Inverse depth is linear in screen space (eq. 6), so the part of a
// pixel's span where z <= the stored depth is found by solving one linear
// equation; its two ends, mapped back to t perspective-correctly, are an
// overlap interval of the ancestor (eq. 7), joined to the previous one when it
// starts at or before that one's end. Intervals of all ancestors are merged
// into one sorted list of disjoint intervals per ray. The 3D DDA then counts
// an unknown voxel towards the absolute bin of the ray's column, and towards
// the marginal bin unless the midpoint of its chord [t_enter, min(t_exit, Rv)]
// lies in a merged interval. Window selection reuses the per-level finish
// kernel; the nodes of the level then render their buffers at the chosen yaw.
//
// No voxel past the ray's first hit h is counted, and every counted midpoint
// is <= h (the last chord before the hit ends at h exactly). An ancestor's
// intervals start strictly later one after another, so once one starts past h
// it and all later ones cover no counted midpoint: the walk of that ancestor
// stops there, which leaves every count as it is.
//
// The merged list lives in registers/scratch with room for kIvlCap intervals
// per ray, as a window of the union: it holds the union's components from t0
// on, exactly up to a cut tcut (the start of the first interval it had no room
// for). A voxel past the cut moves the window (t0 = tcut) and regenerates the
// ancestors' intervals, so results never depend on the capacity; most rays
// need a single window.
//
// Camera frame of yaw psi: x right = (sin psi, -cos psi, 0), y down =
// (0, 0, -1), z forward = (cos psi, sin psi, 0), in voxel units. The yaw of
// window k is az_offset + (k + w/2) * 360 / B degrees. Geometry is binary32
// in the order written (no contraction); tables are computed in double on the
// host and rounded once.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "mg_batch.h"

using namespace mgk;

namespace mgi {

constexpr int kIvlThreads = 256;
constexpr int kIvlCap = 16;        // merged intervals held per ray
constexpr int kMaxSide = 4096;     // buffer width / height limit

// Device view of the interval-mode camera and the tree's buffers.
struct Cam {
    const float4* pdir;   // [hd*wd] unit camera-frame direction of pixel (i, j) at j*wd + i
    const float2* cs;     // [B] cos, sin of the yaw of window k
    float* dpin;          // [n][hd*wd] the nodes' depth buffers (camera z)
    float* winv;          // [n][hd*wd] their inverse depths 1/z (0 where z = 0)
    int32_t wd, hd, npx;
    float fx, fy, cx, cy, znear, rv;
};

// One ancestor of the node a workgroup evaluates (LDS copy).
struct Anc {
    float qx, qy, qz, c, s;
    uint32_t node;
    uint32_t pad[2];
};

// t of screen parameter s: w(s) = (1 - s) w_A + s w_B (eq. 6); the fraction of
// the 3D segment at s is s w_B / w(s).
__device__ __forceinline__ float t_of_s(float s, float wa, float wb, float tlo, float thi) {
    const float lam = (s * wb) / ((1.0f - s) * wa + s * wb);
    return tlo + lam * (thi - tlo);
}

// Overlap intervals of ancestor A on the ray from qn along d, 0 <= t <= Rv,
// in the order the 2D DDA finds them: each pixel's observed span [lo, hi] in s
// is mapped to [t(lo), t(hi)]; it joins the open interval when t(lo) <= the
// open one's end, otherwise the open one goes to sink(lo, hi) and the new one
// is opened. The walk ends early once the open interval starts past tstop
// (the ray's first hit) or a sink returns true (then this function returns
// true).
template <class Sink>
__device__ bool anc_intervals(const Cam& C, float qx, float qy, float qz, float dx, float dy, float dz, float tstop,
                              const Anc& A, Sink& sink) {
    const float c = A.c, s = A.s;
    const float ox = qx - A.qx, oy = qy - A.qy, oz = qz - A.qz;
    const float P0x = s * ox - c * oy, P0y = -oz, P0z = c * ox + s * oy;
    const float Dx = s * dx - c * dy, Dy = -dz, Dz = c * dx + s * dy;
    float tlo, thi;
    if (Dz == 0.0f) {
        if (!(P0z >= C.znear && P0z <= C.rv)) return false;
        tlo = 0.0f;
        thi = C.rv;
    } else {
        const float t1 = (C.znear - P0z) / Dz, t2 = (C.rv - P0z) / Dz;
        const float a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
        tlo = a > 0.0f ? a : 0.0f;
        thi = b < C.rv ? b : C.rv;
    }
    if (!(tlo < thi)) return false;
    const float Ax = P0x + tlo * Dx, Ay = P0y + tlo * Dy, Az = P0z + tlo * Dz;
    const float Bx = P0x + thi * Dx, By = P0y + thi * Dy, Bz = P0z + thi * Dz;
    if (!(Az > 0.0f && Bz > 0.0f)) return false;
    const float uA = C.fx * Ax / Az + C.cx, vA = C.fy * Ay / Az + C.cy;
    const float uB = C.fx * Bx / Bz + C.cx, vB = C.fy * By / Bz + C.cy;
    const float wa = 1.0f / Az, wb = 1.0f / Bz;
    const float dw = wb - wa;
    // Liang-Barsky against u >= 0, u <= W_D, v >= 0, v <= H_D
    const float du = uB - uA, dv = vB - vA;
    const float pp[4] = {-du, du, -dv, dv};
    const float qq[4] = {uA, (float)C.wd - uA, vA, (float)C.hd - vA};
    float s0 = 0.0f, s1 = 1.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (pp[e] == 0.0f) {
            if (qq[e] < 0.0f) return false;
            continue;
        }
        const float r = qq[e] / pp[e];
        if (pp[e] < 0.0f) s0 = r > s0 ? r : s0;
        else s1 = r < s1 ? r : s1;
    }
    if (!(s0 < s1)) return false;
    // 2D DDA; crossings recomputed from the integer boundary, ties step u first
    const float u0 = uA + s0 * du, v0 = vA + s0 * dv;
    int32_t i = (int32_t)floorf(u0), j = (int32_t)floorf(v0);
    i = i < 0 ? 0 : (i > C.wd - 1 ? C.wd - 1 : i);
    j = j < 0 ? 0 : (j > C.hd - 1 ? C.hd - 1 : j);
    const int32_t si = du > 0.0f ? 1 : (du < 0.0f ? -1 : 0);
    const int32_t sj = dv > 0.0f ? 1 : (dv < 0.0f ? -1 : 0);
    const float iu = si ? 1.0f / du : 0.0f, iv = sj ? 1.0f / dv : 0.0f;
    int32_t bu = si > 0 ? i + 1 : i, bv = sj > 0 ? j + 1 : j;
    const float inf = __builtin_inff();
    float su = si ? ((float)bu - uA) * iu : inf;
    float sv = sj ? ((float)bv - vA) * iv : inf;
    float sa = s0;
    const float* __restrict__ Wa = C.winv + (size_t)A.node * (size_t)C.npx;
    float olo = 0.0f, ohi = 0.0f;             // the open interval, in t
    bool open = false;
    int32_t off = j * C.wd + i;               // the pixel's offset, kept up to date by the steps
    const int32_t voff = sj * C.wd;
    float wD = Wa[off];                       // 1/D, or 0 for D = 0 (nothing observed)
    for (int32_t it = 0; it < C.wd + C.hd + 2; ++it) {
        float e = su < sv ? su : sv;
        e = e < s1 ? e : s1;
        // the next pixel first, so that its load is in flight while this one is processed
        const bool stepu = su <= sv;
        const int32_t ni = stepu ? i + si : i, nj = stepu ? j : j + sj;
        const bool more = (e < s1) & ((uint32_t)ni < (uint32_t)C.wd) & ((uint32_t)nj < (uint32_t)C.hd);
        const int32_t noff = more ? off + (stepu ? si : voff) : off;
        const float wN = Wa[noff];
        // the part [lo, hi] of [sa, e] where w(s) >= 1/D, i.e. z(s) <= D (w is
        // linear in s, eq. 6; with w constant the whole span or nothing)
        if (wD > 0.0f) {
            const float ss = (wD - wa) / dw;
            const float lo = wb > wa ? (sa > ss ? sa : ss) : sa;
            const float hi = wb < wa ? (e < ss ? e : ss) : e;
            if (((wb != wa) | (wa >= wD)) & (lo <= hi)) {
                const float tl = t_of_s(lo, wa, wb, tlo, thi), th = t_of_s(hi, wa, wb, tlo, thi);
                if (open & (tl <= ohi)) {
                    ohi = th > ohi ? th : ohi;
                } else {
                    if (open && sink(olo, ohi)) return true;
                    if (tl > tstop) return false;     // this and every later interval start past tstop
                    olo = tl;
                    ohi = th;
                    open = true;
                }
            }
        }
        if (!more) break;
        i = ni;
        j = nj;
        off = noff;
        // the stepped axis moves to its next boundary (selects, not a branch: the
        // axis that did not step keeps its value)
        bu += stepu ? si : 0;
        bv += stepu ? 0 : sj;
        const float nsu = ((float)bu - uA) * iu, nsv = ((float)bv - vA) * iv;
        su = stepu ? nsu : su;
        sv = stepu ? sv : nsv;
        sa = e;
        wD = wN;
    }
    return open ? sink(olo, ohi) : false;
}

// Window of the union of intervals: its components that reach t0 or later,
// sorted, at most cap (<= kIvlCap) of them. An interval that would need a
// further component is dropped and lowers tcut to its start (so is the last
// component when an earlier one is inserted into a full list); every
// interval dropped starts at or after tcut, so membership of any t in
// [t0, tcut) is exact. Intervals starting at or after tcut stop the
// ancestor's walk (the rest of its intervals start later still).
struct Window {
    float lo[kIvlCap], hi[kIvlCap];
    int32_t m = 0, cap = kIvlCap;
    float t0 = -__builtin_inff(), tcut = __builtin_inff();
    __device__ bool operator()(float a, float b) {
        if (a >= tcut) return true;
        if (b < t0) return false;
        int32_t i = 0;
        while (i < m && hi[i] < a) ++i;          // components that end before a
        int32_t j = i;
        float nlo = a, nhi = b;
        while (j < m && lo[j] <= b) {            // overlapping or touching ones join
            nlo = lo[j] < nlo ? lo[j] : nlo;
            nhi = hi[j] > nhi ? hi[j] : nhi;
            ++j;
        }
        const int32_t removed = j - i;
        if (removed == 0) {
            if (m == cap) {
                if (i == m) {                    // after every kept component
                    tcut = a;
                    return true;
                }
                tcut = lo[m - 1];                // the last component makes room
                --m;
            }
            for (int32_t k = m; k > i; --k) {
                lo[k] = lo[k - 1];
                hi[k] = hi[k - 1];
            }
            ++m;
        } else {
            for (int32_t k = j; k < m; ++k) {
                lo[k - removed + 1] = lo[k];
                hi[k - removed + 1] = hi[k];
            }
            m -= removed - 1;
        }
        lo[i] = nlo;
        hi[i] = nhi;
        return false;
    }
};

// One level of one tree: workgroup = kIvlThreads panorama rays of one node.
__global__ __launch_bounds__(kIvlThreads) void k_ivl_trace(MapDev M, SensorDev S, TreeDev Tr, Cam C,
                                                           const int32_t* __restrict__ nodes,
                                                           const int32_t* __restrict__ yaw, int32_t tiles,
                                                           int32_t cap) {
    __shared__ Anc s_anc[kMaxAnc];
    __shared__ uint32_t s_bins[2 * kMaxBins];
    const int32_t tid = threadIdx.x;
    const int32_t node = nodes[blockIdx.x / tiles];
    const int32_t tile = blockIdx.x % tiles;
    const int32_t a0 = Tr.anc_ptr[node];
    const int32_t na = Tr.anc_ptr[node + 1] - a0;       // nearest first
    for (int32_t k = tid; k < na; k += kIvlThreads) {
        const int32_t a = Tr.anc_ids[a0 + k];
        const float4 qa = Tr.q4[a];
        const float2 cs = C.cs[yaw[a]];
        Anc A;
        A.qx = qa.x; A.qy = qa.y; A.qz = qa.z;
        A.c = cs.x; A.s = cs.y;
        A.node = (uint32_t)a;
        A.pad[0] = A.pad[1] = 0u;
        s_anc[k] = A;
    }
    for (int32_t i = tid; i < 2 * S.B; i += kIvlThreads) s_bins[i] = 0u;
    __syncthreads();

    const int32_t r = tile * kIvlThreads + tid;
    if (r < S.R) {
        const float4 p = Tr.q4[node];
        const float4 d = S.d4[r];
        const float4 inv = S.iv4[r];
        // 3D DDA (Amanatides-Woo; crossings recomputed as (b - q) / d; ties x, y, z),
        // first to the ray's first hit h, then again counting
        const int32_t ix0 = (int32_t)floorf(p.x), iy0 = (int32_t)floorf(p.y), iz0 = (int32_t)floorf(p.z);
        const int32_t sx = d.x > 0.f ? 1 : (d.x < 0.f ? -1 : 0);
        const int32_t sy = d.y > 0.f ? 1 : (d.y < 0.f ? -1 : 0);
        const int32_t sz = d.z > 0.f ? 1 : (d.z < 0.f ? -1 : 0);
        const int32_t bx0 = sx > 0 ? ix0 + 1 : ix0, by0 = sy > 0 ? iy0 + 1 : iy0, bz0 = sz > 0 ? iz0 + 1 : iz0;
        const float inf = __builtin_inff();
        const float tx0 = sx ? ((float)bx0 - p.x) * inv.x : inf;
        const float ty0 = sy ? ((float)by0 - p.y) * inv.y : inf;
        const float tz0 = sz ? ((float)bz0 - p.z) * inv.z : inf;
        float h = S.rv;
        {
            int32_t ix = ix0, iy = iy0, iz = iz0, bx = bx0, by = by0, bz = bz0;
            float tx = tx0, ty = ty0, tz = tz0, t = 0.0f;
            for (;;) {
                if (ix < 0 || ix >= M.nx || iy < 0 || iy >= M.ny || iz < 0 || iz >= M.nz) break;
                if (!(t < S.rv)) break;
                const uint32_t st = M.bricks[voxel_addr(ix, iy, iz, M)];
                if (st == kOccupied) {
                    h = t;
                    break;
                }
                const uint32_t level = (st >> kLevelShift) & kLevelMask;
                if (level != 0u) {          // a marked block holds no occupied voxel
                    t = cross_block(32 >> level, p, inv, sx, sy, sz, ix, iy, iz, bx, by, bz, tx, ty, tz);
                    continue;
                }
                const int ax = (tx <= ty && tx <= tz) ? 0 : (ty <= tz ? 1 : 2);
                if (ax == 0) {
                    t = tx; ix += sx; bx += sx; tx = ((float)bx - p.x) * inv.x;
                } else if (ax == 1) {
                    t = ty; iy += sy; by += sy; ty = ((float)by - p.y) * inv.y;
                } else {
                    t = tz; iz += sz; bz += sz; tz = ((float)bz - p.z) * inv.z;
                }
            }
        }
        Window U;
        U.cap = cap;
        for (int32_t k = 0; k < na; ++k) anc_intervals(C, p.x, p.y, p.z, d.x, d.y, d.z, h, s_anc[k], U);
        int32_t ix = ix0, iy = iy0, iz = iz0, bx = bx0, by = by0, bz = bz0;
        float tx = tx0, ty = ty0, tz = tz0;
        float t = 0.0f;
        uint32_t n_abs = 0, n_marg = 0;
        int32_t ptr = 0;
        for (;;) {
            if (ix < 0 || ix >= M.nx || iy < 0 || iy >= M.ny || iz < 0 || iz >= M.nz) break;
            if (!(t < S.rv)) break;
            const uint8_t st = M.bricks[voxel_addr(ix, iy, iz, M)];
            if (st == kOccupied) break;
            const uint32_t level = (st >> kLevelShift) & kLevelMask;
            if ((level != 0u) & ((st & 3u) == kFree)) {    // a free block counts nothing
                t = cross_block(32 >> level, p, inv, sx, sy, sz, ix, iy, iz, bx, by, bz, tx, ty, tz);
                continue;
            }
            const int ax = (tx <= ty && tx <= tz) ? 0 : (ty <= tz ? 1 : 2);
            const float tn = ax == 0 ? tx : (ax == 1 ? ty : tz);
            if (is_unknown(st)) {
                ++n_abs;
                const float tex = tn < S.rv ? tn : S.rv;
                const float tm = 0.5f * (t + tex);
                while (tm >= U.tcut) {               // move the window past the cut
                    U.t0 = U.tcut;
                    U.tcut = inf;
                    U.m = 0;
                    for (int32_t k = 0; k < na; ++k) anc_intervals(C, p.x, p.y, p.z, d.x, d.y, d.z, h, s_anc[k], U);
                    ptr = 0;
                }
                while (ptr < U.m && U.hi[ptr] < tm) ++ptr;
                const bool covered = ptr < U.m && U.lo[ptr] <= tm;
                n_marg += covered ? 0u : 1u;
            }
            t = tn;
            if (ax == 0) {
                ix += sx;
                bx += sx;
                tx = ((float)bx - p.x) * inv.x;
            } else if (ax == 1) {
                iy += sy;
                by += sy;
                ty = ((float)by - p.y) * inv.y;
            } else {
                iz += sz;
                bz += sz;
                tz = ((float)bz - p.z) * inv.z;
            }
        }
        const int32_t bin = S.bin_of_col[r / S.H];
        if (n_abs) atomicAdd(&s_bins[bin], n_abs);
        if (n_marg) atomicAdd(&s_bins[S.B + bin], n_marg);
    }
    __syncthreads();
    uint32_t* gb = Tr.bins + (size_t)node * 2 * S.B;
    for (int32_t i = tid; i < 2 * S.B; i += kIvlThreads) {
        const uint32_t v = s_bins[i];
        if (v) atomicAdd(&gb[i], v);
    }
}

// Depth buffers of one level's nodes at their chosen windows: one thread per
// pixel; the first occupied voxel's entry t (or Rv) times the pixel
// direction's camera z.
__global__ __launch_bounds__(kIvlThreads) void k_ivl_render(MapDev M, Cam C, TreeDev Tr,
                                                            const int32_t* __restrict__ nodes,
                                                            const int32_t* __restrict__ yaw, int32_t tiles) {
    const int32_t node = nodes[blockIdx.x / tiles];
    const int32_t px = (blockIdx.x % tiles) * kIvlThreads + (int32_t)threadIdx.x;
    if (px >= C.npx) return;
    const float2 cs = C.cs[yaw[node]];
    const float c = cs.x, s = cs.y;
    const float4 pd = C.pdir[px];
    const float d[3] = {s * pd.x + c * pd.z, s * pd.z - c * pd.x, -pd.y};
    float iv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) iv[a] = d[a] != 0.0f ? 1.0f / d[a] : 0.0f;
    const float4 q = Tr.q4[node];
    const float qv[3] = {q.x, q.y, q.z};
    const int32_t n[3] = {M.nx, M.ny, M.nz};
    int32_t i[3], st[3], nb[3];
    float tn[3];
    const float inf = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        i[a] = (int32_t)floorf(qv[a]);
        st[a] = d[a] > 0.0f ? 1 : (d[a] < 0.0f ? -1 : 0);
        nb[a] = st[a] > 0 ? i[a] + 1 : i[a];
        tn[a] = st[a] ? ((float)nb[a] - qv[a]) * iv[a] : inf;
    }
    float t = 0.0f, h = C.rv;
    for (;;) {
        if (i[0] < 0 || i[0] >= n[0] || i[1] < 0 || i[1] >= n[1] || i[2] < 0 || i[2] >= n[2]) break;
        if (!(t < C.rv)) break;
        const uint32_t sv = M.bricks[voxel_addr(i[0], i[1], i[2], M)];
        if (sv == kOccupied) {
            h = t;
            break;
        }
        const uint32_t level = (sv >> kLevelShift) & kLevelMask;
        if (level != 0u) {              // a marked block holds no occupied voxel
            t = cross_block(32 >> level, make_float4(qv[0], qv[1], qv[2], 0.f), make_float4(iv[0], iv[1], iv[2], 0.f),
                            st[0], st[1], st[2], i[0], i[1], i[2], nb[0], nb[1], nb[2], tn[0], tn[1], tn[2]);
            continue;
        }
        const int ax = (tn[0] <= tn[1] && tn[0] <= tn[2]) ? 0 : (tn[1] <= tn[2] ? 1 : 2);
        t = tn[ax];
        i[ax] += st[ax];
        nb[ax] += st[ax];
        tn[ax] = ((float)nb[ax] - qv[ax]) * iv[ax];
    }
    const float z = h * pd.z;
    C.dpin[(size_t)node * (size_t)C.npx + px] = z;
    C.winv[(size_t)node * (size_t)C.npx + px] = z > 0.0f ? 1.0f / z : 0.0f;
}

// ---------------------------------------------------------------- host

double snap(double x) { return std::fabs(x) < 1e-9 ? 0.0 : x; }

struct HostCam {
    int32_t wd = 0, hd = 0;
    float fx = 0, fy = 0, cx = 0, cy = 0, znear = 0, rv = 0;
    std::vector<float4> pdir;
    std::vector<float2> cs;
};

// Buffer size by the resolution rule of Sec. IV-A when wd or hd <= 0; the
// pinhole's principal point is the buffer centre and its focal lengths make
// the buffer span the field of view. Tables in double, rounded once.
int build_camera(const mg_sensor& p, float voxel_m, int32_t wd, int32_t hd, HostCam* out) {
    if (!(voxel_m > 0.0f) || !(p.range_m > 0.0f) || !(p.fov_h_deg > 0.0f) || !(p.fov_h_deg < 180.0f) ||
        !(p.fov_v_deg > 0.0f) || !(p.fov_v_deg < 180.0f) || p.yaw_bins < 1)
        return mgb::set_error(MG_E_INVALID, "interval camera: invalid sensor or voxel size");
    const double wdb = (double)p.yaw_bins * (double)p.fov_h_deg / 360.0;
    const long w = std::lround(wdb);
    if (w < 1 || std::fabs(wdb - (double)w) > 1e-6)
        return mgb::set_error(MG_E_INVALID, "interval camera: yaw_bins * fov_h / 360 is not an integer");
    const double deg = M_PI / 180.0;
    const double th = std::tan((double)p.fov_h_deg * 0.5 * deg);
    const double tv = std::tan((double)p.fov_v_deg * 0.5 * deg);
    if (wd <= 0) {
        const double x = std::ceil(2.0 * (double)p.range_m * th / (double)voxel_m);
        if (!(x >= 1.0 && x <= (double)kMaxSide))
            return mgb::set_error(MG_E_UNSUPPORTED, "interval camera: buffer wider than 4096 pixels");
        wd = (int32_t)x;
    }
    if (hd <= 0) {
        const double x = std::ceil(2.0 * (double)p.range_m * tv / (double)voxel_m);
        if (!(x >= 1.0 && x <= (double)kMaxSide))
            return mgb::set_error(MG_E_UNSUPPORTED, "interval camera: buffer taller than 4096 pixels");
        hd = (int32_t)x;
    }
    if (wd > kMaxSide || hd > kMaxSide)
        return mgb::set_error(MG_E_UNSUPPORTED, "interval camera: buffer side above 4096 pixels");
    const double cxd = (double)wd * 0.5, cyd = (double)hd * 0.5;
    const double fxd = cxd / th, fyd = cyd / tv;
    out->wd = wd;
    out->hd = hd;
    out->fx = (float)fxd;
    out->fy = (float)fyd;
    out->cx = (float)cxd;
    out->cy = (float)cyd;
    out->znear = 1.0f / 64.0f;
    out->rv = p.range_m / voxel_m;
    out->pdir.resize((size_t)wd * hd);
    for (int32_t j = 0; j < hd; ++j)
        for (int32_t i = 0; i < wd; ++i) {
            const double x = ((double)i + 0.5 - cxd) / fxd, y = ((double)j + 0.5 - cyd) / fyd;
            const double nrm = std::sqrt(x * x + y * y + 1.0);
            out->pdir[(size_t)j * wd + i] =
                make_float4((float)snap(x / nrm), (float)snap(y / nrm), (float)(1.0 / nrm), 0.0f);
        }
    out->cs.resize(p.yaw_bins);
    for (int32_t k = 0; k < p.yaw_bins; ++k) {
        const double psi =
            ((double)p.az_offset_deg + ((double)k + 0.5 * (double)w) * 360.0 / (double)p.yaw_bins) * deg;
        out->cs[k] = make_float2((float)snap(std::cos(psi)), (float)snap(std::sin(psi)));
    }
    return MG_OK;
}

// Per-tree device state of the interval mode, made on the first call.
struct State {
    int32_t wd = 0, hd = 0;
    void* block = nullptr;   // pdir | cs | dpin | winv
    Cam cam{};
};

std::mutex g_mu;
std::map<mg_tree, State> g_state;
int32_t g_cap = kIvlCap;     // union components held per ray (window size)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int fail_hip(hipError_t e, const char* what) {
    return mgb::set_error(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, what);
}

}  // namespace mgi

namespace mgb {
void forget_interval(mg_tree t) {
    std::lock_guard<std::mutex> lk(mgi::g_mu);
    auto it = mgi::g_state.find(t);
    if (it == mgi::g_state.end()) return;
    (void)hipFree(it->second.block);
    mgi::g_state.erase(it);
}
}  // namespace mgb

extern "C" int mg_interval_config(int32_t cap) {
    if (cap == 0 || cap < -1 || cap > mgi::kIvlCap)
        return mgb::set_error(MG_E_INVALID, "interval capacity outside 1..16 (or -1)");
    std::lock_guard<std::mutex> lk(mgi::g_mu);
    mgi::g_cap = cap < 0 ? mgi::kIvlCap : cap;
    return MG_OK;
}

extern "C" int mg_interval_tables(const mg_sensor* sensor, float voxel_m, int32_t wd, int32_t hd, int32_t* wh,
                                  float* intr, float* pdir, float* cs) {
    if (!sensor || !wh) return mgb::set_error(MG_E_INVALID, "sensor/wh is NULL");
    mgi::HostCam H;
    int rc = mgi::build_camera(*sensor, voxel_m, wd, hd, &H);
    if (rc != MG_OK) return rc;
    wh[0] = H.wd;
    wh[1] = H.hd;
    if (intr) {
        const float v[6] = {H.fx, H.fy, H.cx, H.cy, H.znear, H.rv};
        std::memcpy(intr, v, sizeof(v));
    }
    if (pdir)
        for (size_t i = 0; i < H.pdir.size(); ++i) {
            pdir[3 * i] = H.pdir[i].x;
            pdir[3 * i + 1] = H.pdir[i].y;
            pdir[3 * i + 2] = H.pdir[i].z;
        }
    if (cs)
        for (size_t k = 0; k < H.cs.size(); ++k) {
            cs[2 * k] = H.cs[k].x;
            cs[2 * k + 1] = H.cs[k].y;
        }
    return MG_OK;
}

extern "C" int mg_eval_interval(mg_tree t, void* hip_stream, int32_t wd, int32_t hd, uint32_t* gain,
                                int32_t* yaw_bin, float* depth) {
    using namespace mgi;
    if (!t || !gain || !yaw_bin) return mgb::set_error(MG_E_INVALID, "tree/gain/yaw_bin is NULL");
    mgb::TreeView v;
    int rc = mgb::tree_view(t, &v);
    if (rc != MG_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != v.device) return mgb::set_error(MG_E_INVALID, "the tree lives on another device");
    HostCam H;
    rc = build_camera(v.params, v.voxel_m, wd, hd, &H);
    if (rc != MG_OK) return rc;
    const size_t npx = (size_t)H.wd * H.hd;
    if ((size_t)v.n * npx > ((size_t)1 << 40)) return mgb::set_error(MG_E_UNSUPPORTED, "interval buffers too large");
    hipStream_t s = (hipStream_t)hip_stream;
    Cam cam{};
    int32_t cap = kIvlCap;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        cap = g_cap;
        State& st = g_state[t];
        if (!st.block || st.wd != H.wd || st.hd != H.hd) {
            if (st.block) {
                e = hipStreamSynchronize(s);      // earlier calls may still read the old buffers
                if (e != hipSuccess) return fail_hip(e, "interval state");
                (void)hipFree(st.block);
                st.block = nullptr;
            }
            const size_t o_cs = align256(sizeof(float4) * npx);
            const size_t o_d = o_cs + align256(sizeof(float2) * H.cs.size());
            const size_t o_w = o_d + align256(sizeof(float) * npx * (size_t)v.n);
            const size_t total = o_w + sizeof(float) * npx * (size_t)v.n;
            e = hipMalloc(&st.block, total);
            if (e != hipSuccess) {
                st.block = nullptr;
                return fail_hip(e, "interval buffers");
            }
            char* base = (char*)st.block;
            e = hipMemcpy(base, H.pdir.data(), sizeof(float4) * npx, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(base + o_cs, H.cs.data(), sizeof(float2) * H.cs.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail_hip(e, "interval tables");
            st.wd = H.wd;
            st.hd = H.hd;
            st.cam.pdir = (const float4*)base;
            st.cam.cs = (const float2*)(base + o_cs);
            st.cam.dpin = (float*)(base + o_d);
            st.cam.winv = (float*)(base + o_w);
            st.cam.wd = H.wd;
            st.cam.hd = H.hd;
            st.cam.npx = (int32_t)npx;
            st.cam.fx = H.fx;
            st.cam.fy = H.fy;
            st.cam.cx = H.cx;
            st.cam.cy = H.cy;
            st.cam.znear = H.znear;
            st.cam.rv = H.rv;
        }
        cam = st.cam;
    }
    const SensorDev& S = *v.sd;
    const TreeDev& Tr = *v.td;
    e = launch_zero_u32(Tr.bins, (size_t)2 * S.B * v.n, s);
    if (e != hipSuccess) return fail_hip(e, "interval bins");
    const int32_t tiles = (S.R + kIvlThreads - 1) / kIvlThreads;
    const int32_t rtiles = (int32_t)((npx + kIvlThreads - 1) / kIvlThreads);
    for (int32_t d = 0; d < v.levels; ++d) {
        const int32_t b = (*v.level_ptr)[d], cnt = (*v.level_ptr)[d + 1] - b;
        if (cnt <= 0) continue;
        const int32_t* nodes = Tr.level_nodes + b;
        hipLaunchKernelGGL(k_ivl_trace, dim3((unsigned)cnt * (unsigned)tiles), dim3(kIvlThreads), 0, s, *v.map, S, Tr,
                           cam, nodes, (const int32_t*)yaw_bin, tiles, cap);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_finish(S, Tr, nodes, cnt, true, gain, yaw_bin, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_ivl_render, dim3((unsigned)cnt * (unsigned)rtiles), dim3(kIvlThreads), 0, s, *v.map,
                               cam, Tr, nodes, (const int32_t*)yaw_bin, rtiles);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return fail_hip(e, "interval level");
    }
    if (depth) {
        e = hipMemcpyAsync(depth, cam.dpin, sizeof(float) * npx * (size_t)v.n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail_hip(e, "interval depth copy");
    }
    return MG_OK;
}
