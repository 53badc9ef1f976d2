// Host side of the C ABI declared in include/mg.h: validation, device
// layouts, sensor tables and launch sequencing.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mg.h"
#include "mg_batch.h"
#include "mg_internal.h"

using namespace mgk;

// ---------------------------------------------------------------- errors

static thread_local std::string t_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                      \
    } while (0)

extern "C" const char* mg_last_error(void) { return t_err.c_str(); }

// ---------------------------------------------------------------- sensor tables

namespace {

struct SensorKey {
    int32_t n_az, n_el, bins;
    float fov_h, fov_v, range, az_off;
    int device;
    bool operator<(const SensorKey& o) const {
        return std::tie(n_az, n_el, bins, fov_h, fov_v, range, az_off, device) <
               std::tie(o.n_az, o.n_el, o.bins, o.fov_h, o.fov_v, o.range, o.az_off, o.device);
    }
};

struct HostTables {
    int32_t W = 0, H = 0, B = 0, w = 0, WB = 0;
    double az0 = 0.0, fov_v = 0.0;         // radians: column 0's left boundary, vertical field of view
    std::vector<float> dir, inv, bv, ts;   // dir/inv [R*3], bv [W*2], ts [H+1]
    std::vector<int32_t> bins, c0;
    // pixel-guess tables (see SensorDev)
    std::vector<uint16_t> lut_col, lut_row;
    float lut_col_scale = 0.f, lut_row_lo = 0.f, lut_row_scale = 0.f;
};

double snap_small(double x) { return std::fabs(x) < 1e-9 ? 0.0 : x; }

// Validates a sensor and derives the window geometry. Column c's centre is at
// az_offset + (c + 1/2) 360/W degrees, its bin the one holding that centre,
// bin(c) = floor((2c+1) B / (2W)); window k holds the w_buf columns whose
// centres fall in bins k..k+w-1, the first being ceil((2kW - B)/(2B)) mod W.
int check_sensor(const mg_sensor* s, int32_t* w_out, int32_t* wb_out) {
    if (!s) return fail(MG_E_INVALID, "sensor is NULL");
    if (s->n_az < 1 || s->n_el < 1 || s->yaw_bins < 1)
        return fail(MG_E_INVALID, "sensor sizes must be positive");
    if (!(s->fov_h_deg > 0.0f) || !(s->fov_v_deg > 0.0f) || !(s->fov_v_deg < 180.0f) || !(s->range_m > 0.0f) ||
        !std::isfinite(s->az_offset_deg))
        return fail(MG_E_INVALID, "sensor angles/range out of range");
    double wd = (double)s->yaw_bins * (double)s->fov_h_deg / 360.0;
    long w = std::lround(wd);
    if (w < 1 || std::fabs(wd - (double)w) > 1e-6)
        return fail(MG_E_INVALID, "yaw_bins * fov_h / 360 must be an integer >= 1");
    if (2 * w >= s->yaw_bins) return fail(MG_E_INVALID, "a yaw window must span less than 180 degrees");
    if (((long)s->n_az * w) % s->yaw_bins != 0)
        return fail(MG_E_INVALID, "n_az * window_bins must be a multiple of yaw_bins");
    if (s->yaw_bins > kMaxBins || s->n_az > kMaxAz || s->n_el > kMaxEl || (long)s->n_az * s->n_el > (1L << 22))
        return fail(MG_E_UNSUPPORTED, "sensor larger than this library supports");
    *w_out = (int32_t)w;
    *wb_out = (int32_t)((long)s->n_az * w / s->yaw_bins);
    return MG_OK;
}

// The trigonometry of the sensor, evaluated once in double precision and
// rounded to float (components below 1e-9 in magnitude become +0).
void build_tables(const mg_sensor* s, int32_t w, int32_t wb, HostTables* T) {
    const int W = s->n_az, H = s->n_el, B = s->yaw_bins;
    T->W = W; T->H = H; T->B = B; T->w = w; T->WB = wb;
    T->dir.assign((size_t)W * H * 3, 0.f);
    T->inv.assign((size_t)W * H * 3, 0.f);
    T->bv.assign((size_t)W * 2, 0.f);
    T->ts.assign((size_t)H + 1, 0.f);
    T->bins.assign(W, 0);
    T->c0.assign(B, 0);
    const double rad = M_PI / 180.0;
    T->az0 = (double)s->az_offset_deg * rad;
    T->fov_v = (double)s->fov_v_deg * rad;
    const double step_az = 360.0 / (double)W;
    const double step_el = (double)s->fov_v_deg / (double)H;
    for (int c = 0; c < W; ++c) {
        const double az = ((double)s->az_offset_deg + ((double)c + 0.5) * step_az) * rad;
        for (int j = 0; j < H; ++j) {
            const double el = (-(double)s->fov_v_deg / 2.0 + ((double)j + 0.5) * step_el) * rad;
            const double v[3] = {std::cos(el) * std::cos(az), std::cos(el) * std::sin(az), std::sin(el)};
            const size_t r = (size_t)c * H + j;
            for (int a = 0; a < 3; ++a) {
                const float f = (float)snap_small(v[a]);
                T->dir[3 * r + a] = f;
                T->inv[3 * r + a] = f != 0.0f ? 1.0f / f : 0.0f;
            }
        }
        const double beta = ((double)s->az_offset_deg + (double)c * step_az) * rad;
        T->bv[2 * c] = (float)snap_small(std::cos(beta));
        T->bv[2 * c + 1] = (float)snap_small(std::sin(beta));
        T->bins[c] = (int32_t)(((long)(2 * c + 1) * B) / (2L * W));
    }
    for (int j = 0; j <= H; ++j) {
        const double e = (-(double)s->fov_v_deg / 2.0 + (double)j * step_el) * rad;
        const double t = snap_small(std::tan(e));
        T->ts[j] = (float)(t * std::fabs(t));
    }
    for (int k = 0; k < B; ++k) {
        const long num = 2L * k * W - B, den = 2L * B;
        const long first = num >= 0 ? (num + den - 1) / den : 0;
        T->c0[k] = (int32_t)(first % W);
    }
    // Column guess: pseudo-angle p of a direction theta degrees past the window's
    // left boundary, p = t/(1+t) with t = tan(theta) below 90 degrees and
    // 2 - p(180 - theta) above; monotone in theta and cheap on the device.
    auto pseudo = [](double th) {
        if (th >= 90.0) {
            const double t = std::tan((180.0 - th) * M_PI / 180.0);
            return 2.0 - t / (1.0 + t);
        }
        const double t = std::tan(th * M_PI / 180.0);
        return t / (1.0 + t);
    };
    auto unpseudo = [](double p) {
        if (p <= 1.0) return std::atan2(p, 1.0 - p) * 180.0 / M_PI;
        const double q = 2.0 - p;
        return 180.0 - std::atan2(q, 1.0 - q) * 180.0 / M_PI;
    };
    const double fov_h = (double)wb * step_az;
    const double p_end = pseudo(fov_h);
    // the smallest table (from 4 entries per column, doubling up to 4096) in
    // which no bucket spans more than one column boundary
    int ncol = std::max(1, std::min(4096, 4 * wb));
    for (;;) {
        T->lut_col.assign(ncol, 0);
        bool fine = true;
        long prev = 0;
        for (int i = 0; i <= ncol; ++i) {
            const double th = unpseudo((double)i * p_end / (double)ncol);
            const long c = std::min<long>(std::max<long>((long)std::floor(th / step_az), 0), wb - 1);
            if (i < ncol) T->lut_col[i] = (uint16_t)c;
            if (i > 0 && c - prev > 1) fine = false;
            prev = c;
        }
        if (fine || ncol >= 4096) break;
        ncol = std::min(4096, ncol * 2);
    }
    T->lut_col_scale = (float)((double)ncol / p_end);
    // Row guess: elevation tangent, uniform table between the band's limits.
    const double half = (double)s->fov_v_deg / 2.0;
    const double t_lo = std::tan(-half * M_PI / 180.0), t_hi = std::tan(half * M_PI / 180.0);
    int nrow = std::max(1, std::min(4096, 4 * H));
    for (;;) {
        T->lut_row.assign(nrow, 0);
        bool fine = true;
        long prev = 0;
        for (int i = 0; i <= nrow; ++i) {
            const double el = std::atan(t_lo + (double)i * (t_hi - t_lo) / (double)nrow) * 180.0 / M_PI;
            const long r = std::min<long>(std::max<long>((long)std::floor((el + half) / step_el), 0), H - 1);
            if (i < nrow) T->lut_row[i] = (uint16_t)r;
            if (i > 0 && r - prev > 1) fine = false;
            prev = r;
        }
        if (fine || nrow >= 4096) break;
        nrow = std::min(4096, nrow * 2);
    }
    T->lut_row_lo = (float)t_lo;
    T->lut_row_scale = (float)((double)nrow / (t_hi - t_lo));
}

// Device copy of one sensor's tables, shared by all trees with that sensor on
// that device (reference counted).
struct SensorRes {
    SensorKey key;
    int refs = 0;
    HostTables host;
    float4 *d4 = nullptr, *iv4 = nullptr;
    int32_t *bins = nullptr, *c0 = nullptr;
    float2* bv = nullptr;
    float* ts = nullptr;
    uint16_t* luts = nullptr;   // lut_col then lut_row
    size_t bytes = 0;
};

std::mutex g_sensor_mu;
std::map<SensorKey, SensorRes*> g_sensors;

void free_sensor(SensorRes* r) {
    (void)hipFree(r->d4); (void)hipFree(r->iv4); (void)hipFree(r->bins); (void)hipFree(r->c0); (void)hipFree(r->bv); (void)hipFree(r->ts);
    (void)hipFree(r->luts);
    delete r;
}

int acquire_sensor(const mg_sensor* s, hipStream_t stream, SensorRes** out) {
    int32_t w, wb;
    int rc = check_sensor(s, &w, &wb);
    if (rc != MG_OK) return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    SensorKey key{s->n_az, s->n_el, s->yaw_bins, s->fov_h_deg, s->fov_v_deg, s->range_m, s->az_offset_deg, dev};
    std::lock_guard<std::mutex> lk(g_sensor_mu);
    auto it = g_sensors.find(key);
    if (it != g_sensors.end()) {
        it->second->refs++;
        *out = it->second;
        return MG_OK;
    }
    std::unique_ptr<SensorRes> r(new (std::nothrow) SensorRes());
    if (!r) return fail(MG_E_NOMEM, "host allocation failed");
    r->key = key;
    build_tables(s, w, wb, &r->host);
    const HostTables& T = r->host;
    const size_t R = (size_t)T.W * T.H;
    std::vector<float4> d4(R), iv4(R);
    for (size_t i = 0; i < R; ++i) {
        d4[i] = make_float4(T.dir[3 * i], T.dir[3 * i + 1], T.dir[3 * i + 2], 0.f);
        iv4[i] = make_float4(T.inv[3 * i], T.inv[3 * i + 1], T.inv[3 * i + 2], 0.f);
    }
    auto cleanup = [&]() { SensorRes* p = r.release(); free_sensor(p); };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&r->d4, R * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(&r->iv4, R * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(&r->bins, T.W * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&r->c0, T.B * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&r->bv, T.W * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&r->ts, (T.H + 1) * sizeof(float));
    const size_t nlut = T.lut_col.size() + T.lut_row.size();
    std::vector<uint16_t> luts(T.lut_col);
    luts.insert(luts.end(), T.lut_row.begin(), T.lut_row.end());
    if (e == hipSuccess) e = hipMalloc(&r->luts, nlut * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpyAsync(r->luts, luts.data(), nlut * sizeof(uint16_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d4, d4.data(), R * sizeof(float4), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->iv4, iv4.data(), R * sizeof(float4), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->bins, T.bins.data(), T.W * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->c0, T.c0.data(), T.B * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->bv, T.bv.data(), T.W * sizeof(float2), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->ts, T.ts.data(), (T.H + 1) * sizeof(float), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, "sensor upload: %s", hipGetErrorString(e));
    }
    r->bytes = R * 2 * sizeof(float4) + T.W * (sizeof(int32_t) + sizeof(float2)) + T.B * sizeof(int32_t) +
               (T.H + 1) * sizeof(float);
    r->refs = 1;
    SensorRes* p = r.release();
    g_sensors[key] = p;
    *out = p;
    return MG_OK;
}

void release_sensor(SensorRes* r) {
    std::lock_guard<std::mutex> lk(g_sensor_mu);
    if (--r->refs == 0) {
        g_sensors.erase(r->key);
        free_sensor(r);
    }
}

SensorDev sensor_dev(const SensorRes* r, float rv) {
    const HostTables& T = r->host;
    SensorDev sd;
    sd.d4 = r->d4; sd.iv4 = r->iv4; sd.bin_of_col = r->bins; sd.bv = r->bv; sd.ts = r->ts; sd.c0_of_win = r->c0;
    sd.W = T.W; sd.H = T.H; sd.B = T.B; sd.w = T.w; sd.WB = T.WB;
    sd.R = T.W * T.H;
    sd.nrb = (T.H + kRayBlockRows - 1) / kRayBlockRows;
    sd.n_blocks = (T.W + kRayBlockCols - 1) / kRayBlockCols * sd.nrb;
    sd.T = (sd.n_blocks * 64 + kThreads - 1) / kThreads;
    sd.tcols = (T.WB + kTileCols - 1) / kTileCols;
    sd.trows = (T.H + kTileRows - 1) / kTileRows;
    sd.n_tiles = sd.tcols * sd.trows;
    sd.az0 = (float)T.az0;
    sd.daz_inv = (float)((double)T.W / (2.0 * M_PI));
    sd.el0 = (float)(-T.fov_v / 2.0);
    sd.del_inv = (float)((double)T.H / T.fov_v);
    sd.rv = rv;
    sd.rv2 = rv * rv;
    sd.lut_col = r->luts;
    sd.lut_row = r->luts + T.lut_col.size();
    sd.n_lut_col = (int32_t)T.lut_col.size();
    sd.n_lut_row = (int32_t)T.lut_row.size();
    sd.lut_col_scale = T.lut_col_scale;
    sd.lut_row_lo = T.lut_row_lo;
    sd.lut_row_scale = T.lut_row_scale;
    return sd;
}

}  // namespace

extern "C" int mg_sensor_tables(const mg_sensor* sensor, float* dir, float* inv, float* bv, float* ts, int32_t* bins,
                                int32_t* c0) {
    int32_t w, wb;
    int rc = check_sensor(sensor, &w, &wb);
    if (rc != MG_OK) return rc;
    HostTables T;
    build_tables(sensor, w, wb, &T);
    if (dir) std::memcpy(dir, T.dir.data(), T.dir.size() * sizeof(float));
    if (inv) std::memcpy(inv, T.inv.data(), T.inv.size() * sizeof(float));
    if (bv) std::memcpy(bv, T.bv.data(), T.bv.size() * sizeof(float));
    if (ts) std::memcpy(ts, T.ts.data(), T.ts.size() * sizeof(float));
    if (bins) std::memcpy(bins, T.bins.data(), T.bins.size() * sizeof(int32_t));
    if (c0) std::memcpy(c0, T.c0.data(), T.c0.size() * sizeof(int32_t));
    return MG_OK;
}

// ---------------------------------------------------------------- maps

struct mg_map_s {
    MapDev dev{};
    uint8_t* bricks = nullptr;
    float voxel_m = 0.f;
    float origin[3] = {0, 0, 0};
    int device = 0;
    size_t bytes = 0;
    std::atomic<int> trees{0};
};

namespace {

int32_t bricks_for(int32_t n) {     // power of two holding at least n + 1 voxels
    int32_t nb = 1;
    while (nb * 8 < n + 1) nb *= 2;
    return nb;
}

// Host-only validation of a map's geometry (no device call).
int check_geometry(int32_t nx, int32_t ny, int32_t nz, float voxel_m, const float origin_m[3]) {
    if (!origin_m) return fail(MG_E_INVALID, "origin is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 8192 || ny > 8192 || nz > 8192)
        return fail(MG_E_INVALID, "grid dims must be in [1, 8192]");
    if (!(voxel_m > 0.0f) || !std::isfinite(voxel_m)) return fail(MG_E_INVALID, "voxel_m must be positive");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(origin_m[a])) return fail(MG_E_INVALID, "origin must be finite");
    if ((size_t)nx * ny * nz >= (1ull << 32)) return fail(MG_E_INVALID, "grid has 2^32 voxels or more");
    const int32_t nbx = bricks_for(nx), nby = bricks_for(ny), nbz = bricks_for(nz);
    if ((size_t)nbx * nby * nbz * 512u > (1ull << 32) - 256)
        return fail(MG_E_UNSUPPORTED, "bricked grid (%d x %d x %d bricks) exceeds 2^32 - 256 bytes", nbx, nby, nbz);
    return MG_OK;
}

// Lays out the padded bricked grid (power-of-two brick counts holding at
// least n + 1 voxels per axis) and allocates it.
int map_alloc(int32_t nx, int32_t ny, int32_t nz, float voxel_m, const float origin_m[3],
              std::unique_ptr<mg_map_s>* out) {
    int rc0 = check_geometry(nx, ny, nz, voxel_m, origin_m);
    if (rc0 != MG_OK) return rc0;
    const int32_t nbx = bricks_for(nx), nby = bricks_for(ny), nbz = bricks_for(nz);
    const size_t padded = (size_t)nbx * nby * nbz * 512u;
    std::unique_ptr<mg_map_s> m(new (std::nothrow) mg_map_s());
    if (!m) return fail(MG_E_NOMEM, "host allocation failed");
    HIP_TRY(hipGetDevice(&m->device));
    const size_t n_mbricks = (size_t)((nx + 7) / 8) * ((ny + 7) / 8) * ((nz + 7) / 8);
    hipError_t e = hipMalloc(&m->bricks, padded + n_mbricks);      // the grid, then the brick flags
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, "map allocation: %s", hipGetErrorString(e));
    m->dev.bricks = m->bricks;
    m->dev.nx = nx; m->dev.ny = ny; m->dev.nz = nz;
    m->dev.nbx = nbx; m->dev.nby = nby; m->dev.nbz = nbz;
    auto log2i = [](int32_t v) { uint32_t l = 0; while ((1 << l) < v) ++l; return l; };
    m->dev.xm = (uint32_t)(8 * nbx - 1) & ~7u;
    m->dev.ym = (uint32_t)(8 * nby - 1) & ~7u;
    m->dev.zm = (uint32_t)(8 * nbz - 1) & ~7u;
    m->dev.shy = 6u + log2i(nbx);
    m->dev.shz = 6u + log2i(nbx) + log2i(nby);
    m->dev.outside = voxel_addr(8 * nbx - 1, 0, 0, m->dev);
    m->dev.mbx = (uint32_t)(nx + 7) / 8u;
    m->dev.mby = (uint32_t)(ny + 7) / 8u;
    m->dev.mbz = (uint32_t)(nz + 7) / 8u;
    m->dev.mask_words = 16u * m->dev.mbx * m->dev.mby * m->dev.mbz;    // < 2^32 / 32 (voxels < 2^32)
    m->dev.build_slots = 8u * ((m->dev.mbx + 1u) / 2u) * ((m->dev.mby + 1u) / 2u) * ((m->dev.mbz + 1u) / 2u);
    m->dev.brick_unk = m->bricks + padded;
    m->voxel_m = voxel_m;
    for (int a = 0; a < 3; ++a) m->origin[a] = origin_m[a];
    m->bytes = padded + n_mbricks;
    *out = std::move(m);
    return MG_OK;
}

}  // namespace

extern "C" int mg_map_create(const uint8_t* states, int32_t nx, int32_t ny, int32_t nz, float voxel_m,
                             const float origin_m[3], void* hip_stream, mg_map* out) {
    if (!out) return fail(MG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!states) return fail(MG_E_INVALID, "states is NULL");
    int rc = check_geometry(nx, ny, nz, voxel_m, origin_m);
    if (rc != MG_OK) return rc;
    const size_t nvox = (size_t)nx * ny * nz;
    for (size_t i = 0; i < nvox; ++i)
        if (states[i] > 2) return fail(MG_E_INVALID, "voxel %zu has state %u (expected 0, 1 or 2)", i, states[i]);
    std::unique_ptr<mg_map_s> m;
    rc = map_alloc(nx, ny, nz, voxel_m, origin_m, &m);
    if (rc != MG_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    uint8_t* dense = nullptr;
    hipError_t e = hipMalloc(&dense, nvox);
    if (e == hipSuccess) e = hipMemcpyAsync(dense, states, nvox, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_brick(dense, m->bricks, m->dev, s);
    if (e == hipSuccess) e = launch_brick_flags(m->dev, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dense);
    if (e != hipSuccess) {
        (void)hipFree(m->bricks);
        return fail(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, "map upload: %s", hipGetErrorString(e));
    }
    *out = m.release();
    return MG_OK;
}

extern "C" int mg_map_create_tsdf(const float* distance, const float* weight, int32_t nx, int32_t ny, int32_t nz,
                                  float voxel_m, const float origin_m[3], float surface_m, float min_weight,
                                  void* hip_stream, mg_map* out) {
    if (!out) return fail(MG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!distance || !weight) return fail(MG_E_INVALID, "distance/weight is NULL");
    if (!std::isfinite(surface_m) || !std::isfinite(min_weight))
        return fail(MG_E_INVALID, "surface_m and min_weight must be finite");
    int rc = check_geometry(nx, ny, nz, voxel_m, origin_m);
    if (rc != MG_OK) return rc;
    std::unique_ptr<mg_map_s> m;
    rc = map_alloc(nx, ny, nz, voxel_m, origin_m, &m);
    if (rc != MG_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_fill_outside(m->dev, s);
    // (the whole-grid conversion takes the bricks' summaries itself)
    if (e == hipSuccess) e = launch_tsdf_grid(distance, weight, m->dev, surface_m, min_weight, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(m->bricks);
        return fail(MG_E_DEVICE, "TSDF conversion: %s", hipGetErrorString(e));
    }
    *out = m.release();
    return MG_OK;
}

extern "C" int mg_map_update_tsdf(mg_map map, void* hip_stream, const float* distance, const float* weight,
                                  const int32_t lo[3], const int32_t size[3], float surface_m, float min_weight) {
    if (!map || !lo || !size) return fail(MG_E_INVALID, "NULL argument");
    if ((!distance || !weight) && (int64_t)size[0] * size[1] * size[2] != 0)
        return fail(MG_E_INVALID, "distance/weight is NULL");
    if (!std::isfinite(surface_m) || !std::isfinite(min_weight))
        return fail(MG_E_INVALID, "surface_m and min_weight must be finite");
    const int32_t dims[3] = {map->dev.nx, map->dev.ny, map->dev.nz};
    bool whole = true;
    for (int a = 0; a < 3; ++a) {
        if (lo[a] < 0 || size[a] < 0 || (int64_t)lo[a] + size[a] > dims[a])
            return fail(MG_E_INVALID, "box [%d, %d) on axis %d leaves the grid (%d)", lo[a], lo[a] + size[a], a, dims[a]);
        whole = whole && lo[a] == 0 && size[a] == dims[a];
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != map->device) return fail(MG_E_INVALID, "the map lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    // (the whole-grid conversion takes the bricks' summaries itself; a box needs the pass)
    if (whole) {
        HIP_TRY(launch_tsdf_grid(distance, weight, map->dev, surface_m, min_weight, s));
    } else {
        HIP_TRY(launch_tsdf_box(distance, weight, map->dev, lo, size, surface_m, min_weight, s));
        HIP_TRY(launch_brick_flags(map->dev, s));
    }
    return MG_OK;
}

extern "C" int mg_map_update(mg_map map, void* hip_stream, const uint32_t* voxel_ids, const uint8_t* states,
                             int32_t count, uint32_t* rejected) {
    if (!map || count < 0 || (count > 0 && (!voxel_ids || !states))) return fail(MG_E_INVALID, "bad update arguments");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != map->device) return fail(MG_E_INVALID, "the map lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    if (rejected) HIP_TRY(launch_zero_u32(rejected, 1, s));
    HIP_TRY(launch_map_scatter(voxel_ids, states, (uint32_t)count, map->dev, rejected, s));
    HIP_TRY(launch_brick_flags(map->dev, s));
    return MG_OK;
}

extern "C" int mg_map_read(mg_map map, void* hip_stream, uint8_t* states) {
    if (!map || !states) return fail(MG_E_INVALID, "map/states is NULL");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != map->device) return fail(MG_E_INVALID, "the map lives on another device");
    HIP_TRY(launch_unbrick(map->dev, states, (hipStream_t)hip_stream));
    return MG_OK;
}

extern "C" int mg_map_read_marked(mg_map map, void* hip_stream, uint8_t* bytes) {
    if (!map || !bytes) return fail(MG_E_INVALID, "map/bytes is NULL");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != map->device) return fail(MG_E_INVALID, "the map lives on another device");
    HIP_TRY(launch_unbrick(map->dev, bytes, (hipStream_t)hip_stream, true));
    return MG_OK;
}

extern "C" int mg_map_destroy(mg_map map) {
    if (!map) return fail(MG_E_INVALID, "map is NULL");
    if (map->trees.load() != 0)
        return fail(MG_E_BUSY, "%d trees or server requests still use this map", map->trees.load());
    (void)hipFree(map->bricks);
    delete map;
    return MG_OK;
}

// ---------------------------------------------------------------- trees

struct mg_tree_s {
    mg_map map = nullptr;
    SensorRes* sensor = nullptr;
    mg_sensor params{};
    int32_t n = 0;
    int32_t levels = 0;
    std::vector<int32_t> level_ptr;       // host copy [levels+1]
    std::vector<int32_t> level_nodes_h;   // host copy [n]
    std::vector<int32_t> mask_level_ptr;  // host copy [levels+1]: nodes with children, by level
    std::vector<int32_t> mask_nodes_h;    // host copy
    std::vector<int32_t> parent_h;
    std::vector<int32_t> depth_h;
    // device
    void* block = nullptr;                // one allocation for all node data
    bool owns_block = true;               // false when placed in a server's arena
    TreeDev dev{};
    SensorDev sd{};
    size_t bytes = 0;
    int device = 0;
    uint32_t* scratch_gain = nullptr;     // device outputs used when the caller gives none
    int32_t* scratch_yaw = nullptr;
};

namespace mgb {

// Host side of a tree upload: validation and every array the device needs.
struct HostTree {
    int32_t n = 0, maxd = 0, n_masks = 0;
    std::vector<float4> q4, pm;
    std::vector<int32_t> depth, level_ptr, level_nodes, anc_ptr, anc_ids, child_ptr, child_ids, parent;
    // path masks: slot per node (-1 for leaves), nodes with children by level
    std::vector<int32_t> mask_slot, mask_level_ptr, mask_nodes;
    // device block layout
    size_t o_q4 = 0, o_pm = 0, o_ap = 0, o_ai = 0, o_ln = 0, o_cp = 0, o_ci = 0, o_c0 = 0, o_g = 0, o_y = 0, o_bins = 0,
           o_dpan = 0, o_ms = 0, o_mn = 0, o_masks = 0, o_tm = 0, o_mc = 0, total = 0;
};

}  // namespace mgb

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Validates the tree against the map and sensor (parent[0] = -1, 0 <= parent[i] < i,
// depth <= 64, every node inside the map, q = (p - origin) / voxel in float),
// builds levels (ids ascending within a level), nearest-first ancestor lists
// and child lists, and lays out the device block.
int prepare_tree(mg_map map, const float* pos_m, const int32_t* parent, int32_t n, const mg_sensor* sensor,
                 mgb::HostTree* H) {
    if (!map || !pos_m || !parent) return fail(MG_E_INVALID, "map/pos/parent is NULL");
    if (n < 1) return fail(MG_E_INVALID, "a tree needs at least one node");
    if (n > (1 << 24)) return fail(MG_E_UNSUPPORTED, "more than 2^24 nodes");
    int32_t w, wb;
    int rc = check_sensor(sensor, &w, &wb);
    if (rc != MG_OK) return rc;
    if (parent[0] != -1) return fail(MG_E_INVALID, "parent[0] must be -1");
    H->n = n;
    H->parent.assign(parent, parent + n);
    H->depth.assign(n, 0);
    for (int32_t i = 1; i < n; ++i) {
        if (parent[i] < 0 || parent[i] >= i) return fail(MG_E_INVALID, "parent[%d] = %d must be in [0, %d)", i, parent[i], i);
        H->depth[i] = H->depth[parent[i]] + 1;
        if (H->depth[i] > kMaxAnc) return fail(MG_E_INVALID, "node %d is deeper than %d", i, kMaxAnc);
    }
    H->q4.resize(n);
    H->pm.resize(n);
    const int32_t dims[3] = {map->dev.nx, map->dev.ny, map->dev.nz};
    for (int32_t i = 0; i < n; ++i) {
        float qv[3];
        for (int a = 0; a < 3; ++a) {
            const float v = (pos_m[3 * i + a] - map->origin[a]) / map->voxel_m;
            if (!(v >= 0.0f) || !(v < (float)dims[a]) || (int32_t)std::floor(v) >= dims[a])
                return fail(MG_E_INVALID, "node %d lies outside the map", i);
            qv[a] = v;
        }
        H->q4[i] = make_float4(qv[0], qv[1], qv[2], 0.f);
        H->pm[i] = make_float4(pos_m[3 * i], pos_m[3 * i + 1], pos_m[3 * i + 2], 0.f);
    }
    H->maxd = 0;
    for (int32_t i = 0; i < n; ++i) H->maxd = std::max(H->maxd, H->depth[i]);
    H->level_ptr.assign(H->maxd + 2, 0);
    H->level_nodes.assign(n, 0);
    for (int32_t i = 0; i < n; ++i) H->level_ptr[H->depth[i] + 1]++;
    for (int32_t d = 0; d <= H->maxd; ++d) H->level_ptr[d + 1] += H->level_ptr[d];
    {
        std::vector<int32_t> fill(H->level_ptr.begin(), H->level_ptr.end() - 1);
        for (int32_t i = 0; i < n; ++i) H->level_nodes[fill[H->depth[i]]++] = i;
    }
    H->anc_ptr.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) H->anc_ptr[i + 1] = H->anc_ptr[i] + H->depth[i];
    H->anc_ids.assign((size_t)H->anc_ptr[n] + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t k = H->anc_ptr[i];
        for (int32_t a = parent[i]; a >= 0; a = parent[a]) H->anc_ids[k++] = a;
    }
    H->child_ptr.assign(n + 1, 0);
    H->child_ids.assign((size_t)n, 0);
    for (int32_t i = 1; i < n; ++i) H->child_ptr[parent[i] + 1]++;
    for (int32_t i = 0; i < n; ++i) H->child_ptr[i + 1] += H->child_ptr[i];
    {
        std::vector<int32_t> fill(H->child_ptr.begin(), H->child_ptr.end() - 1);
        for (int32_t i = 1; i < n; ++i) H->child_ids[fill[parent[i]]++] = i;
    }
    // path masks for the nodes with children, slots in level order
    H->mask_slot.assign(n, -1);
    H->mask_level_ptr.assign(H->maxd + 2, 0);
    H->mask_nodes.clear();
    for (int32_t d = 0; d <= H->maxd; ++d) {
        for (int32_t k = H->level_ptr[d]; k < H->level_ptr[d + 1]; ++k) {
            const int32_t v = H->level_nodes[k];
            if (H->child_ptr[v + 1] > H->child_ptr[v]) {
                H->mask_slot[v] = (int32_t)H->mask_nodes.size();
                H->mask_nodes.push_back(v);
            }
        }
        H->mask_level_ptr[d + 1] = (int32_t)H->mask_nodes.size();
    }
    H->n_masks = (int32_t)H->mask_nodes.size();
    const size_t R = (size_t)sensor->n_az * sensor->n_el;
    if (R * (size_t)n >= (1ull << 32)) return fail(MG_E_UNSUPPORTED, "nodes x rays = %zu exceeds 2^32 per tree", R * (size_t)n);
    // one device block: q4 | pm | anc_ptr | anc_ids | level_nodes | child_ptr | child_ids | c0 | gain | yaw | bins |
    // dpan | mask_slot | mask_nodes | masks | tile maxima | mask brick codes
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    H->o_q4 = take(sizeof(float4) * n);
    H->o_pm = take(sizeof(float4) * n);
    H->o_ap = take(sizeof(int32_t) * (n + 1));
    H->o_ai = take(sizeof(int32_t) * H->anc_ids.size());
    H->o_ln = take(sizeof(int32_t) * n);
    H->o_cp = take(sizeof(int32_t) * (n + 1));
    H->o_ci = take(sizeof(int32_t) * n);
    H->o_c0 = take(sizeof(int32_t) * n);
    H->o_g = take(sizeof(uint32_t) * n);
    H->o_y = take(sizeof(int32_t) * n);
    H->o_bins = take(sizeof(uint32_t) * 2 * sensor->yaw_bins * (size_t)n);
    H->o_dpan = take(sizeof(float) * R * (size_t)n);
    H->o_ms = take(sizeof(int32_t) * n);
    H->o_mn = take(sizeof(int32_t) * std::max<size_t>(H->mask_nodes.size(), 1));
    H->o_masks = take(sizeof(uint32_t) * (size_t)map->dev.mask_words * (size_t)H->n_masks);
    const size_t n_tiles = (size_t)((wb + kTileCols - 1) / kTileCols) * (size_t)((sensor->n_el + kTileRows - 1) / kTileRows);
    H->o_tm = take(sizeof(float) * 2 * n_tiles * (size_t)std::max(H->n_masks, 1));
    H->o_mc = take(sizeof(uint32_t) * (size_t)(map->dev.mask_words >> 4) * (size_t)std::max(H->n_masks, 1));
    H->total = off;
    return MG_OK;
}

// Copies the host arrays into `block` (at least H.total bytes) on `s` and waits
// for the copies, then builds the handle. The handle frees the block on
// destruction only when it owns it.
int finish_upload(mg_map map, const mgb::HostTree& H, const mg_sensor* sensor, hipStream_t s, void* block,
                  bool owns, mg_tree* out) {
    std::unique_ptr<mg_tree_s> t(new (std::nothrow) mg_tree_s());
    if (!t) return fail(MG_E_NOMEM, "host allocation failed");
    int rc = acquire_sensor(sensor, s, &t->sensor);
    if (rc != MG_OK) return rc;
    const int32_t n = H.n;
    char* base = (char*)block;
    auto up = [&](size_t o, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    std::vector<int32_t> zeros_c0(n, 0);
    hipError_t e = up(H.o_q4, H.q4.data(), sizeof(float4) * n);
    if (e == hipSuccess) e = up(H.o_pm, H.pm.data(), sizeof(float4) * n);
    if (e == hipSuccess) e = up(H.o_ap, H.anc_ptr.data(), sizeof(int32_t) * (n + 1));
    if (e == hipSuccess) e = up(H.o_ai, H.anc_ids.data(), sizeof(int32_t) * H.anc_ids.size());
    if (e == hipSuccess) e = up(H.o_ln, H.level_nodes.data(), sizeof(int32_t) * n);
    if (e == hipSuccess) e = up(H.o_cp, H.child_ptr.data(), sizeof(int32_t) * (n + 1));
    if (e == hipSuccess) e = up(H.o_ci, H.child_ids.data(), sizeof(int32_t) * n);
    if (e == hipSuccess) e = up(H.o_c0, zeros_c0.data(), sizeof(int32_t) * n);
    if (e == hipSuccess) e = up(H.o_ms, H.mask_slot.data(), sizeof(int32_t) * n);
    if (e == hipSuccess) e = up(H.o_mn, H.mask_nodes.data(), sizeof(int32_t) * H.mask_nodes.size());
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release_sensor(t->sensor);
        return fail(MG_E_DEVICE, "tree upload: %s", hipGetErrorString(e));
    }
    t->dev.q4 = (const float4*)(base + H.o_q4);
    t->dev.pm = (const float4*)(base + H.o_pm);
    t->dev.anc_ptr = (const int32_t*)(base + H.o_ap);
    t->dev.anc_ids = (const int32_t*)(base + H.o_ai);
    t->dev.level_nodes = (const int32_t*)(base + H.o_ln);
    t->dev.child_ptr = (const int32_t*)(base + H.o_cp);
    t->dev.child_ids = (const int32_t*)(base + H.o_ci);
    t->dev.c0 = (int32_t*)(base + H.o_c0);
    t->dev.bins = (uint32_t*)(base + H.o_bins);
    t->dev.dpan = (float*)(base + H.o_dpan);
    t->dev.mask_slot = (const int32_t*)(base + H.o_ms);
    t->dev.mask_nodes = (const int32_t*)(base + H.o_mn);
    t->dev.masks = (uint32_t*)(base + H.o_masks);
    t->dev.tmax = (float*)(base + H.o_tm);
    t->dev.mcode = (uint32_t*)(base + H.o_mc);
    t->dev.n = n;
    t->dev.anc_cap = kMaxAnc;
    t->scratch_gain = (uint32_t*)(base + H.o_g);
    t->scratch_yaw = (int32_t*)(base + H.o_y);
    t->sd = sensor_dev(t->sensor, sensor->range_m / map->voxel_m);
    if (build_lds_total(t->sd) > lds_limit()) {
        release_sensor(t->sensor);
        return fail(MG_E_UNSUPPORTED, "sensor tables need %zu bytes of LDS per workgroup, the device has %zu",
                    build_lds_total(t->sd), lds_limit());
    }
    t->map = map;
    t->params = *sensor;
    t->n = n;
    t->levels = H.maxd + 1;
    t->level_ptr = H.level_ptr;
    t->level_nodes_h = H.level_nodes;
    t->mask_level_ptr = H.mask_level_ptr;
    t->mask_nodes_h = H.mask_nodes;
    t->parent_h = H.parent;
    t->depth_h = H.depth;
    t->block = block;
    t->owns_block = owns;
    t->bytes = H.total;
    (void)hipGetDevice(&t->device);
    map->trees++;
    *out = t.release();
    return MG_OK;
}

}  // namespace

namespace mgb {
int prepare(mg_map map, const float* pos_m, const int32_t* parent, int32_t n, const mg_sensor* sensor, HostTree* H) {
    return prepare_tree(map, pos_m, parent, n, sensor, H);
}
size_t block_bytes(const HostTree& H) { return H.total; }
int upload_into(mg_map map, const HostTree& H, const mg_sensor* sensor, hipStream_t s, void* block, mg_tree* out) {
    return finish_upload(map, H, sensor, s, block, false, out);
}
void free_host_tree(HostTree* H) { delete H; }
HostTree* new_host_tree() { return new (std::nothrow) HostTree(); }
}  // namespace mgb

extern "C" int mg_tree_upload(mg_map map, const float* pos_m, const int32_t* parent, int32_t n,
                              const mg_sensor* sensor, void* hip_stream, mg_tree* out) {
    if (!out) return fail(MG_E_INVALID, "out is NULL");
    *out = nullptr;
    mgb::HostTree H;
    int rc = prepare_tree(map, pos_m, parent, n, sensor, &H);
    if (rc != MG_OK) return rc;
    void* block = nullptr;
    hipError_t e = hipMalloc(&block, H.total);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? MG_E_NOMEM : MG_E_DEVICE, "tree allocation (%zu bytes): %s", H.total,
                    hipGetErrorString(e));
    rc = finish_upload(map, H, sensor, (hipStream_t)hip_stream, block, true, out);
    if (rc != MG_OK) (void)hipFree(block);
    return rc;
}

extern "C" int mg_tree_destroy(mg_tree t) {
    if (!t) return fail(MG_E_INVALID, "tree is NULL");
    mgb::forget_tree(t);
    mgb::forget_interval(t);
    mgb::forget_exact(t);
    if (t->owns_block) (void)hipFree(t->block);
    release_sensor(t->sensor);
    t->map->trees--;
    delete t;
    return MG_OK;
}

extern "C" int32_t mg_tree_nodes(mg_tree t) { return t ? t->n : -1; }
extern "C" int32_t mg_tree_buffer_pixels(mg_tree t) { return t ? t->sd.H * t->sd.WB : -1; }
extern "C" int64_t mg_tree_footprint_bytes(mg_tree t) { return t ? (int64_t)t->bytes : -1; }

// ---------------------------------------------------------------- evaluation

namespace {

int check_device(mg_tree t) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != t->device) return fail(MG_E_INVALID, "tree lives on device %d, current device is %d", t->device, dev);
    return MG_OK;
}

// Depth-ordered evaluation: for each level, trace all its nodes' rays, select
// their windows, then build the path masks of those with children; level d+1
// reads the masks of level d.
int eval_levels(mg_tree t, hipStream_t s, uint32_t* gain, int32_t* yaw, float* depth, uint32_t* host_gain,
                int32_t* host_yaw, int32_t anc_cap = kMaxAnc) {
    TreeDev td = t->dev;
    td.anc_cap = anc_cap;
    HIP_TRY(launch_zero_u32(td.bins, (size_t)2 * t->sd.B * t->n, s));
    for (int32_t d = 0; d < t->levels; ++d) {
        const int32_t b = t->level_ptr[d], cnt = t->level_ptr[d + 1] - b;
        const int32_t* nodes = td.level_nodes + b;
        HIP_TRY(launch_trace(t->map->dev, t->sd, td, nodes, cnt, true, s));
        HIP_TRY(launch_finish(t->sd, td, nodes, cnt, true, gain, yaw, s));
        const int32_t mb = t->mask_level_ptr[d], mcnt = t->mask_level_ptr[d + 1] - mb;
        HIP_TRY(launch_mask_build(t->map->dev, t->sd, td, td.mask_nodes + mb, mcnt, s));
        if (host_gain) {
            // results of this level back to the host before the next level (Sec. IV-C)
            HIP_TRY(hipMemcpyAsync(host_gain, gain, sizeof(uint32_t) * t->n, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(host_yaw, yaw, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    if (depth) HIP_TRY(launch_depth_out(t->sd, t->dev, depth, s));
    return MG_OK;
}

}  // namespace

extern "C" int mg_eval_marginal(mg_tree t, void* hip_stream, uint32_t* gain, int32_t* yaw_bin, float* depth) {
    if (!t || !gain || !yaw_bin) return fail(MG_E_INVALID, "tree/gain/yaw_bin is NULL");
    int rc = check_device(t);
    if (rc != MG_OK) return rc;
    return eval_levels(t, (hipStream_t)hip_stream, gain, yaw_bin, depth, nullptr, nullptr);
}

extern "C" int mg_eval_single_parent(mg_tree t, void* hip_stream, uint32_t* gain, int32_t* yaw_bin, float* depth) {
    if (!t || !gain || !yaw_bin) return fail(MG_E_INVALID, "tree/gain/yaw_bin is NULL");
    int rc = check_device(t);
    if (rc != MG_OK) return rc;
    return eval_levels(t, (hipStream_t)hip_stream, gain, yaw_bin, depth, nullptr, nullptr, 1);
}

extern "C" int mg_eval_marginal_levelsync(mg_tree t, void* hip_stream, uint32_t* gain, int32_t* yaw_bin,
                                          float* depth, uint32_t* host_gain, int32_t* host_yaw_bin) {
    if (!t || !host_gain || !host_yaw_bin) return fail(MG_E_INVALID, "tree/host outputs are NULL");
    int rc = check_device(t);
    if (rc != MG_OK) return rc;
    if (!gain) gain = t->scratch_gain;
    if (!yaw_bin) yaw_bin = t->scratch_yaw;
    hipStream_t s = (hipStream_t)hip_stream;
    rc = eval_levels(t, s, gain, yaw_bin, depth, host_gain, host_yaw_bin);
    if (rc != MG_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return MG_OK;
}

extern "C" int mg_eval_absolute(mg_tree t, void* hip_stream, uint32_t* gain, int32_t* yaw_bin) {
    if (!t || !gain || !yaw_bin) return fail(MG_E_INVALID, "tree/gain/yaw_bin is NULL");
    int rc = check_device(t);
    if (rc != MG_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(launch_zero_u32(t->dev.bins, (size_t)2 * t->sd.B * t->n, s));
    HIP_TRY(launch_trace(t->map->dev, t->sd, t->dev, t->dev.level_nodes, t->n, false, s));
    HIP_TRY(launch_finish(t->sd, t->dev, t->dev.level_nodes, t->n, false, gain, yaw_bin, s));
    return MG_OK;
}

// ---------------------------------------------------------------- batch (see mg_batch.hip)

namespace mgb {
int tree_view(mg_tree t, TreeView* v) {
    v->map = &t->map->dev;
    v->sd = &t->sd;
    v->td = &t->dev;
    v->level_ptr = &t->level_ptr;
    v->level_nodes = &t->level_nodes_h;
    v->mask_level_ptr = &t->mask_level_ptr;
    v->mask_nodes = &t->mask_nodes_h;
    v->parent = &t->parent_h;
    v->depth = &t->depth_h;
    v->scratch_gain = t->scratch_gain;
    v->scratch_yaw = t->scratch_yaw;
    v->params = t->params;
    v->voxel_m = t->map->voxel_m;
    v->n = t->n;
    v->levels = t->levels;
    v->device = t->device;
    return MG_OK;
}
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
const mgk::MapDev* map_dev(mg_map m) { return &m->dev; }
void map_ref(mg_map m, int delta) { m->trees += delta; }
size_t map_voxel_count(mg_map m) { return (size_t)m->dev.nx * m->dev.ny * m->dev.nz; }
}  // namespace mgb
