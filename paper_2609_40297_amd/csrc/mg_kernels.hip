// gfx950 kernels of the marginal-gain path.
//
// Exactness: every decision (which voxels a ray visits, whether an ancestor
// sees a voxel, which window wins) is taken in IEEE binary32 with the
// operation order of the definitions below and without contraction into
// fused multiply-adds. Approximate arithmetic (hardware reciprocal and
// reciprocal square root) appears only in *estimates* of a pixel index that
// are then corrected by the exact boundary tests, so it never changes a result.
#pragma clang fp contract(off)

#include <hip/hip_ext.h>

#include "mg_internal.h"

namespace mgk {

// Global-memory views of pointers that reach a kernel through a descriptor in
// memory: the compiler then issues global (not flat) loads for them.
typedef const __attribute__((address_space(1))) uint8_t* gbytes_t;
typedef const __attribute__((address_space(1))) float* gfloats_t;
typedef const __attribute__((address_space(1))) uint32_t* gwords_t;
__device__ __forceinline__ gbytes_t as_global(const uint8_t* p) { return (gbytes_t)p; }
__device__ __forceinline__ gfloats_t as_global(const float* p) { return (gfloats_t)p; }
__device__ __forceinline__ gwords_t as_global(const uint32_t* p) { return (gwords_t)p; }

// A workgroup-uniform pointer moved to scalar registers (loads through it then
// take a scalar base and a 32-bit vector offset).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

// Wave ballot of a boolean (no widening of the predicate to an integer).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// ---------------------------------------------------------------- map layout

// Dense [nz][ny][nx] -> bricks; padding voxels (beyond the true extent) are
// set to kOutside, which ends a traversal that reaches them.
__global__ void k_brick(const uint8_t* __restrict__ dense, uint8_t* __restrict__ bricks, MapDev m) {
    const uint32_t total = (uint32_t)m.nbx * m.nby * m.nbz * 512u;
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < total; o += gridDim.x * blockDim.x) {
        uint32_t b = o >> 9, in = o & 511u;
        int32_t bx = (int32_t)(b % (uint32_t)m.nbx);
        int32_t by = (int32_t)((b / (uint32_t)m.nbx) % (uint32_t)m.nby);
        int32_t bz = (int32_t)(b / ((uint32_t)m.nbx * (uint32_t)m.nby));
        int32_t x = bx * 8 + (int32_t)(in & 7u), y = by * 8 + (int32_t)((in >> 3) & 7u),
                z = bz * 8 + (int32_t)(in >> 6);
        uint8_t v = kOutside;
        if (x < m.nx && y < m.ny && z < m.nz)
            v = dense[(size_t)x + (size_t)m.nx * ((size_t)y + (size_t)m.ny * (size_t)z)];
        bricks[o] = v;
    }
}

// Per-brick summaries, after any write of the states: brick_unk[b] says whether
// brick b holds no, some or only unknown voxels, and every unknown and free
// voxel gets the level of the largest block around it that holds its state
// only (mark_brick_row). One wave per brick, each lane reading 8 of its 512
// bytes and writing them back only if a mark changes (padding voxels past the
// grid hold kOutside, so a block that reaches past the grid is never marked).
__global__ void k_brick_flags(MapDev m) {
    const uint32_t nb = m.mask_words >> 4;
    const uint32_t lane = threadIdx.x & 63u;
    uint8_t* grid = const_cast<uint8_t*>(m.bricks);
    for (uint32_t b = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < nb; b += (gridDim.x * blockDim.x) >> 6) {
        const uint32_t bx = b % m.mbx, by = (b / m.mbx) % m.mby, bz = b / (m.mbx * m.mby);
        const uint32_t base = voxel_addr((int32_t)(bx * 8u), (int32_t)(by * 8u), (int32_t)(bz * 8u), m);
        uint64_t* p = reinterpret_cast<uint64_t*>(grid + base + lane * 8u);
        const uint64_t v = *p;
        bool any_unk, all_unk, all_free;
        const uint64_t w = mark_brick_row(v, lane, &any_unk, &all_unk, &all_free);
        if (lane == 0) m.brick_unk[b] = brick_summary(any_unk, all_unk, all_free);
        if (w != v) *p = w;
    }
}

// 16x16x16 blocks, after the bricks' summaries: a brick whose aligned block
// of 2x2x2 bricks lies in the grid's bricks and holds only wholly free (or
// only wholly unknown) bricks has its voxels marked at level 1. One thread per
// brick; the few bricks of such blocks are written by their thread, 16 bytes
// at a time.
__global__ void k_blocks16(MapDev m) {
    const uint32_t nb = m.mask_words >> 4;
    uint8_t* grid = const_cast<uint8_t*>(m.bricks);
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        const uint32_t own = m.brick_unk[b];
        const bool free_b = (own & kBrickAllFree) != 0, unk_b = (own & 3u) == kBrickAllUnknown;
        if (!free_b && !unk_b) continue;
        const uint32_t bx = b % m.mbx, by = (b / m.mbx) % m.mby, bz = b / (m.mbx * m.mby);
        const uint32_t x0 = bx & ~1u, y0 = by & ~1u, z0 = bz & ~1u;
        if (x0 + 1u >= m.mbx || y0 + 1u >= m.mby || z0 + 1u >= m.mbz) continue;
        bool all = true;
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
            const uint32_t n = (x0 + (k & 1u)) + m.mbx * ((y0 + ((k >> 1) & 1u)) + m.mby * (z0 + (k >> 2)));
            const uint32_t s = m.brick_unk[n];
            all = all && (free_b ? (s & kBrickAllFree) != 0 : (s & 3u) == kBrickAllUnknown);
        }
        if (!all) continue;
        const uint32_t base = voxel_addr((int32_t)(bx * 8u), (int32_t)(by * 8u), (int32_t)(bz * 8u), m);
        const uint32_t w = ((free_b ? kFree : kUnknown) | (1u << kLevelShift)) * 0x01010101u;
        uint4* p = reinterpret_cast<uint4*>(grid + base);        // (a brick is 512 contiguous, aligned bytes)
        for (int k = 0; k < 32; ++k) p[k] = make_uint4(w, w, w, w);
    }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------- window geometry

// A node's position (voxel units) and its window: first column and the unit
// vectors of its left and right boundaries.
struct WindowGeom {
    float qx, qy, qz;
    int32_t c0;
    float b0x, b0y;       // left boundary of the window
    float b1x, b1y;       // right boundary (left boundary of column c0 + w_buf)
};

__device__ __forceinline__ int32_t wrap(int32_t c, int32_t W) { return c >= W ? c - W : c; }

// r lies at or to the left (counter-clockwise side) of boundary direction b.
__device__ __forceinline__ bool left_of(float2 b, float rx, float ry) { return b.x * ry - b.y * rx >= 0.f; }

// ---------------------------------------------------------------- path masks

// Mask builder launch shapes (rays per workgroup of the trace kernel, bricks
// per workgroup of the builder), all compiled; shape 0 is the default.
struct Shape {
    int threads, bricks;
};
constexpr Shape kShapes[] = {{256, 64}, {128, 64}, {512, 64}, {256, 128}, {256, 32}, {256, 256}, {128, 128}, {128, 256}, {512, 128}, {128, 512}, {128, 1024}, {64, 1024}, {64, 256}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kMaxBuildBricks = 1024;
// the builder's fixed LDS beside its tables: a flag byte, a code word and a brick index per slot, and a word
constexpr size_t kBuildFixedLds = (size_t)kMaxBuildBricks * 9u + 16u;
constexpr int kBuildThreads = 256;

struct TableLDS {
    float2* bv;
    float* ts;
    uint16_t* lut_col;
    uint16_t* lut_row;
};

// LDS carve-up of the builder, for one node: the column boundaries of its
// window (boundary k of the window = column c0 + k, k = 0 .. W_buf + 1) | row
// table | guess tables.
__device__ __forceinline__ TableLDS carve_tables(char* smem, const SensorDev& S) {
    TableLDS L;
    L.bv = reinterpret_cast<float2*>(smem);                 // [W_buf + 2]
    L.ts = reinterpret_cast<float*>(L.bv + S.WB + 2);
    L.lut_col = reinterpret_cast<uint16_t*>(L.ts + S.H + 1);
    L.lut_row = L.lut_col + S.n_lut_col;
    return L;
}

__device__ __forceinline__ void load_tables(const TableLDS& L, const SensorDev& S, int32_t c0) {
    for (int32_t i = threadIdx.x; i < S.WB + 2; i += blockDim.x) {
        int32_t c = c0 + i;
        c = c >= S.W ? c - S.W : c;
        c = c >= S.W ? c - S.W : c;
        L.bv[i] = S.bv[c];
    }
    for (int32_t i = threadIdx.x; i <= S.H; i += blockDim.x) L.ts[i] = S.ts[i];
    for (int32_t i = threadIdx.x; i < S.n_lut_col; i += blockDim.x) L.lut_col[i] = S.lut_col[i];
    for (int32_t i = threadIdx.x; i < S.n_lut_row; i += blockDim.x) L.lut_row[i] = S.lut_row[i];
}

// What the node can observe of brick (bx, by, bz), from below: the pixels that
// the brick's voxel centres can fall in lie inside a rectangle of the window
// (azimuth from the corners of the centres' box seen from outside, elevation
// from its nearest and farthest horizontal distance; both widened by a pixel,
// so float angles cannot drop a pixel), and every centre lies between the
// box's nearest and farthest distances. Returns kViewNone when the largest
// first hit over the tiles that cover the rectangle is below the nearest
// distance (no voxel is observed); kViewAll when the rectangle lies inside the
// window and its row band with a pixel to spare and the farthest distance is
// within the range and below the smallest first hit over those tiles (every
// voxel centre passes the per-voxel test, with margins for rounding); else
// kViewSome (the node is within a voxel of the box horizontally, the rectangle
// covers more than 64 tiles, or the voxels must be tested one by one).
// tm: the node's tile maxima, then its tile minima.
enum : int { kViewNone = 0, kViewSome = 1, kViewAll = 2 };
__device__ int brick_view(const SensorDev& S, const float* __restrict__ tm, float4 q, int32_t c0, uint32_t bx,
                          uint32_t by, uint32_t bz) {
    const float x0 = (float)(bx * 8u) + 0.5f - q.x, x1 = x0 + 7.f;
    const float y0 = (float)(by * 8u) + 0.5f - q.y, y1 = y0 + 7.f;
    const float z0 = (float)(bz * 8u) + 0.5f - q.z, z1 = z0 + 7.f;
    if (x0 <= 1.f && x1 >= -1.f && y0 <= 1.f && y1 >= -1.f) return kViewSome;
    // window columns of the four corners, unwrapped around the window
    const float W = (float)S.W, sh = 0.5f * (float)(S.W - S.WB);
    float lo = 1e30f, hi = -1e30f;
    const float cx[4] = {x0, x1, x0, x1}, cy[4] = {y0, y0, y1, y1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float v = (atan2f(cy[k], cx[k]) - S.az0) * S.daz_inv - (float)c0;
        v -= W * floorf((v + sh) / W);
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    if (hi - lo > 0.5f * W) return kViewSome;
    if (hi + 1.f < 0.f || lo - 1.f >= (float)S.WB) return kViewNone;
    const float fc_lo = floorf(lo) - 1.f, fc_hi = floorf(hi) + 1.f;
    const int32_t c_lo = (int32_t)fmaxf(fc_lo, 0.f);
    const int32_t c_hi = (int32_t)fminf(fc_hi, (float)(S.WB - 1));
    const float dx = x0 > 0.f ? x0 : (x1 < 0.f ? -x1 : 0.f);
    const float dy = y0 > 0.f ? y0 : (y1 < 0.f ? -y1 : 0.f);
    const float dz = z0 > 0.f ? z0 : (z1 < 0.f ? -z1 : 0.f);
    const float rmin = sqrtf(dx * dx + dy * dy);
    const float rmax = sqrtf(fmaxf(x0 * x0, x1 * x1) + fmaxf(y0 * y0, y1 * y1));
    const float e_hi = atan2f(z1, z1 >= 0.f ? rmin : rmax);
    const float e_lo = atan2f(z0, z0 >= 0.f ? rmax : rmin);
    const float r_lo = floorf((e_lo - S.el0) * S.del_inv) - 1.f, r_hi = floorf((e_hi - S.el0) * S.del_inv) + 1.f;
    if (r_hi < 0.f || r_lo > (float)(S.H - 1)) return kViewNone;
    const int32_t j_lo = (int32_t)fmaxf(r_lo, 0.f), j_hi = (int32_t)fminf(r_hi, (float)(S.H - 1));
    const int32_t tc0 = c_lo / kTileCols, tc1 = c_hi / kTileCols, tr0 = j_lo / kTileRows, tr1 = j_hi / kTileRows;
    if ((tc1 - tc0 + 1) * (tr1 - tr0 + 1) > 64) return kViewSome;
    float m = 0.f, mn = __builtin_inff();
    for (int32_t tc = tc0; tc <= tc1; ++tc)
        for (int32_t tr = tr0; tr <= tr1; ++tr) {
            m = fmaxf(m, tm[tc * S.trows + tr]);
            mn = fminf(mn, tm[S.n_tiles + tc * S.trows + tr]);
        }
    const float dmin2 = dx * dx + dy * dy + dz * dz;
    if (!(m * m * 1.0001f + 0.01f >= dmin2)) return kViewNone;
    const bool inside = (fc_lo >= 0.f) & (fc_hi <= (float)(S.WB - 1)) & (r_lo >= 0.f) & (r_hi <= (float)(S.H - 1));
    const float dmax2 = fmaxf(x0 * x0, x1 * x1) + fmaxf(y0 * y0, y1 * y1) + fmaxf(z0 * z0, z1 * z1);
    return (inside && dmax2 * 1.0001f + 0.01f <= fminf(S.rv2, mn * mn)) ? kViewAll : kViewSome;
}

// Path mask of node `node` over bricks [chunk * bricks, ...) of the mask grid:
// the parent's path mask (none at the root, and none with anc_cap = 1) ORed
// with the voxels the node itself observes. A voxel is observed when its
// centre lies in a pixel cell of the node's window (azimuth between two column
// boundaries by exact left-of tests, elevation between two row boundaries by
// r_z|r_z| against rho^2 times the tabulated t|t| of the boundary; cells
// half-open) and its squared range is at most the squared first hit stored for
// that pixel: the test its descendants would make against it. A brick keeps
// the parent's bits (and code) without testing when it lies beyond the range,
// wholly outside the node's azimuth wedge (margins cover the brick's voxel
// centres, within 3.5 sqrt(3) of its centre and 3.5 sqrt(2) across in x and
// y, and rounding), holds no unknown voxel, has every bit set already, or
// fails the depth cull (brick_view); a brick whose voxels the node observes
// all (brick_view again) gets every bit set without testing. Of these bricks
// only what can be read is written (the code, and the words when they can be
// read). The window's tables are loaded into LDS only when some
// brick of the chunk is tested. One wave tests one brick: each lane one (x, y)
// column of 8 voxels. Whole workgroup; chunks past the map's last brick do
// nothing (a batch launch covers its largest map).
__device__ __forceinline__ void build_live(const MapDev& M, const SensorDev& S, const TreeDev& Tr, int32_t node,
                                           const WindowGeom& A, float4 q, const uint32_t* par, uint32_t* out,
                                           char* smem, const uint8_t* s_live, uint32_t* s_cw, const uint32_t* s_b,
                                           int32_t cnt);

__device__ __forceinline__ void build_chunk(const MapDev& M, const SensorDev& S, const TreeDev& Tr, int32_t node,
                                            int32_t chunk, int32_t bricks, char* smem, uint8_t* s_live,
                                            uint32_t* s_cw, uint32_t* s_b, int32_t* s_any) {
    const int32_t tid = threadIdx.x;
    const int32_t slot = Tr.mask_slot[node];
    const uint32_t nb = M.mask_words >> 4;
    const uint32_t lo = (uint32_t)chunk * (uint32_t)bricks;  // first build slot (bricks is a multiple of 8)
    if (slot < 0 || lo >= M.build_slots) return;             // a leaf (nothing reads its mask), or past the map
    uint32_t* out = Tr.masks + (size_t)slot * M.mask_words;
    const int32_t a0 = Tr.anc_ptr[node];
    const uint32_t* par = nullptr;
    const uint32_t* pcode = nullptr;
    if (Tr.anc_cap > 1 && Tr.anc_ptr[node + 1] > a0) {
        const int32_t ps = Tr.mask_slot[Tr.anc_ids[a0]];
        par = Tr.masks + (size_t)ps * M.mask_words;
        pcode = Tr.mcode + (size_t)ps * nb;
    }
    const float4 q = Tr.q4[node];
    const int32_t c0 = Tr.c0[node];
    int32_t c1 = c0 + S.WB;
    c1 = c1 >= S.W ? c1 - S.W : c1;
    WindowGeom A;
    A.qx = q.x; A.qy = q.y; A.qz = q.z; A.c0 = c0;
    const float2 b0 = S.bv[c0], b1 = S.bv[c1];
    A.b0x = b0.x; A.b0y = b0.y; A.b1x = b1.x; A.b1y = b1.y;
    const int32_t cnt = bricks;
    if (tid == 0) *s_any = 0;
    // The chunk's slots, a block of 2x2x2 bricks per 8 slots: s_b holds each slot's
    // brick (~0 for a slot past the grid's bricks).
    const uint32_t mbx2 = (M.mbx + 1u) >> 1, mby2 = (M.mby + 1u) >> 1;
    for (int32_t i = tid; i < cnt; i += (int32_t)blockDim.x) {
        const uint32_t sl = lo + (uint32_t)i, blk = sl >> 3, j = sl & 7u;
        const uint32_t bx = 2u * (blk % mbx2) + (j & 1u), by = 2u * ((blk / mbx2) % mby2) + ((j >> 1) & 1u),
                       bz = 2u * (blk / (mbx2 * mby2)) + (j >> 2);
        s_b[i] = (bx < M.mbx && by < M.mby && bz < M.mbz) ? bx + M.mbx * (by + M.mby * bz) : ~0u;
    }
    __syncthreads();
    // per brick of the chunk (s_live): bit 4 live, bits 2-3 its brick_unk value,
    // bits 0-1 the parent's code (kMaskNone at the root); a slot past the grid's
    // bricks holds no unknown voxel
    for (int32_t i = tid; i < cnt; i += (int32_t)blockDim.x) {
        const uint32_t b = s_b[i];
        if (b == ~0u) {
            s_live[i] = (uint8_t)(kBrickKnown << 2);
            continue;
        }
        const uint32_t bx = b % M.mbx, by = (b / M.mbx) % M.mby, bz = b / (M.mbx * M.mby);
        const float rx = (float)(bx * 8u) + 4.0f - q.x, ry = (float)(by * 8u) + 4.0f - q.y,
                    rz = (float)(bz * 8u) + 4.0f - q.z;
        const float reach = S.rv + 6.6f;                     // 3.5 sqrt(3) = 6.06, plus rounding
        const bool near = rx * rx + ry * ry + rz * rz <= reach * reach;
        const float w0 = A.b0x * ry - A.b0y * rx, w1 = A.b1x * ry - A.b1y * rx;
        const bool wedge = (w0 >= -5.5f) & (w1 < 5.5f);      // 3.5 sqrt(2) = 4.95, plus rounding
        const uint32_t bu = M.brick_unk[b] & 3u;            // (without the all-free bit)
        const uint32_t pcw = par ? pcode[b] : uniform_code_word(kMaskNone);   // the parent's code word
        const uint32_t pc = pcw & 3u;
        // (a brick without unknown voxels needs no bits: only unknown voxels' bits
        // are read; nor does one whose voxels an ancestor all observes)
        const int view = (near && wedge && bu != kBrickKnown && pc != kMaskAll)
                             ? brick_view(S, Tr.tmax + (size_t)slot * 2 * S.n_tiles, q, c0, bx, by, bz)
                             : kViewNone;
        // (a brick whose voxels the node observes all gets every bit set, as the
        // per-voxel test would give it)
        const bool live = view == kViewSome;
        s_live[i] = (uint8_t)(((uint32_t)live << 4) | (bu << 2) | (view == kViewAll ? (uint32_t)kMaskAll : pc));
        s_cw[i] = view == kViewAll ? uniform_code_word(kMaskAll) : pcw;
        if (live) *s_any = 1;
    }
    __syncthreads();
    // Bricks that cannot hold a newly observed voxel keep the parent's code and
    // the bits that can be read: its words when they are mixed, constant words
    // for a brick that also holds known voxels, none for a wholly unknown brick
    // with a uniform code; bricks without unknown voxels are left alone.
    for (int32_t w = tid; w < cnt * 16; w += blockDim.x) {
        const uint32_t f = s_live[w >> 4];
        const uint32_t pc = f & 3u, bu = (f >> 2) & 3u;
        if ((f & 16u) || bu == kBrickKnown || (bu == kBrickAllUnknown && pc != kMaskMixed)) continue;
        const uint32_t wi = s_b[w >> 4] * 16u + (uint32_t)(w & 15);
        out[wi] = pc == kMaskMixed ? par[wi] : (pc == kMaskAll ? ~0u : 0u);
    }
    uint32_t* code = Tr.mcode + (size_t)slot * nb;
    if (*s_any) build_live(M, S, Tr, node, A, q, par, out, smem, s_live, s_cw, s_b, cnt);
    __syncthreads();
    // Code words of the chunk's bricks that hold an unknown voxel, with the code
    // of their block of 2x2x2 bricks (bits 18-19): uniform when the block's 8
    // bricks are all wholly unknown and their codes all clear or all set.
    for (int32_t i = tid; i < cnt; i += (int32_t)blockDim.x) {
        const uint32_t f = s_live[i];
        if (((f >> 2) & 3u) != kBrickKnown) {
            const int32_t g = i & ~7;
            uint32_t all_none = 1u, all_set = 1u;
#pragma unroll
            for (int32_t k = 0; k < 8; ++k) {
                const uint32_t fk = s_live[g + k], ck = s_cw[g + k] & 3u;
                const bool unk = ((fk >> 2) & 3u) == kBrickAllUnknown;
                all_none &= (unk && ck == kMaskNone) ? 1u : 0u;
                all_set &= (unk && ck == kMaskAll) ? 1u : 0u;
            }
            const uint32_t bc = all_none ? (uint32_t)kMaskNone : (all_set ? (uint32_t)kMaskAll : (uint32_t)kMaskMixed);
            code[s_b[i]] = (s_cw[i] & 0x3ffffu) | (bc << 18);
        }
    }
}

// The live bricks of a chunk (build_chunk): one wave tests one brick, each lane
// one (x, y) column of 8 voxels; the brick's code word goes to s_cw.
__device__ __forceinline__ void build_live(const MapDev& M, const SensorDev& S, const TreeDev& Tr, int32_t node,
                                           const WindowGeom& A, float4 q, const uint32_t* par, uint32_t* out,
                                           char* smem, const uint8_t* s_live, uint32_t* s_cw, const uint32_t* s_b,
                                           int32_t cnt) {
    const int32_t tid = threadIdx.x;
    const int32_t c0 = A.c0;
    const TableLDS L = carve_tables(smem, S);
    load_tables(L, S, c0);
    __syncthreads();
    const int32_t lane = tid & 63;
    const float ts0 = L.ts[0], tsH = L.ts[S.H];
    const gfloats_t dnode = as_global(uniform_ptr(Tr.dpan + (size_t)node * S.R));   // the node's panorama
    // (the wave's brick is wave-uniform: its index arithmetic stays scalar)
    const int32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int32_t i = wave; i < cnt; i += (int32_t)(blockDim.x >> 6)) {
        const uint32_t f = s_live[i];
        if (!(f & 16u)) continue;
        const uint32_t b = s_b[i];
        const int32_t bx = (int32_t)(b % M.mbx), by = (int32_t)((b / M.mbx) % M.mby), bz = (int32_t)(b / (M.mbx * M.mby));
        const int32_t x = bx * 8 + (lane & 7), y = by * 8 + (lane >> 3);
        const float cx = (float)x + 0.5f, cy = (float)y + 0.5f;
        const uint32_t wbase = b << 4;
        uint32_t pw = 0u;                 // the parent's bits (a live brick's parent code is not all set)
        if ((f & 3u) == kMaskMixed && lane < 16) pw = par[wbase + (uint32_t)lane];
        // The lane's column of the brick: the azimuth column of its pixels (the
        // same for the 8 voxels, which share x and y), the row of each voxel,
        // then the 8 depths, loaded together. The voxels' states are not read: only unknown voxels' bits are ever looked
        // up, so bits of known voxels (and of voxels past the grid) do not matter.
        const float rx = cx - A.qx, ry = cy - A.qy;
        const float w0 = A.b0x * ry - A.b0y * rx;
        const float w1 = A.b1x * ry - A.b1y * rx;
        const bool wedge = (w0 >= 0.f) & (w1 < 0.f);
        const float rho2 = rx * rx + ry * ry;
        // column (computed for every lane; only lanes in the wedge use it, and the
        // clamps keep every table index inside its table)
        const float u0 = A.b0x * rx + A.b0y * ry;
        float pa = w0 * __builtin_amdgcn_rcpf(fabsf(u0) + w0);
        pa = u0 < 0.f ? 2.f - pa : pa;
        const int32_t gc =
            L.lut_col[(int32_t)__builtin_amdgcn_fmed3f(pa * S.lut_col_scale, 0.f, (float)(S.n_lut_col - 1))];
        const float2 v0 = L.bv[gc], v1 = L.bv[gc + 1], v2 = L.bv[gc + 2];
        const bool l0 = (gc == 0) | left_of(v0, rx, ry);
        const bool l1 = (gc + 1 < S.WB) & left_of(v1, rx, ry);
        const bool l2 = (gc + 2 < S.WB) & left_of(v2, rx, ry);
        int32_t col = gc + (int32_t)l1;
        if (wedge & !(l0 & !l2)) {      // (rare: a guess at a bucket edge)
            for (;;) {
                if (col + 1 >= S.WB || !left_of(L.bv[col + 1], rx, ry)) break;
                ++col;
            }
            for (;;) {
                if (col == 0 || left_of(L.bv[col], rx, ry)) break;
                --col;
            }
        }
        // (column < 4096 and H <= 2048: the product fits the 24-bit multiplier; the
        // index is into the node's own panorama, R < 2^22 entries)
        const uint32_t colbase = __umul24((uint32_t)wrap(A.c0 + col, S.W), (uint32_t)S.H);
        const float irho = __builtin_amdgcn_rsqf(rho2);
        // Rows: the row of a voxel is the number of inner row boundaries j in
        // 1..H-1 with sz >= rho2 * ts[j] (ts and hence rho2 * ts[j] grow with j,
        // so they form a prefix). Within the lane's column sz grows with z, so
        // the count never falls from one slice to the next: slice 0 takes the
        // guess table and its settle (exact for any sz: the table's clamped ends
        // give 0 and H - 1 outside the band), each later slice checks the next
        // two boundaries and walks on only when both are passed (steep voxels
        // near the node). Lanes outside the wedge never use their rows.
        uint32_t idx[8];
        float r2[8];
        bool ok[8];
        int32_t row = 0;
#pragma unroll
        for (int32_t pz = 0; pz < 8; ++pz) {
            const float rz = ((float)(bz * 8 + pz) + 0.5f) - A.qz;
            const float range2 = rho2 + rz * rz;
            const float sz = rz * fabsf(rz);
            ok[pz] = wedge & (range2 <= S.rv2) & (sz >= rho2 * ts0) & (sz < rho2 * tsH);
            r2[pz] = range2;
            if (pz == 0) {
                const float tg = rz * irho;
                const int32_t gr = L.lut_row[(int32_t)__builtin_amdgcn_fmed3f((tg - S.lut_row_lo) * S.lut_row_scale,
                                                                             0.f, (float)(S.n_lut_row - 1))];
                const float e0 = L.ts[gr], e1 = L.ts[gr + 1], e2 = L.ts[min(gr + 2, S.H)];
                const bool q0 = (gr == 0) | (sz >= rho2 * e0);
                const bool q1 = (gr + 1 < S.H) & (sz >= rho2 * e1);
                const bool q2 = (gr + 2 < S.H) & (sz >= rho2 * e2);
                row = gr + (int32_t)q1;
                if (wedge & !(q0 & !q2)) {   // (rare: a guess at a bucket edge)
                    for (;;) {
                        if (row + 1 >= S.H || !(sz >= rho2 * L.ts[row + 1])) break;
                        ++row;
                    }
                    for (;;) {
                        if (row == 0 || sz >= rho2 * L.ts[row]) break;
                        --row;
                    }
                }
            } else {
                const float e1 = L.ts[min(row + 1, S.H)], e2 = L.ts[min(row + 2, S.H)];
                const bool a1 = (row + 1 < S.H) & (sz >= rho2 * e1);
                const bool a2 = (row + 2 < S.H) & (sz >= rho2 * e2);
                row += (int32_t)a1;
                if (wedge & a2) {            // (two or more boundaries between neighbouring voxels)
                    for (;;) {
                        if (row + 1 >= S.H || !(sz >= rho2 * L.ts[row + 1])) break;
                        ++row;
                    }
                }
            }
            idx[pz] = ok[pz] ? colbase + (uint32_t)row : 0u;
        }
        float D[8];
#pragma unroll
        for (int32_t pz = 0; pz < 8; ++pz) D[pz] = *(gfloats_t)((gbytes_t)dnode + (idx[pz] << 2));
        // observed: the centre's squared range is at most its pixel's squared depth;
        // lane l < 16 collects mask word l of the brick (slice l / 2) and stores it
        uint32_t word = 0u;
#pragma unroll
        for (int32_t pz = 0; pz < 8; ++pz) {
            const uint64_t bal = ballot(ok[pz] & (r2[pz] <= D[pz] * D[pz]));
            word = lane == 2 * pz ? (uint32_t)bal : word;
            word = lane == 2 * pz + 1 ? (uint32_t)(bal >> 32) : word;
        }
        word |= pw;
        if (lane < 16) out[wbase + (uint32_t)lane] = word;
        // the brick's code word: its 512 bits and each quarter's 64 all clear, all
        // set, or mixed (word l holds slice l / 2, rows 4 (l & 1) .. + 3, x in its
        // bytes' low and high nibbles)
        const bool w_ok = lane < 16;
        const uint64_t nz_lo = ballot(w_ok & ((word & 0x0f0f0f0fu) != 0u)), nz_hi = ballot(w_ok & ((word & 0xf0f0f0f0u) != 0u));
        const uint64_t nf_lo = ballot(w_ok & ((word | 0xf0f0f0f0u) != ~0u)), nf_hi = ballot(w_ok & ((word | 0x0f0f0f0fu) != ~0u));
        uint32_t cw = (nz_lo | nz_hi) == 0ull ? (uint32_t)kMaskNone : ((nf_lo | nf_hi) == 0ull ? (uint32_t)kMaskAll : (uint32_t)kMaskMixed);
#pragma unroll
        for (uint32_t qd = 0; qd < 8; ++qd) {
            const uint64_t lq = 0x55ull << (8u * (qd >> 2) + ((qd >> 1) & 1u));   // words of the quarter's slices and rows
            const uint64_t nz = (qd & 1u) ? nz_hi : nz_lo, nf = (qd & 1u) ? nf_hi : nf_lo;
            const uint32_t qc = (nz & lq) == 0ull ? (uint32_t)kMaskNone : ((nf & lq) == 0ull ? (uint32_t)kMaskAll : (uint32_t)kMaskMixed);
            cw |= qc << (2u + 2u * qd);
        }
        if (lane == 0) s_cw[i] = cw;
    }
}

__global__ __launch_bounds__(kBuildThreads) void k_mask_build(MapDev M, SensorDev S, TreeDev Tr,
                                                              const int32_t* __restrict__ nodes, int32_t chunks,
                                                              int32_t bricks) {
    extern __shared__ char smem[];
    __shared__ uint8_t s_live[kMaxBuildBricks];
    __shared__ uint32_t s_cw[kMaxBuildBricks];
    __shared__ uint32_t s_b[kMaxBuildBricks];
    __shared__ int32_t s_any;
    build_chunk(M, S, Tr, nodes[blockIdx.x / chunks], (int32_t)(blockIdx.x % chunks), bricks, smem, s_live, s_cw, s_b, &s_any);
}

// ---------------------------------------------------------------- ray traversal

// One workgroup = kTh / 64 pixel blocks (tile `tile`) of one node, one block of
// kRayBlockCols x kRayBlockRows rays per wave: neighbouring pixels have rays of
// similar length, so a wave's lanes run for similar numbers of steps. A lane walks
// its ray with the Amanatides-Woo 3D DDA (face-crossing parameters recomputed
// as (boundary - q) * (1/d); ties step x, then y, then z; a voxel is visited
// while its entry parameter is below the range and it is inside the grid). An
// occupied voxel ends the ray and its entry parameter (or the range) is the
// ray's first hit. Unknown voxels count into the absolute bin of the ray's
// column and, in marginal mode, into the marginal bin unless the parent's
// path mask holds them (some ancestor observes them); the root has no
// ancestor, so all its unknown voxels count. The grid byte of the next voxel is
// requested before the step ends, and a mask word is used one step after it
// was requested, so both loads have a step of work to hide behind. Ends with
// the tile's bins added to the node's global bins.
template <bool kMarginal, int kTh>
__device__ __forceinline__ void trace_tile(const MapDev& M, const SensorDev& S, const TreeDev& Tr, int32_t node,
                                           int32_t tile, uint32_t* __restrict__ s_bins) {
    const int32_t tid = threadIdx.x;
    const uint32_t* pmask = nullptr;     // the parent's path mask
    const uint32_t* pcode = nullptr;     // and its bricks' code words
    if (kMarginal) {
        const int32_t a0 = Tr.anc_ptr[node];
        if (Tr.anc_cap > 0 && Tr.anc_ptr[node + 1] > a0) {
            const int32_t ps = Tr.mask_slot[Tr.anc_ids[a0]];
            pmask = Tr.masks + (size_t)ps * M.mask_words;
            pcode = Tr.mcode + (size_t)ps * (M.mask_words >> 4);
        }
    }
    const gwords_t pm = as_global(uniform_ptr(pmask));
    const gwords_t pc = as_global(uniform_ptr(pcode));
    for (int32_t i = tid; i < 2 * S.B; i += kTh) s_bins[i] = 0u;
    __syncthreads();

    // this wave's pixel block and this lane's pixel in it (column c, row j)
    const int32_t blk = __builtin_amdgcn_readfirstlane(tile * (kTh / 64) + (tid >> 6));
    const int32_t cb = __builtin_amdgcn_readfirstlane(blk / S.nrb);
    const int32_t c = cb * kRayBlockCols + (tid & (kRayBlockCols - 1));
    const int32_t j = (blk - cb * S.nrb) * kRayBlockRows + ((tid & 63) / kRayBlockCols);
    const bool has_ray = (blk < S.n_blocks) & (c < S.W) & (j < S.H);
    const int32_t r = c * S.H + j;
    const int32_t rr = has_ray ? r : 0;
    const int32_t bin = S.bin_of_col[has_ray ? c : 0];
    const float4 p = Tr.q4[node];
    const float4 d = S.d4[rr];
    const float4 iv = S.iv4[rr];
    const int32_t sx = d.x > 0.f ? 1 : (d.x < 0.f ? -1 : 0);
    const int32_t sy = d.y > 0.f ? 1 : (d.y < 0.f ? -1 : 0);
    const int32_t sz = d.z > 0.f ? 1 : (d.z < 0.f ? -1 : 0);
    int32_t ix = (int32_t)floorf(p.x), iy = (int32_t)floorf(p.y), iz = (int32_t)floorf(p.z);
    // Face-crossing parameters (b - q) / d with b the next voxel boundary,
    // kept as floats (integers, exact): b moves by the step sign. An axis the
    // ray does not move along has b = +inf and a factor 1, so its parameter
    // stays +inf.
    const float inf = __builtin_inff();
    float bx = sx ? (float)(ix + (sx > 0 ? 1 : 0)) : inf;
    float by = sy ? (float)(iy + (sy > 0 ? 1 : 0)) : inf;
    float bz = sz ? (float)(iz + (sz > 0 ? 1 : 0)) : inf;
    const float fx = sx ? iv.x : 1.f, fy = sy ? iv.y : 1.f, fz = sz ? iv.z : 1.f;
    const float dbx = (float)sx, dby = (float)sy, dbz = (float)sz;
    // the node's coordinates, -inf on an axis the ray does not move along: every
    // boundary parameter of that axis, (b - q) * 1 with b = +inf or a brick
    // exit, is then +inf
    const float qx = sx ? p.x : -inf, qy = sy ? p.y : -inf, qz = sz ? p.z : -inf;
    // a block's exit boundary along an axis: its low face, plus its edge when moving up
    const int32_t upx = sx > 0 ? -1 : 0, upy = sy > 0 ? -1 : 0, upz = sz > 0 ? -1 : 0;
    float tx = (bx - qx) * fx;
    float ty = (by - qy) * fy;
    float tz = (bz - qz) * fz;
    float t = 0.f, h = S.rv;
    uint32_t n_abs = 0, n_new = 0;
    const gbytes_t grid = as_global(M.bricks);
    // the node lies inside the grid and t = 0 < rv, so its own voxel is
    // visited; a lane without a ray reads a padding byte and is done at once
    uint32_t addr = has_ray ? voxel_addr(ix, iy, iz, M) : M.outside;   // address of the current voxel
    // (this first byte is read through the generic pointer and the loop's through
    // the global one, so the compiler keeps the loop's load at the end of the
    // step instead of merging the two into one load at the top of the loop)
    uint32_t st = M.bricks[addr];
    uint32_t mw = 0u, mb = 0u;          // mask word of the last unknown voxel, and its bit
    bool pend = false;                  // (a word requested in the previous step)
    uint32_t cb_idx = ~0u, cw = 0u;     // the last unknown block's brick and its code word
    if (ballot(has_ray)) {
        uint64_t alive;
        do {
            // Straight-line step: the mask word requested in the previous step
            // and the current voxel's byte are used first, then the next voxel is
            // found and its byte requested. A lane that has finished (or left the
            // grid) reads a padding byte, which is neither unknown nor occupied.
            if (kMarginal) {
                n_new += (pend & !((mw >> mb) & 1u)) ? 1u : 0u;
                pend = false;
            }
            h = st == kOccupied ? t : h;
            // An aligned block (a block of 2x2x2 bricks, a brick, a quarter brick
            // or, for free voxels, a 2x2x2 block) whose voxels are all free, or
            // all unknown with the parent's mask uniform over it (every bit clear
            // or every bit set; a wholly unknown block over which the mask is
            // mixed is crossed a brick or a quarter at a time where it is uniform
            // over that), is crossed in one step: it is left through the face whose
            // boundary parameter comes first (ties x, y, z) and every other axis
            // has crossed the boundaries that come before that crossing in the
            // same order. The voxels crossed are one per crossing; crossing an
            // unknown block counts them all as absolute, and as marginal when no
            // ancestor observes any of them. An unknown block that the range ends
            // in is finished in one step too: its voxels visited before the range
            // ends are counted and the ray ends.
            float tn;                           // entry parameter of the next voxel
            float kx, ky, kz;                   // boundaries this step crosses along each axis (set by
                                                // the crossing when it is taken, else by the voxel step)
            uint32_t level = (st >> kLevelShift) & kLevelMask;   // the voxel's block: edge 32 >> level, or none (0)
            const bool free_blk = (level != 0u) & ((st & 3u) == kFree);
            bool cand = free_blk;
            uint32_t code = kMaskNone;          // (the absolute pass, and the root, see nothing observed)
            // (a wholly unknown block with a uniform code is always crossed by its
            // code: the words of its brick need not exist)
            if ((level != 0u) & ((st & 3u) == kUnknown)) {
                if (kMarginal && pc != nullptr) {
                    const uint32_t b = mask_brick(ix, iy, iz, M);
                    if (b != cb_idx) {
                        cw = pc[b];
                        cb_idx = b;
                    }
                    // the code of its block of 2x2x2 bricks (a 16-voxel block), else the
                    // brick's (a brick at most), else its quarter's (a quarter at most)
                    const uint32_t qs = 2u + ((((uint32_t)ix >> 1) & 2u) | ((uint32_t)iy & 4u) | (((uint32_t)iz << 1) & 8u));
                    const uint32_t bc = (cw >> 18) & 3u;
                    const bool block_uniform = (level == 1u) & (bc != kMaskMixed);
                    const bool brick_uniform = (cw & 3u) != kMaskMixed;
                    code = block_uniform ? bc : (brick_uniform ? (cw & 3u) : ((cw >> qs) & 3u));
                    level = block_uniform ? 1u : (brick_uniform ? (level > 2u ? level : 2u) : 3u);
                }
                cand = code != kMaskMixed;
            }
            if (cand) {
                const int32_t edge = 32 >> level;
                const float Tx = ((float)((ix & -edge) + (edge & upx)) - qx) * fx;
                const float Ty = ((float)((iy & -edge) + (edge & upy)) - qy) * fy;
                const float Tz = ((float)((iz & -edge) + (edge & upz)) - qz) * fz;
                const bool fx_ = (Tx <= Ty) & (Tx <= Tz);
                const bool fy_ = !fx_ & (Ty <= Tz);
                const bool fz_ = !fx_ & !fy_;
                const float T = fx_ ? Tx : (fy_ ? Ty : Tz);
                // An axis that precedes the exit axis in the tie order also
                // counts a boundary whose parameter equals T: it compares with
                // the next float above T (T >= 0; +0 for -0 first). When the
                // range ends inside an unknown block (cut), the ray's remaining
                // voxels are the current one and one per boundary whose
                // parameter is below the range, all inside the block: every
                // axis counts against the range, and the ray ends (T >= range).
                const bool cut = !free_blk & !(T < S.rv);
                const float Tn = __uint_as_float(__float_as_uint(T + 0.f) + 1u);
                const bool wide = ballot(level == 1u) != 0ull;     // some lane crosses a 16-voxel block
                kx = crossings_before(bx, dbx, qx, fx, cut ? S.rv : (fx_ ? T : Tn), wide) + (fx_ ? 1.f : 0.f);
                ky = crossings_before(by, dby, qy, fy, cut ? S.rv : (fz_ ? Tn : T), wide) + (fy_ ? 1.f : 0.f);
                kz = crossings_before(bz, dbz, qz, fz, cut ? S.rv : T, wide) + (fz_ ? 1.f : 0.f);
                tn = T;
                if (!free_blk) {
                    const uint32_t v = (uint32_t)(kx + ky + kz);
                    n_abs += v;
                    if (kMarginal) n_new += code == kMaskNone ? v : 0u;
                }
            }
            if (!cand) {
                const bool unk = is_unknown(st);
                n_abs += unk ? 1u : 0u;
                if (kMarginal && pm != nullptr) {
                    // every lane loads (a lane off unknown voxels reads word 0), so the
                    // word lands in the register the next step reads
                    const uint32_t off = (unk ? mask_word(ix, iy, iz, M) : 0u) << 2;   // < 2^29 bytes
                    mw = *(gwords_t)((gbytes_t)pm + off);
                    mb = mask_bit(ix, iy);
                    pend = unk;
                }
                const bool mx = (tx <= ty) & (tx <= tz);
                const bool my = !mx & (ty <= tz);
                const bool mz = !mx & !my;
                tn = mx ? tx : (my ? ty : tz);
                kx = mx ? 1.f : 0.f;
                ky = my ? 1.f : 0.f;
                kz = mz ? 1.f : 0.f;
            }
            // one update for both kinds of step (counts are small integers: exact)
            ix += __mul24((int32_t)kx, sx);
            iy += __mul24((int32_t)ky, sy);
            iz += __mul24((int32_t)kz, sz);
            bx = __builtin_fmaf(kx, dbx, bx);
            by = __builtin_fmaf(ky, dby, by);
            bz = __builtin_fmaf(kz, dbz, bz);
            // a lane that stops here (occupied, finished or outside) compares +inf
            // with the range: one comparison gives the mask the ballot takes
            const float tn_go = (st & 2u) == 0u ? tn : inf;
            const bool next_ok = tn_go < S.rv;
            alive = ballot(next_ok);
            addr = next_ok ? voxel_addr(ix, iy, iz, M) : M.outside;
            st = grid[addr];
            tx = (bx - qx) * fx;
            ty = (by - qy) * fy;
            tz = (bz - qz) * fz;
            t = tn;
        } while (alive);
    }
    if (kMarginal) {
        n_new += (pend & !((mw >> mb) & 1u)) ? 1u : 0u;
        if (pm == nullptr) n_new = n_abs;                   // the root: nothing is observed yet
        if (has_ray) Tr.dpan[(size_t)node * S.R + r] = h;
        if (n_new) atomicAdd(&s_bins[S.B + bin], n_new);
    }
    if (n_abs) atomicAdd(&s_bins[bin], n_abs);
    __syncthreads();
    uint32_t* gb = Tr.bins + (size_t)node * 2 * S.B;
    for (int32_t i = tid; i < 2 * S.B; i += kTh) {
        const uint32_t v = s_bins[i];
        if (v) atomicAdd(&gb[i], v);
    }
}

// Per-tree levels: one-wave workgroups (as the batch autotuner picks for the
// large workloads).
constexpr int kTreeTraceThreads = 64;
template <bool kMarginal>
__global__ __launch_bounds__(kTreeTraceThreads) void k_trace(MapDev M, SensorDev S, TreeDev Tr,
                                                             const int32_t* __restrict__ nodes) {
    __shared__ uint32_t s_bins[2 * kMaxBins];
    // (workgroup-uniform values kept in scalar registers)
    const int32_t item = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / (uint32_t)S.T));
    const int32_t tile = __builtin_amdgcn_readfirstlane((int32_t)blockIdx.x - item * S.T);
    trace_tile<kMarginal, kTreeTraceThreads>(M, S, Tr, nodes[item], tile, s_bins);
}

// ---------------------------------------------------------------- window selection

// Window sums from a prefix sum over the bins taken circularly
// (P[i+1] = P[i] + bins[i mod B], S(k) = P[k+w] - P[k]), then the largest sum
// with the smallest k. Whole workgroup; returns (sum << 32) | (B - 1 - k) to
// every thread. Bins are read with atomic loads (they were accumulated with
// device-scope atomics, possibly by other workgroups).
// The largest and the smallest first hit of each tile of a node's window
// (kTileCols x kTileRows pixels, partial at the window's edges), for the mask
// builder's whole-brick tests of the node's bricks; only nodes with children
// have a path mask to build.
// Consecutive threads take consecutive tiles of a tile column, so their reads
// of the column-major panorama are contiguous.
__device__ __forceinline__ void tile_max(const SensorDev& S, const TreeDev& Tr, int32_t node, int32_t c0) {
    const int32_t slot = Tr.mask_slot[node];
    if (slot < 0) return;
    const float* src = Tr.dpan + (size_t)node * S.R;
    float* dst = Tr.tmax + (size_t)slot * 2 * S.n_tiles;
    for (int32_t t = threadIdx.x; t < S.n_tiles; t += blockDim.x) {
        const int32_t tc = t / S.trows, tr = t - tc * S.trows;
        const int32_t j0 = tr * kTileRows, j1 = min(j0 + kTileRows, S.H);
        float m = 0.f, mn = __builtin_inff();
        for (int32_t i = tc * kTileCols; i < min((tc + 1) * kTileCols, S.WB); ++i) {
            const float* col = src + (size_t)wrap(c0 + i, S.W) * S.H;
            for (int32_t j = j0; j < j1; ++j) {
                m = fmaxf(m, col[j]);
                mn = fminf(mn, col[j]);
            }
        }
        dst[t] = m;
        dst[S.n_tiles + t] = mn;
    }
}

__device__ __forceinline__ unsigned long long select_window(const uint32_t* bins, const SensorDev& S,
                                                            uint32_t* s_p, unsigned long long* s_best) {
    const int32_t tid = threadIdx.x;
    const int32_t L = S.B + S.w;   // extended length <= 2*kMaxBins
    for (int32_t i = tid; i < L; i += kThreads)
        s_p[i + 1] = __hip_atomic_load(&bins[i % S.B], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) s_p[0] = 0u;
    __syncthreads();
    // inclusive Hillis-Steele scan of s_p[1..L]
    for (int32_t off = 1; off < L; off <<= 1) {
        uint32_t v0 = 0, v1 = 0;
        const int32_t i0 = tid + 1, i1 = tid + 1 + kThreads;
        if (i0 <= L && i0 - off >= 1) v0 = s_p[i0 - off];
        if (i1 <= L && i1 - off >= 1) v1 = s_p[i1 - off];
        __syncthreads();
        if (i0 <= L) s_p[i0] += v0;
        if (i1 <= L) s_p[i1] += v1;
        __syncthreads();
    }
    unsigned long long key = 0ull;
    for (int32_t k = tid; k < S.B; k += kThreads) {
        const uint32_t sum = s_p[k + S.w] - s_p[k];
        const unsigned long long kk = ((unsigned long long)sum << 32) | (uint32_t)(S.B - 1 - k);
        key = kk > key ? kk : key;
    }
    for (int32_t off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
    }
    if ((tid & 63) == 0) s_best[tid >> 6] = key;
    __syncthreads();
    unsigned long long best = s_best[0];
    for (int32_t i = 1; i < kThreads / 64; ++i) best = s_best[i] > best ? s_best[i] : best;
    __syncthreads();
    return best;
}

// One workgroup per node of a level: gain and window; in marginal mode also
// the node's window start column for its descendants.
__global__ __launch_bounds__(kThreads) void k_finish(SensorDev S, TreeDev Tr, const int32_t* __restrict__ nodes,
                                                     int marginal, uint32_t* __restrict__ gain,
                                                     int32_t* __restrict__ yaw) {
    __shared__ uint32_t s_p[2 * kMaxBins + 1];
    __shared__ unsigned long long s_best[kThreads / 64];
    const int32_t node = nodes[blockIdx.x];
    const unsigned long long best =
        select_window(Tr.bins + (size_t)node * 2 * S.B + (marginal ? S.B : 0), S, s_p, s_best);
    const int32_t k = S.B - 1 - (int32_t)(uint32_t)(best & 0xffffffffull);
    if (threadIdx.x == 0) {
        gain[node] = (uint32_t)(best >> 32);
        yaw[node] = k;
        if (marginal) Tr.c0[node] = S.c0_of_win[k];
    }
    if (marginal) tile_max(S, Tr, node, S.c0_of_win[k]);
}

// ---------------------------------------------------------------- multi-tree, level by level

// Clears the bins of every tree in a batch. Grid: (blocks, n_trees).
__global__ void k_batch_zero(const BatchTree* __restrict__ trees, int32_t B2) {
    const BatchTree& T = trees[blockIdx.y];
    const size_t nb = (size_t)T.td.n * (size_t)B2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nb; i += (size_t)gridDim.x * blockDim.x)
        T.td.bins[i] = 0u;
}

// Workgroups are dealt to the chip's 8 XCDs (each with its own L2) in turn:
// this permutation of the grid gives each XCD runs of kXcdRun consecutive work
// units (neighbouring pixel blocks, or bricks, of one node) while the runs
// still alternate over the whole grid; the grid's last partial round keeps
// the identity.
constexpr uint32_t kXcdRun = 16;
__device__ __forceinline__ uint32_t xcd_grouped(uint32_t g, uint32_t n) {
    const uint32_t full = (n / (8u * kXcdRun)) * (8u * kXcdRun);
    return g < full ? ((g >> 3) / kXcdRun) * (8u * kXcdRun) + (g & 7u) * kXcdRun + (g >> 3) % kXcdRun : g;
}

// One depth level of all trees at once: work item = (tree, node) from
// `items` (tree << 32 | node), T workgroups per item.
template <int kTh>
__global__ __launch_bounds__(kTh) void k_trace_multi(const BatchTree* __restrict__ trees,
                                                     const unsigned long long* __restrict__ items, SensorDev S) {
    __shared__ uint32_t s_bins[2 * kMaxBins];
    // (workgroup-uniform values kept in scalar registers)
    const uint32_t g = xcd_grouped(blockIdx.x, gridDim.x);
    const int32_t item = __builtin_amdgcn_readfirstlane((int32_t)(g / (uint32_t)S.T));
    const int32_t tile = __builtin_amdgcn_readfirstlane((int32_t)g - item * S.T);
    const unsigned long long it = items[item];
    const BatchTree& BT = trees[(uint32_t)(it >> 32)];
    if (BT.status != nullptr && *BT.status != 0) return;      // (the request has failed)
    SensorDev St = S;
    St.rv = BT.rv;
    St.rv2 = BT.rv2;
    const MapDev M = BT.map;     // copies: loaded once, not re-read through the descriptor
    const TreeDev Tr = BT.td;
    trace_tile<true, kTh>(M, St, Tr, (int32_t)(uint32_t)it, tile, s_bins);
}

// Path masks of one depth level's nodes with children, all trees at once:
// `chunks` workgroups per item, `bricks` bricks each.
__global__ __launch_bounds__(kBuildThreads) void k_mask_build_multi(const BatchTree* __restrict__ trees,
                                                                    const unsigned long long* __restrict__ items,
                                                                    SensorDev S, int32_t chunks, int32_t bricks) {
    extern __shared__ char smem[];
    __shared__ uint8_t s_live[kMaxBuildBricks];
    __shared__ uint32_t s_cw[kMaxBuildBricks];
    __shared__ uint32_t s_b[kMaxBuildBricks];
    __shared__ int32_t s_any;
    const uint32_t g = xcd_grouped(blockIdx.x, gridDim.x);
    const unsigned long long it = items[g / (uint32_t)chunks];
    const BatchTree& BT = trees[(uint32_t)(it >> 32)];
    if (BT.status != nullptr && *BT.status != 0) return;      // (the request has failed)
    SensorDev St = S;
    St.rv = BT.rv;
    St.rv2 = BT.rv2;
    const MapDev M = BT.map;
    const TreeDev Tr = BT.td;
    build_chunk(M, St, Tr, (int32_t)(uint32_t)it, (int32_t)(g % (uint32_t)chunks), bricks, smem, s_live, s_cw, s_b, &s_any);
}

// Window selection of one (tree, node) item of a batch: gain, window, the
// window's first column, the depth-cull tile maxima and, when asked for, the
// node's depth buffer. One workgroup of kThreads.
__device__ __forceinline__ void finish_item(const BatchTree* __restrict__ trees, unsigned long long it,
                                            const SensorDev& S, uint32_t* s_p, unsigned long long* s_best) {
    const BatchTree& BT = trees[(uint32_t)(it >> 32)];
    if (BT.status != nullptr && *BT.status != 0) return;      // (the request has failed)
    const int32_t node = (int32_t)(uint32_t)it;
    const unsigned long long best = select_window(BT.td.bins + (size_t)node * 2 * S.B + S.B, S, s_p, s_best);
    const int32_t k = S.B - 1 - (int32_t)(uint32_t)(best & 0xffffffffull);
    const int32_t c0 = S.c0_of_win[k];
    if (threadIdx.x == 0) {
        BT.gain[node] = (uint32_t)(best >> 32);
        BT.yaw[node] = k;
        BT.td.c0[node] = c0;
    }
    tile_max(S, BT.td, node, c0);
    if (BT.depth) {
        const int32_t per = S.H * S.WB;
        const float* src = BT.td.dpan + (size_t)node * S.R;
        float* dst = BT.depth + (size_t)node * per;
        for (int32_t o = threadIdx.x; o < per; o += kThreads) {
            const int32_t j = o / S.WB, ii = o - j * S.WB;
            int32_t c = c0 + ii;
            c = c >= S.W ? c - S.W : c;
            dst[o] = src[c * S.H + j];
        }
    }
}

// Window selection for one depth level of all trees: one workgroup per item.
__global__ __launch_bounds__(kThreads) void k_finish_multi(const BatchTree* __restrict__ trees,
                                                           const unsigned long long* __restrict__ items, SensorDev S) {
    __shared__ uint32_t s_p[2 * kMaxBins + 1];
    __shared__ unsigned long long s_best[kThreads / 64];
    finish_item(trees, items[blockIdx.x], S, s_p, s_best);
}

// ---------------------------------------------------------------- persistent batch

// Barrier over the whole grid of the persistent batch kernel, whose workgroups
// are all resident at once (the cooperative launch refuses a grid that cannot
// be). sync[0] counts arrivals and only grows: after k barriers it reaches
// k * gridDim.x, which each workgroup tracks in *target. A wait that polls
// `spin_limit` times without every workgroup arriving sets sync[1], and every
// workgroup then leaves at its next barrier, so the kernel always ends; the
// host reads sync[1] afterwards. An agent-scope release fence before the
// arrival and an acquire fence after the wait make each phase's writes visible
// to the next phase on every XCD; the polls themselves are relaxed loads, which
// leave the caches of the workgroups still working alone. Returns false once a
// wait has given up.
__device__ bool grid_barrier(uint32_t* sync, uint32_t* target, uint32_t spin_limit, int32_t* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        *target += gridDim.x;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t ok = 1;
        for (uint32_t polls = 0;; ++polls) {
            const uint32_t a = __hip_atomic_load(&sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int32_t)(a - *target) >= 0) break;
            if (__hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || polls >= spin_limit) {
                __hip_atomic_store(&sync[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// The whole batch in one launch (Sec. IV-C's depth order across all trees):
// for each depth level, every (node, ray tile) is traced, then every node's
// window is chosen, then the path masks of the level's nodes with children
// are built, with a grid barrier after each phase. Work units of a phase are
// dealt to the workgroups in turn (unit = blockIdx.x + k * gridDim.x); every
// workgroup passes every barrier, whether it had units or not.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_batch_persistent(
    const BatchTree* __restrict__ trees, const unsigned long long* __restrict__ items,
    const int32_t* __restrict__ level_ptr, const unsigned long long* __restrict__ mitems,
    const int32_t* __restrict__ mlevel_ptr, int32_t levels, SensorDev S, int32_t chunks, int32_t bricks,
    uint32_t* sync, uint32_t spin_limit) {
    extern __shared__ char smem[];
    __shared__ uint32_t s_bins[2 * kMaxBins];
    __shared__ uint32_t s_p[2 * kMaxBins + 1];
    __shared__ unsigned long long s_best[kThreads / 64];
    __shared__ uint8_t s_live[kMaxBuildBricks];
    __shared__ uint32_t s_cw[kMaxBuildBricks];
    __shared__ uint32_t s_b[kMaxBuildBricks];
    __shared__ int32_t s_any, s_ok;
    uint32_t target = 0;
    const uint32_t G = gridDim.x;
    for (int32_t d = 0; d < levels; ++d) {
        const int32_t i0 = level_ptr[d], n = level_ptr[d + 1] - i0;
        const uint32_t units = (uint32_t)n * (uint32_t)S.T;
        for (uint32_t u = blockIdx.x; u < units; u += G) {
            const int32_t item = __builtin_amdgcn_readfirstlane((int32_t)(u / (uint32_t)S.T));
            const int32_t tile = __builtin_amdgcn_readfirstlane((int32_t)u - item * S.T);
            const unsigned long long it = items[i0 + item];
            const BatchTree& BT = trees[(uint32_t)(it >> 32)];
            if (BT.status == nullptr || *BT.status == 0) {
                SensorDev St = S;
                St.rv = BT.rv;
                St.rv2 = BT.rv2;
                const MapDev M = BT.map;
                const TreeDev Tr = BT.td;
                trace_tile<true, kThreads>(M, St, Tr, (int32_t)(uint32_t)it, tile, s_bins);
            }
            __syncthreads();
        }
        if (!grid_barrier(sync, &target, spin_limit, &s_ok)) return;
        for (uint32_t u = blockIdx.x; u < (uint32_t)n; u += G) {
            finish_item(trees, items[i0 + (int32_t)u], S, s_p, s_best);
            __syncthreads();
        }
        if (!grid_barrier(sync, &target, spin_limit, &s_ok)) return;
        const int32_t m0 = mlevel_ptr[d];
        const uint32_t bunits = (uint32_t)(mlevel_ptr[d + 1] - m0) * (uint32_t)chunks;
        for (uint32_t u = blockIdx.x; u < bunits; u += G) {
            const int32_t item = __builtin_amdgcn_readfirstlane((int32_t)(u / (uint32_t)chunks));
            const int32_t chunk = __builtin_amdgcn_readfirstlane((int32_t)u - item * chunks);
            const unsigned long long it = mitems[m0 + item];
            const BatchTree& BT = trees[(uint32_t)(it >> 32)];
            if (BT.status == nullptr || *BT.status == 0) {
                SensorDev St = S;
                St.rv = BT.rv;
                St.rv2 = BT.rv2;
                const MapDev M = BT.map;
                const TreeDev Tr = BT.td;
                build_chunk(M, St, Tr, (int32_t)(uint32_t)it, chunk, bricks, smem, s_live, s_cw, s_b, &s_any);
            }
            __syncthreads();
        }
        if (d + 1 < levels && !grid_barrier(sync, &target, spin_limit, &s_ok)) return;
    }
}

// depth[n][j][i] = first hit of ray ((c0[n] + i) mod W, j)
__global__ void k_depth_out(SensorDev S, TreeDev Tr, float* __restrict__ depth) {
    const size_t per = (size_t)S.H * S.WB;
    const size_t total = per * (size_t)Tr.n;
    for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total; o += (size_t)gridDim.x * blockDim.x) {
        const int32_t node = (int32_t)(o / per);
        const int32_t rem = (int32_t)(o - (size_t)node * per);
        const int32_t j = rem / S.WB, i = rem - j * S.WB;
        int32_t c = Tr.c0[node] + i;
        c = c >= S.W ? c - S.W : c;
        depth[o] = Tr.dpan[(size_t)node * S.R + (size_t)c * S.H + j];
    }
}

// ---------------------------------------------------------------- launchers

static int grid_for(size_t n, int threads) {
    size_t g = (n + threads - 1) / threads;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_brick(const uint8_t* dense, uint8_t* bricks, const MapDev& m, hipStream_t s) {
    size_t total = (size_t)m.nbx * m.nby * m.nbz * 512u;
    hipLaunchKernelGGL(k_brick, dim3(grid_for(total, 256)), dim3(256), 0, s, dense, bricks, m);
    return hipGetLastError();
}

hipError_t launch_brick_flags(const MapDev& m, hipStream_t s) {
    const size_t threads = (size_t)(m.mask_words >> 4) * 64u;
    hipLaunchKernelGGL(k_brick_flags, dim3(grid_for(threads, 256)), dim3(256), 0, s, m);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_blocks16(m, s) : e;
}

hipError_t launch_blocks16(const MapDev& m, hipStream_t s) {
    const size_t threads = (size_t)(m.mask_words >> 4);
    hipLaunchKernelGGL(k_blocks16, dim3(grid_for(threads, 256)), dim3(256), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

int shape_count() { return kNumShapes; }

// The server's launch shape: one-wave trace workgroups and 256-brick builder
// chunks (its levels hold a few nodes of each request in flight, so small
// trace workgroups and few builder workgroups suit it; measured on 16 robots'
// requests: 9.25 -> 10.3 G rays/s saturated against shape 0).
static constexpr int find_shape(int threads, int bricks) {
    for (int i = 0; i < kNumShapes; ++i)
        if (kShapes[i].threads == threads && kShapes[i].bricks == bricks) return i;
    return 0;
}
int serve_shape() {
    constexpr int k = find_shape(64, 256);
    static_assert(kShapes[k].threads == 64 && kShapes[k].bricks == 256, "the server's shape is compiled");
    return k;
}

void shape_of(int shape, int* threads, int* bricks) {
    *threads = kShapes[shape].threads;
    *bricks = kShapes[shape].bricks;
}

size_t build_lds_bytes(const SensorDev& sd) {
    return sizeof(float2) * (sd.WB + 2) + sizeof(float) * (sd.H + 1) +
           sizeof(uint16_t) * (sd.n_lut_col + sd.n_lut_row);
}

size_t build_lds_total(const SensorDev& sd) { return build_lds_bytes(sd) + kBuildFixedLds; }

size_t lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64u * 1024u;
    return (size_t)v;
}

int32_t tiles_per_node(const SensorDev& sd, int shape) {
    return (sd.n_blocks * 64 + kShapes[shape].threads - 1) / kShapes[shape].threads;
}

hipError_t launch_trace(const MapDev& m, const SensorDev& sd, const TreeDev& td, const int32_t* nodes,
                        int32_t n_nodes, bool marginal, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    SensorDev st = sd;
    st.T = (sd.n_blocks * 64 + kTreeTraceThreads - 1) / kTreeTraceThreads;   // tiles per node at this size
    dim3 grid((unsigned)n_nodes * (unsigned)st.T);
    if (marginal)
        hipLaunchKernelGGL((k_trace<true>), grid, dim3(kTreeTraceThreads), 0, s, m, st, td, nodes);
    else
        hipLaunchKernelGGL((k_trace<false>), grid, dim3(kTreeTraceThreads), 0, s, m, st, td, nodes);
    return hipGetLastError();
}

static int32_t build_chunks(const MapDev& m, int32_t bricks) {
    return (int32_t)((m.build_slots + (uint32_t)bricks - 1) / (uint32_t)bricks);
}

// Builder chunk of a per-tree level: 256 bricks once the level still gives
// every CU about eight workgroups with them, else 64 (small levels need the
// finer split to fill the chip).
static int32_t tree_build_bricks(const MapDev& m, int32_t n_nodes) {
    return (int64_t)n_nodes * build_chunks(m, 256) >= 2048 ? 256 : 64;
}

hipError_t launch_mask_build(const MapDev& m, const SensorDev& sd, const TreeDev& td, const int32_t* nodes,
                             int32_t n_nodes, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    const int32_t bricks = tree_build_bricks(m, n_nodes), chunks = build_chunks(m, bricks);
    const size_t lds = build_lds_bytes(sd);
    if (lds + kBuildFixedLds > lds_limit()) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_mask_build, dim3((unsigned)n_nodes * (unsigned)chunks), dim3(kBuildThreads), lds, s, m, sd,
                       td, nodes, chunks, bricks);
    return hipGetLastError();
}

hipError_t launch_finish(const SensorDev& sd, const TreeDev& td, const int32_t* nodes, int32_t n_nodes,
                         bool marginal, uint32_t* gain, int32_t* yaw, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(n_nodes), dim3(kThreads), 0, s, sd, td, nodes, marginal ? 1 : 0, gain, yaw);
    return hipGetLastError();
}

hipError_t launch_depth_out(const SensorDev& sd, const TreeDev& td, float* depth, hipStream_t s) {
    size_t total = (size_t)sd.H * sd.WB * td.n;
    hipLaunchKernelGGL(k_depth_out, dim3(grid_for(total, 256)), dim3(256), 0, s, sd, td, depth);
    return hipGetLastError();
}

// ---------------------------------------------------------------- path score (eq. 3, eq. 4)

// Traversal cost (eq. 3) and exponential objective (eq. 4) of one node, summed
// from the root down its ancestor list (nearest first, so walked backwards) in
// the order the recursions take: c += |p_m - p_prev| and
// o += g(m) v^3 exp(-lambda c), in float64 on the float32 positions in metres.
__device__ __forceinline__ void score_node(const BatchTree& T, const uint32_t* __restrict__ g, int32_t node,
                                           double lambda, double* c_out, double* o_out) {
    const int32_t a0 = T.td.anc_ptr[node], a1 = T.td.anc_ptr[node + 1];
    int32_t prev = a1 > a0 ? T.td.anc_ids[a1 - 1] : node;      // the root
    double c = 0.0;
    double o = (double)g[prev] * T.vox3;
    for (int32_t k = a1 - 2; k >= a0 - 1; --k) {
        const int32_t m = k >= a0 ? T.td.anc_ids[k] : node;
        const float4 pa = T.td.pm[prev], pb = T.td.pm[m];
        const double dx = (double)pb.x - (double)pa.x;
        const double dy = (double)pb.y - (double)pa.y;
        const double dz = (double)pb.z - (double)pa.z;
        c = c + sqrt(dx * dx + dy * dy + dz * dz);
        o = o + (double)g[m] * T.vox3 * exp(-lambda * c);
        prev = m;
    }
    *c_out = c;
    *o_out = o;
}

// One thread per node of one tree (grid: blocks x trees).
__global__ void k_score(const BatchTree* __restrict__ trees, const uint32_t* __restrict__ gain, double lambda,
                        double* __restrict__ cost, double* __restrict__ obj) {
    const BatchTree& T = trees[blockIdx.y];
    const int32_t node = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (node >= T.td.n) return;
    double c, o;
    score_node(T, gain + T.out_off, node, lambda, &c, &o);
    if (cost) cost[T.out_off + node] = c;
    obj[T.out_off + node] = o;
}

// Whole workgroup: the node of largest objective among the threads'
// candidates (bo, bi), smallest id on ties, written to best[tree]; and (if
// asked) its root path, root first, padded with -1.
__device__ __forceinline__ void best_and_branch(const BatchTree& T, double bo, int32_t bi, int32_t tree,
                                                int32_t* __restrict__ best, int32_t* __restrict__ branch) {
    __shared__ double s_o[kThreads];
    __shared__ int32_t s_i[kThreads];
    s_o[threadIdx.x] = bo;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    for (int32_t off = kThreads / 2; off > 0; off >>= 1) {
        if ((int32_t)threadIdx.x < off) {
            const double po = s_o[threadIdx.x + off];
            const int32_t pi = s_i[threadIdx.x + off];
            const double mo = s_o[threadIdx.x];
            const int32_t mi = s_i[threadIdx.x];
            if (pi >= 0 && (mi < 0 || po > mo || (po == mo && pi < mi))) {
                s_o[threadIdx.x] = po;
                s_i[threadIdx.x] = pi;
            }
        }
        __syncthreads();
    }
    const int32_t b = s_i[0];
    if (threadIdx.x == 0) best[tree] = b;
    if (branch && threadIdx.x < kMaxAnc + 1) {
        const int32_t a0 = T.td.anc_ptr[b], d = T.td.anc_ptr[b + 1] - a0;     // ancestors, nearest first
        const int32_t t = (int32_t)threadIdx.x;
        branch[(size_t)tree * (kMaxAnc + 1) + t] = t < d ? T.td.anc_ids[a0 + d - 1 - t] : t == d ? b : -1;
    }
}

// One workgroup per tree: argmax over the objectives k_score wrote.
__global__ __launch_bounds__(kThreads) void k_best(const BatchTree* __restrict__ trees,
                                                   const double* __restrict__ obj, int32_t* __restrict__ best,
                                                   int32_t* __restrict__ branch) {
    const BatchTree& T = trees[blockIdx.x];
    const double* o = obj + T.out_off;
    double bo = 0.0;
    int32_t bi = -1;
    for (int32_t i = threadIdx.x; i < T.td.n; i += kThreads)
        if (bi < 0 || o[i] > bo) {           // ids ascend, so a later equal value never wins
            bo = o[i];
            bi = i;
        }
    best_and_branch(T, bo, bi, (int32_t)blockIdx.x, best, branch);
}

// Small trees: score and argmax in one launch, one workgroup per tree.
__global__ __launch_bounds__(kThreads) void k_score_best(const BatchTree* __restrict__ trees,
                                                         const uint32_t* __restrict__ gain, double lambda,
                                                         double* __restrict__ cost, double* __restrict__ obj,
                                                         int32_t* __restrict__ best, int32_t* __restrict__ branch) {
    const BatchTree& T = trees[blockIdx.x];
    double bo = 0.0;
    int32_t bi = -1;
    for (int32_t i = threadIdx.x; i < T.td.n; i += kThreads) {
        double c, o;
        score_node(T, gain + T.out_off, i, lambda, &c, &o);
        if (cost) cost[T.out_off + i] = c;
        obj[T.out_off + i] = o;
        if (bi < 0 || o > bo) {
            bo = o;
            bi = i;
        }
    }
    best_and_branch(T, bo, bi, (int32_t)blockIdx.x, best, branch);
}

// Trees of up to kFuseNodes nodes take the single-launch kernel.
constexpr uint32_t kFuseNodes = 8192;

hipError_t launch_score(const BatchTree* trees, int32_t n_trees, uint32_t max_nodes, const uint32_t* gain,
                        double lambda, double* cost, double* obj, int32_t* best, int32_t* branch, hipStream_t s) {
    if (max_nodes <= kFuseNodes) {
        hipLaunchKernelGGL(k_score_best, dim3((unsigned)n_trees), dim3(kThreads), 0, s, trees, gain, lambda, cost, obj,
                           best, branch);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_score, dim3((unsigned)grid_for(max_nodes, 256), (unsigned)n_trees), dim3(256), 0, s, trees,
                       gain, lambda, cost, obj);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_best, dim3((unsigned)n_trees), dim3(kThreads), 0, s, trees, obj, best, branch);
    return hipGetLastError();
}

}  // namespace mgk

namespace mgk {

hipError_t launch_batch_zero(const BatchTree* trees, int32_t n_trees, uint32_t max_nodes, const SensorDev& sd,
                             hipStream_t s) {
    const uint32_t blocks = (uint32_t)grid_for((size_t)max_nodes * 2 * sd.B, 256);
    hipLaunchKernelGGL(k_batch_zero, dim3(blocks, (unsigned)n_trees), dim3(256), 0, s, trees, 2 * sd.B);
    return hipGetLastError();
}

namespace {

template <int kTh>
void launch_multi(const BatchTree* trees, const unsigned long long* items, int32_t n_items, const SensorDev& sd,
                  hipStream_t s, hipEvent_t t0, hipEvent_t t1, int shape) {
    SensorDev st = sd;
    st.T = tiles_per_node(sd, shape);
    const dim3 grid((unsigned)n_items * (unsigned)st.T);
    if (t0 && t1)
        hipExtLaunchKernelGGL(k_trace_multi<kTh>, grid, dim3(kTh), 0, s, t0, t1, 0u, trees, items, st);
    else
        hipLaunchKernelGGL(k_trace_multi<kTh>, grid, dim3(kTh), 0, s, trees, items, st);
}

template <int I>
void launch_multi_shape(int shape, const BatchTree* trees, const unsigned long long* items, int32_t n_items,
                        const SensorDev& sd, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if constexpr (I < kNumShapes) {
        if (shape == I)
            launch_multi<kShapes[I].threads>(trees, items, n_items, sd, s, t0, t1, I);
        else
            launch_multi_shape<I + 1>(shape, trees, items, n_items, sd, s, t0, t1);
    }
}

}  // namespace

hipError_t launch_batch_level(const BatchTree* trees, const unsigned long long* items, int32_t n_items,
                              const unsigned long long* mitems, int32_t n_mitems, uint32_t mask_bricks,
                              const SensorDev& sd, hipStream_t s, int shape, hipEvent_t t0, hipEvent_t t1,
                              hipEvent_t b0, hipEvent_t b1) {
    if (n_items <= 0) return hipSuccess;
    if (shape < 0 || shape >= kNumShapes) return hipErrorInvalidValue;
    const size_t lds = build_lds_bytes(sd);
    if (lds + kBuildFixedLds > lds_limit()) return hipErrorInvalidConfiguration;
    launch_multi_shape<0>(shape, trees, items, n_items, sd, s, t0, t1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish_multi, dim3((unsigned)n_items), dim3(kThreads), 0, s, trees, items, sd);
    e = hipGetLastError();
    if (e != hipSuccess || n_mitems <= 0) return e;
    const int32_t bricks = kShapes[shape].bricks;
    const int32_t chunks = (int32_t)((mask_bricks + (uint32_t)bricks - 1) / (uint32_t)bricks);
    if ((uint64_t)n_mitems * (uint64_t)chunks >= (1ull << 32)) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)n_mitems * (unsigned)chunks);
    if (b0 && b1)
        hipExtLaunchKernelGGL(k_mask_build_multi, grid, dim3(kBuildThreads), lds, s, b0, b1, 0u, trees, mitems, sd,
                              chunks, bricks);
    else
        hipLaunchKernelGGL(k_mask_build_multi, grid, dim3(kBuildThreads), lds, s, trees, mitems, sd, chunks, bricks);
    return hipGetLastError();
}

hipError_t persistent_grid(const SensorDev& sd, int32_t* grid) {
    int dev = 0, cus = 0, coop = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e != hipSuccess) return e;
    if (!coop) return hipErrorNotSupported;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, kThreads, build_lds_bytes(sd));
    if (e != hipSuccess) return e;
    if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
    *grid = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_batch_persistent(const BatchTree* trees, const unsigned long long* items, const int32_t* level_ptr,
                                   const unsigned long long* mitems, const int32_t* mlevel_ptr, int32_t levels,
                                   uint32_t mask_bricks, const SensorDev& sd, uint32_t* sync, uint32_t spin_limit,
                                   hipStream_t s) {
    if (levels <= 0) return hipSuccess;
    const size_t lds = build_lds_bytes(sd);
    if (lds + kBuildFixedLds > lds_limit()) return hipErrorInvalidConfiguration;
    int32_t grid = 0;
    hipError_t e = persistent_grid(sd, &grid);
    if (e != hipSuccess) return e;
    SensorDev st = sd;
    st.T = tiles_per_node(sd, 0);
    int32_t bricks = kShapes[0].bricks;
    int32_t chunks = (int32_t)((mask_bricks + (uint32_t)bricks - 1) / (uint32_t)bricks);
    e = launch_zero_u32(sync, 2, s);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&trees, (void*)&items, (void*)&level_ptr, (void*)&mitems, (void*)&mlevel_ptr,
                    (void*)&levels, (void*)&st, (void*)&chunks, (void*)&bricks, (void*)&sync, (void*)&spin_limit};
    e = hipLaunchCooperativeKernel((const void*)k_batch_persistent, dim3((unsigned)grid), dim3(kThreads), args, lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace mgk
