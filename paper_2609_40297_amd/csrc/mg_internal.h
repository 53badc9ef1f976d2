// Internal device-side descriptors shared by the kernels and the host API.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgk {

constexpr int kThreads = 256;      // rays per workgroup (4 wave64)
constexpr int kMaxAnc = 64;        // deepest supported ancestor chain
constexpr int kMaxBins = 256;      // yaw bins
constexpr int kMaxAz = 4096;       // panorama columns (LDS holds their boundaries)
constexpr int kMaxEl = 2048;
constexpr int kRayBlockCols = 16;  // pixel block of one wave of the trace kernels: 16 columns
constexpr int kRayBlockRows = 4;   // by 4 rows
constexpr int kTileCols = 4;       // depth-cull tiles of a node's window: 4 columns
constexpr int kTileRows = 4;       // by 4 rows

// kOutside marks the padding around the grid: a traversal that reaches it
// has left the grid. The low two bits of a byte are the state, and bit 1 set
// (kOccupied, kOutside) ends a traversal. Bits 2-4 of an unknown or a free
// voxel name the largest aligned block around it that holds that state only
// (the traversal may cross such a block in one step): 1 its 16x16x16 block
// of 8 bricks, 2 its 8x8x8 brick (kUnknownBrick, kFreeBrick), 3 its 4x4x4
// quarter brick, 4 (free voxels only) its 2x2x2 block, 0 none; the block's
// edge is 32 >> level voxels.
enum : uint8_t { kUnknown = 0, kFree = 1, kOccupied = 2, kOutside = 3, kUnknownBrick = 8, kFreeBrick = 9 };
constexpr uint32_t kLevelShift = 2, kLevelMask = 7;
__host__ __device__ inline bool is_unknown(uint32_t s) { return (s & 3u) == 0u; }

// The block levels of one brick's voxels up to the brick (levels 2 to 4; the
// 16x16x16 blocks are marked afterwards, from the bricks' summaries), by one
// wave: each lane holds the 8 voxels (x = 0..7, bytes 0..7 of v) of row
// (y, z) = (lane & 7, lane >> 3) of the brick, as states or as marked bytes;
// returns them marked. any_unk, all_unk, all_free: whether the brick holds an
// unknown voxel, only unknown voxels, only free voxels.
__device__ __forceinline__ uint64_t mark_brick_row(uint64_t v, uint32_t lane, bool* any_unk, bool* all_unk,
                                                   bool* all_free_out) {
    const uint64_t ones = 0x0101010101010101ull;
    const uint64_t s8 = v & (3ull * ones);                       // the states, a byte each
    // (a byte is unknown when it is zero: states are below 0x80, so the borrow test is exact)
    const bool row_unk = ((s8 - ones) & ~s8 & (0x80ull * ones)) != 0ull;
    const bool all_free = __builtin_amdgcn_ballot_w64(s8 != ones) == 0ull;
    *all_free_out = all_free;
    *all_unk = __builtin_amdgcn_ballot_w64(s8 != 0ull) == 0ull;
    *any_unk = __builtin_amdgcn_ballot_w64(row_unk) != 0ull;
    if (all_free | *all_unk) return s8 | ((uint64_t)(2u << kLevelShift) * ones);   // (the whole brick: level 2)
    uint32_t fb = 0u, ub = 0u;          // per byte: free, unknown
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t s = (uint32_t)(s8 >> (8 * k)) & 0xffu;
        fb |= (s == kFree ? 1u : 0u) << k;
        ub |= (s == kUnknown ? 1u : 0u) << k;
    }
    // quarter bricks: x halves of the row, over the 4x4 rows (y, z) of the lane's quarter
    const uint32_t y = lane & 7u, z = lane >> 3;
    const uint64_t quarter = (0x0f0f0f0full << (y & 4u)) << (8u * (z & 4u));
    const uint64_t nf_lo = __builtin_amdgcn_ballot_w64((fb & 0x0fu) != 0x0fu), nf_hi = __builtin_amdgcn_ballot_w64((fb & 0xf0u) != 0xf0u);
    const uint64_t nu_lo = __builtin_amdgcn_ballot_w64((ub & 0x0fu) != 0x0fu), nu_hi = __builtin_amdgcn_ballot_w64((ub & 0xf0u) != 0xf0u);
    // 2x2x2 blocks: x pairs of the row, over the 2x2 rows of the lane's pair of rows
    const uint64_t pairs = 0x303ull << ((y & 6u) + 8u * (z & 6u));
    uint32_t f2 = 0u;                   // bit p: x pair p of this row lies in a wholly free block
#pragma unroll
    for (int p = 0; p < 4; ++p)
        f2 |= ((__builtin_amdgcn_ballot_w64(((fb >> (2 * p)) & 3u) != 3u) & pairs) == 0ull ? 1u : 0u) << p;
    const bool f4lo = (nf_lo & quarter) == 0ull, f4hi = (nf_hi & quarter) == 0ull;
    const bool u4lo = (nu_lo & quarter) == 0ull, u4hi = (nu_hi & quarter) == 0ull;
    uint64_t out = 0ull;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t s = (uint32_t)(v >> (8 * k)) & 3u;
        const bool f4 = k < 4 ? f4lo : f4hi, u4 = k < 4 ? u4lo : u4hi;
        uint32_t lv = 0u;
        if (s == kFree) lv = f4 ? 3u : (((f2 >> (k >> 1)) & 1u) ? 4u : 0u);
        if (s == kUnknown) lv = u4 ? 3u : 0u;
        out |= (uint64_t)(s | (lv << kLevelShift)) << (8 * k);
    }
    return out;
}

// Per brick of a path mask (one byte): its 512 bits are mixed, all clear (no
// voxel of the brick observed) or all set. Only unknown voxels' bits are ever
// read, so a mask keeps its code current for every brick that holds an
// unknown voxel, and its 16 words for such a brick whenever they can be read:
// the code is mixed, or the brick also holds known voxels (unknown voxels of
// such a brick are looked up by word, without the code). Words of bricks
// without unknown voxels, and of wholly unknown bricks with a uniform code,
// are never written.
enum : uint8_t { kMaskMixed = 0, kMaskNone = 1, kMaskAll = 2 };
// A brick's code word: bits 0-1 the code of its 512 bits, bits 2 + 2q and
// 3 + 2q the code of its quarter q (the 4x4x4 voxels with (x & 4, y & 4, z & 4)
// = 4 * (q & 1, (q >> 1) & 1, q >> 2)), bits 18-19 the code of its block of
// 2x2x2 bricks when those are all wholly unknown (else mixed).
__host__ __device__ inline uint32_t uniform_code_word(uint32_t c) { return c * 0x15555u; }
// brick_unk values (bits 0-1): no unknown voxel, some, all 512 (the
// kUnknownBrick marks); bit 2 (kBrickAllFree) set when all 512 are free
enum : uint8_t { kBrickKnown = 0, kBrickSomeUnknown = 1, kBrickAllUnknown = 2, kBrickAllFree = 4 };
__device__ __forceinline__ uint8_t brick_summary(bool any_unk, bool all_unk, bool all_free) {
    return (uint8_t)((any_unk ? (all_unk ? kBrickAllUnknown : kBrickSomeUnknown) : kBrickKnown) |
                     (all_free ? kBrickAllFree : 0));
}

// Occupancy grid in 8x8x8-voxel bricks (512 B each, x fastest inside a
// brick, bricks x fastest): a ray stays inside one brick for several steps,
// so its gathers hit few cache lines. Brick counts are powers of two with at
// least one padding voxel past the grid on every axis, so a voxel's byte
// address is a bit-field merge of its coordinates; coordinate -1 wraps to the
// last padding voxel of its axis, which holds kOutside like all padding.
struct MapDev {
    const uint8_t* bricks;
    int32_t nx, ny, nz;     // true extent in voxels
    int32_t nbx, nby, nbz;  // bricks per axis (powers of two, 8 * nb > n)
    uint32_t xm, ym, zm;    // brick-index bits of a coordinate: (8 * nb - 1) & ~7
    uint32_t shy, shz;      // left shifts placing (y & ym) and (z & zm) in the address
    uint32_t outside;       // address of a padding byte (kOutside)
    // Path masks (one bit per voxel, see mask_word): bricks per axis holding
    // the grid, ceil(n / 8), and 32-bit words per mask (16 per brick).
    uint32_t mbx, mby, mbz;
    uint32_t mask_words;
    // The mask builder visits bricks by blocks of 2x2x2 (ceil(mb / 2) blocks per
    // axis, x fastest; in a block x, then y, then z): slots = 8 * blocks.
    uint32_t build_slots;
    // [mbx * mby * mbz] per mask brick: kBrickKnown, kBrickSomeUnknown or
    // kBrickAllUnknown, with kBrickAllFree (kept current, with the block
    // marks, by every write of the map's states)
    uint8_t* brick_unk;
};

// Byte address of voxel (x, y, z) in the bricked grid, for -1 <= x <= nx
// (likewise y, z): bits 0-8 are the position inside the brick, then the brick
// index x-fastest.
__host__ __device__ inline uint32_t voxel_addr(int32_t x, int32_t y, int32_t z, const MapDev& M) {
    const uint32_t ux = (uint32_t)x, uy = (uint32_t)y, uz = (uint32_t)z;
    return (ux & 7u) | ((uy & 7u) << 3) | ((uz & 7u) << 6) | ((ux & M.xm) << 6) | ((uy & M.ym) << M.shy) |
           ((uz & M.zm) << M.shz);
}

// Path masks: one bit per voxel of the grid, in 8x8x8 bricks of 512 bits (16
// words), bricks x fastest with tight counts mbx = ceil(nx / 8) etc. Voxel
// (x, y, z) is bit (x & 7) | (y & 3) << 3 of word (z & 7) << 1 | (y & 7) >> 2
// of its brick, i.e. bit (x & 7) | (y & 7) << 3 | (z & 7) << 6 of the brick's
// 512 bits: a z-slice of a brick is 64 consecutive bits, two words.
__device__ __forceinline__ uint32_t mask_word(int32_t x, int32_t y, int32_t z, const MapDev& M) {
    const uint32_t b = (uint32_t)(x >> 3) + __umul24(M.mbx, (uint32_t)(y >> 3) + __umul24(M.mby, (uint32_t)(z >> 3)));
    return (b << 4) | ((uint32_t)(z & 7) << 1) | ((uint32_t)(y & 4) >> 2);
}
__device__ __forceinline__ uint32_t mask_bit(int32_t x, int32_t y) { return (uint32_t)(x & 7) | ((uint32_t)(y & 3) << 3); }
__device__ __forceinline__ uint32_t mask_brick(int32_t x, int32_t y, int32_t z, const MapDev& M) {
    return (uint32_t)(x >> 3) + __umul24(M.mbx, (uint32_t)(y >> 3) + __umul24(M.mby, (uint32_t)(z >> 3)));
}

// How many of one axis's boundaries b0, b0 + db, b0 + 2 db, ... the DDA
// crosses before the crossing at parameter Tc: those with parameter
// t = (b - q) * f below Tc (a caller that wants ties counted passes the next
// float above the crossing). Parameters grow by at least 1 from one boundary
// to the next, so these boundaries are a prefix; the caller's crossing leaves
// a block of at most 16 voxels a side, so the prefix ends at the axis's own
// exit from that block, at most 15 boundaries on. Three probes (at 3, then
// 3 +- 2, then +- 1) find its length when the block's edge is at most 8; a
// first probe at 7 (then 11 or 3) extends the search to 15 (`wide`). Boundaries are evaluated exactly as the single step
// evaluates them (the fused multiply-add of integers is exact). Returned as a
// float count.
__device__ __forceinline__ float crossings_before(float b0, float db, float q, float f, float Tc, bool wide) {
    float m = 3.f;
    if (wide) m = ((__builtin_fmaf(7.f, db, b0) - q) * f < Tc) ? 11.f : 3.f;
    m += ((__builtin_fmaf(m, db, b0) - q) * f < Tc) ? 2.f : -2.f;
    m += ((__builtin_fmaf(m, db, b0) - q) * f < Tc) ? 1.f : -1.f;
    return m + (((__builtin_fmaf(m, db, b0) - q) * f < Tc) ? 1.f : 0.f);
}

// One step over the marked block (wholly free or wholly unknown, `edge` voxels
// a side) that voxel (ix, iy, iz) lies in, taken as the per-voxel trace
// takes it: the block is left through the face whose boundary parameter comes
// first (ties x, then y, then z), and every axis has crossed the boundaries
// whose parameters come before that crossing in the same order, which is where
// the voxel-by-voxel DDA stands once it has left the block. Updates the voxel,
// the next boundaries (integers) and their parameters, and returns the entry
// parameter of the voxel it enters.
__device__ __forceinline__ float cross_block(int32_t edge, float4 p, float4 inv, int32_t sx, int32_t sy, int32_t sz,
                                             int32_t& ix, int32_t& iy, int32_t& iz, int32_t& bx, int32_t& by,
                                             int32_t& bz, float& tx, float& ty, float& tz) {
    const float inf = __builtin_inff();
    // (an axis the ray does not move along: boundary +inf, node -inf, factor 1,
    // so each of its parameters is +inf)
    const float qx = sx ? p.x : -inf, qy = sy ? p.y : -inf, qz = sz ? p.z : -inf;
    const float fx = sx ? inv.x : 1.f, fy = sy ? inv.y : 1.f, fz = sz ? inv.z : 1.f;
    const float Tx = ((float)((ix & -edge) + (sx > 0 ? edge : 0)) - qx) * fx;
    const float Ty = ((float)((iy & -edge) + (sy > 0 ? edge : 0)) - qy) * fy;
    const float Tz = ((float)((iz & -edge) + (sz > 0 ? edge : 0)) - qz) * fz;
    const bool ex = (Tx <= Ty) & (Tx <= Tz);
    const bool ey = !ex & (Ty <= Tz);
    const bool ez = !ex & !ey;
    const float T = ex ? Tx : (ey ? Ty : Tz);
    // an axis before the exit axis in the tie order also crosses a boundary at
    // exactly T: it compares with the next float above T (T >= 0; +0 for -0)
    const float Tn = __uint_as_float(__float_as_uint(T + 0.f) + 1u);
    const bool wide = edge > 8;
    const int32_t kx = (int32_t)crossings_before(sx ? (float)bx : inf, (float)sx, qx, fx, ex ? T : Tn, wide) + (ex ? 1 : 0);
    const int32_t ky = (int32_t)crossings_before(sy ? (float)by : inf, (float)sy, qy, fy, ez ? Tn : T, wide) + (ey ? 1 : 0);
    const int32_t kz = (int32_t)crossings_before(sz ? (float)bz : inf, (float)sz, qz, fz, T, wide) + (ez ? 1 : 0);
    ix += kx * sx; bx += kx * sx;
    iy += ky * sy; by += ky * sy;
    iz += kz * sz; bz += kz * sz;
    tx = sx ? ((float)bx - p.x) * inv.x : inf;
    ty = sy ? ((float)by - p.y) * inv.y : inf;
    tz = sz ? ((float)bz - p.z) * inv.z : inf;
    return T;
}

// Panorama ray tables and yaw-window geometry (built on the host, see mg_api).
struct SensorDev {
    const float4* d4;          // [R] unit direction (w unused)
    const float4* iv4;         // [R] 1/d per component, 0 where d == 0
    const int32_t* bin_of_col; // [W]
    const float2* bv;          // [W] left boundary unit vector of each column
    const float* ts;           // [H+1] tan(e)|tan(e)| at the row boundaries
    const int32_t* c0_of_win;  // [B] first column of window k
    int32_t W, H, B, w, WB, R, T;   // R = W*H rays, T = workgroups per node
    // The trace kernels give each wave a block of kRayBlockCols x kRayBlockRows
    // pixels (rays of one block have similar lengths, so a wave's lanes finish
    // at similar steps); blocks are numbered row block fastest.
    int32_t nrb;               // row blocks, ceil(H / kRayBlockRows)
    int32_t n_blocks;          // ceil(W / kRayBlockCols) * nrb
    // Depth cull of the path-mask builder: a window's pixels in tiles of
    // kTileCols x kTileRows (tcols x trows tiles, column-major), and float
    // angles that place a direction's pixel to within a pixel: azimuth of
    // column 0's left boundary and columns per radian, elevation of row 0's
    // lower boundary and rows per radian.
    int32_t tcols, trows, n_tiles;
    float az0, daz_inv, el0, del_inv;
    float rv;                  // range in voxel units
    float rv2;                 // rv*rv (no depth can exceed it)
    // Guess tables for the pixel lookup (a guess only picks where the exact
    // boundary comparisons start): column from a pseudo-angle past the
    // window's left boundary, row from the elevation tangent.
    const uint16_t* lut_col;   // [n_lut_col]
    const uint16_t* lut_row;   // [n_lut_row]
    int32_t n_lut_col, n_lut_row;
    float lut_col_scale;       // pseudo-angle -> lut_col index
    float lut_row_lo;          // tangent at the bottom of the band
    float lut_row_scale;       // tangent -> lut_row index
};

// One tree's device state. Depth buffers are kept as full panoramas: the
// first-hit parameter of every ray of node n lives at dpan[n*R + r] and the
// node's buffer is the window slice starting at column c0[n]. Every node with
// children has a path mask (mask_slot[n] >= 0): the set of voxels that n or
// one of its ancestors observes (with anc_cap = 1: that n observes), which is
// what conditions n's children.
struct TreeDev {
    const float4* q4;          // [n] position in voxel units
    const float4* pm;          // [n] position in metres, as given
    const int32_t* anc_ptr;    // [n+1] CSR into anc_ids
    const int32_t* anc_ids;    // ancestors, nearest first
    const int32_t* level_nodes;// [n] nodes sorted by depth
    const int32_t* child_ptr;  // [n+1]
    const int32_t* child_ids;
    uint32_t* bins;            // [n][2][B]: absolute, then marginal
    float* dpan;               // [n][R]
    int32_t* c0;               // [n]
    uint32_t* masks;           // [nodes with children][mask_words]
    const int32_t* mask_slot;  // [n] index into masks, -1 for a leaf
    const int32_t* mask_nodes; // nodes with children, by depth level
    float* tmax;               // [nodes with children][2][n_tiles]: largest, then smallest first hit of each tile of the window
    uint32_t* mcode;           // [nodes with children][mask bricks]: code words
    int32_t n;
    int32_t anc_cap;           // ancestors that condition a node: kMaxAnc (all) or 1 (the parent only)
};

// One tree of a multi-tree launch: its map and node data, its range in voxel
// units (maps may differ in voxel size) and where its outputs go.
struct BatchTree {
    MapDev map;
    TreeDev td;
    float rv, rv2;
    double vox3;               // voxel volume (m^3): a gain count times this is a volume
    uint32_t out_off;          // first node of this tree in the concatenated outputs
    uint32_t* gain;            // [n]
    int32_t* yaw;              // [n]
    float* depth;              // [n][H][WB] or NULL
    // Device status word of the tree's request, or NULL: nonzero marks the
    // request failed, and every later kernel of it returns at once.
    const int32_t* status;
};

// Launchers (mg_kernels.hip).
hipError_t launch_brick(const uint8_t* dense, uint8_t* bricks, const MapDev& m, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s);
// Map contents (mg_map.hip): TSDF conversion of the whole grid or of a box,
// listed voxel updates, and a dense copy of the states.
hipError_t launch_tsdf_grid(const float* dist, const float* weight, const MapDev& m, float surface, float min_weight,
                            hipStream_t s);
hipError_t launch_tsdf_box(const float* dist, const float* weight, const MapDev& m, const int32_t lo[3],
                           const int32_t size[3], float surface, float min_weight, hipStream_t s);
hipError_t launch_map_scatter(const uint32_t* ids, const uint8_t* states, uint32_t count, const MapDev& m,
                              uint32_t* rejected, hipStream_t s);
hipError_t launch_unbrick(const MapDev& m, uint8_t* dense, hipStream_t s, bool marks = false);
hipError_t launch_fill_outside(const MapDev& m, hipStream_t s);
// Recomputes brick_unk and the block marks from the states (after any write
// of the states): the bricks' summaries, then the 16x16x16 blocks.
hipError_t launch_brick_flags(const MapDev& m, hipStream_t s);
// The 16x16x16 blocks alone (after a conversion that took the bricks' summaries itself).
hipError_t launch_blocks16(const MapDev& m, hipStream_t s);
hipError_t launch_trace(const MapDev& m, const SensorDev& sd, const TreeDev& td, const int32_t* nodes,
                        int32_t n_nodes, bool marginal, hipStream_t s);
// Path masks of the listed nodes (all with children), after their windows are chosen.
hipError_t launch_mask_build(const MapDev& m, const SensorDev& sd, const TreeDev& td, const int32_t* nodes,
                             int32_t n_nodes, hipStream_t s);
hipError_t launch_finish(const SensorDev& sd, const TreeDev& td, const int32_t* nodes, int32_t n_nodes,
                         bool marginal, uint32_t* gain, int32_t* yaw, hipStream_t s);
hipError_t launch_depth_out(const SensorDev& sd, const TreeDev& td, float* depth, hipStream_t s);
// Launch shapes (shape 0 = default): rays per workgroup of the trace kernel
// and bricks per workgroup of the mask builder.
int shape_count();
void shape_of(int shape, int* threads, int* bricks);
int serve_shape();                         // the launch shape the server's level launches use
int32_t tiles_per_node(const SensorDev& sd, int shape);
size_t lds_limit();                        // LDS bytes one workgroup may use on the current device
size_t build_lds_bytes(const SensorDev& sd);   // LDS of the mask builder (sensor tables)
size_t build_lds_total(const SensorDev& sd);   // and with its fixed arrays
// Path score of every node of the trees (eq. 3, eq. 4) and each tree's best node.
hipError_t launch_score(const BatchTree* trees, int32_t n_trees, uint32_t max_nodes, const uint32_t* gain,
                        double lambda, double* cost, double* obj, int32_t* best, int32_t* branch, hipStream_t s);
hipError_t launch_batch_zero(const BatchTree* trees, int32_t n_trees, uint32_t max_nodes, const SensorDev& sd,
                             hipStream_t s);
// One depth level of many trees: trace with launch shape `shape`, window
// selection, then the path masks of the level's nodes with children
// (`mitems`, a subset of `items`). t0/t1 and b0/b1 (may be null): events the
// trace and the builder dispatches themselves record at their start and end.
// mask_bricks: build slots (MapDev::build_slots) of the largest map among the launch's trees.
hipError_t launch_batch_level(const BatchTree* trees, const unsigned long long* items, int32_t n_items,
                              const unsigned long long* mitems, int32_t n_mitems, uint32_t mask_bricks,
                              const SensorDev& sd, hipStream_t s, int shape = 0, hipEvent_t t0 = nullptr,
                              hipEvent_t t1 = nullptr, hipEvent_t b0 = nullptr, hipEvent_t b1 = nullptr);
// The whole batch in one cooperative launch of co-resident workgroups: for each
// depth level d, the trace of items[level_ptr[d] .. level_ptr[d + 1]), their
// windows, then the path masks of mitems[mlevel_ptr[d] .. mlevel_ptr[d + 1]),
// with grid barriers between the phases. sync: 2 device words (zeroed here);
// sync[1] != 0 afterwards when a barrier wait gave up after spin_limit polls.
hipError_t launch_batch_persistent(const BatchTree* trees, const unsigned long long* items, const int32_t* level_ptr,
                                   const unsigned long long* mitems, const int32_t* mlevel_ptr, int32_t levels,
                                   uint32_t mask_bricks, const SensorDev& sd, uint32_t* sync, uint32_t spin_limit,
                                   hipStream_t s);
// Workgroups of the persistent launch: the co-resident capacity of the device.
hipError_t persistent_grid(const SensorDev& sd, int32_t* grid);

}  // namespace mgk
