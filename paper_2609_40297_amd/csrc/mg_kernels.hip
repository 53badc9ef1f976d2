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
__device__ __forceinline__ gbytes_t as_global(const uint8_t* p) { return (gbytes_t)p; }
__device__ __forceinline__ gfloats_t as_global(const float* p) { return (gfloats_t)p; }

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

__global__ void k_zero_u32(uint32_t* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------- ancestor test

struct AncLDS {
    float qx, qy, qz;
    int32_t c0;
    float b0x, b0y;       // left boundary of the window
    float b1x, b1y;       // right boundary (left boundary of column c0 + w_buf)
    uint32_t dpan_off;    // element offset of the ancestor's panorama of first hits
    uint32_t pad[3];
};

__device__ __forceinline__ int32_t wrap(int32_t c, int32_t W) { return c >= W ? c - W : c; }

// r lies at or to the left (counter-clockwise side) of boundary direction b.
__device__ __forceinline__ bool left_of(float2 b, float rx, float ry) { return b.x * ry - b.y * rx >= 0.f; }

// Does ancestor A see the voxel centre (cx, cy, cz)? The centre must fall in a
// pixel cell of A's window (azimuth between two column boundaries, elevation
// between two row boundaries; cells half-open) and its squared range from A
// must be <= the squared depth stored for that pixel. Row and column are the
// numbers of inner boundaries the centre lies at-or-beyond; a table lookup
// guesses them and the exact boundary comparisons settle them. Those
// comparisons are monotone along the boundaries, so the settled index is the
// exact count whatever the guess. The cheap rejections come first: the
// wedge, then range and band as one mask. A lane with act false (no queue
// entry) gets true, so that its negation keeps nothing.
__device__ __forceinline__ bool ancestor_sees(const AncLDS& A, float cx, float cy, float cz, bool act,
                                              const SensorDev& S, const float2* __restrict__ s_bv,
                                              const float* __restrict__ s_ts,
                                              float ts0, float tsH, const uint16_t* __restrict__ s_lut_col,
                                              const uint16_t* __restrict__ s_lut_row,
                                              const float* __restrict__ dpan) {
    const float rx = cx - A.qx;
    const float ry = cy - A.qy;
    const float w0 = A.b0x * ry - A.b0y * rx;
    const float w1 = A.b1x * ry - A.b1y * rx;
    // The result is one comparison after the lookup (so that a ballot of it
    // takes the comparison's mask as it stands): lanes outside the window, band
    // or range keep a limit of -1, which no squared range meets (their range2
    // is 0 unless computed); lanes without an entry (act false) a limit of
    // +inf, which every one meets. The wedge is tested first and alone: the
    // voxels of a chunk often lie outside an ancestor's window together, and
    // the wave then skips the rest.
    float lim = act ? -1.f : __builtin_inff();
    float range2 = 0.f;
    if (act & (w0 >= 0.f) & (w1 < 0.f)) {
        const float rz = cz - A.qz;
        const float rho2 = rx * rx + ry * ry;
        range2 = rho2 + rz * rz;
        const float sz = rz * fabsf(rz);
        if ((range2 <= S.rv2) & (sz >= rho2 * ts0) & (sz < rho2 * tsH)) {
            // Column: pseudo-angle past the left boundary (monotone in the angle) picks a
            // table bucket holding at most one column boundary, giving a guess gc. The
            // boundaries gc, gc + 1 and gc + 2 of the window are read at once (the LDS
            // table holds the boundaries twice over, so window boundary k is entry
            // c0 + k). When boundary gc lies at or left of r and gc + 2 does not, the
            // column is gc + 1 if boundary gc + 1 does and gc otherwise. Other lanes
            // (rounding at a bucket edge) settle with the boundary-by-boundary walk,
            // which also returns gc + l1 in the two patterns that break monotonicity
            // (1-0-1 and 0-1-0).
            const float u0 = A.b0x * rx + A.b0y * ry;
            float pa = w0 * __builtin_amdgcn_rcpf(fabsf(u0) + w0);
            pa = u0 < 0.f ? 2.f - pa : pa;
            // (pa and tg are finite here: the wedge excludes r = 0 in x and y, so
            // one median-of-three clamps the table index)
            const int32_t gc =
                s_lut_col[(int32_t)__builtin_amdgcn_fmed3f(pa * S.lut_col_scale, 0.f, (float)(S.n_lut_col - 1))];
            const int32_t cb = A.c0 + gc;
            const float2 v0 = s_bv[cb], v1 = s_bv[cb + 1], v2 = s_bv[cb + 2];
            const bool l0 = (gc == 0) | left_of(v0, rx, ry);
            const bool l1 = (gc + 1 < S.WB) & left_of(v1, rx, ry);
            const bool l2 = (gc + 2 < S.WB) & left_of(v2, rx, ry);
            // (and/or rather than a select, so that all three reads stay unconditional)
            int32_t col = gc + (int32_t)l1;
            const bool c_ok = l0 & !l2;
            if (!c_ok) {      // (a divergent branch: skipped when no lane needs it)
                for (;;) {
                    if (col + 1 >= S.WB || !left_of(s_bv[A.c0 + col + 1], rx, ry)) break;
                    ++col;
                }
                for (;;) {
                    if (col == 0 || left_of(s_bv[A.c0 + col], rx, ry)) break;
                    --col;
                }
            }
            // Row: elevation tangent picks a bucket holding at most one row boundary;
            // the same three-boundary decision, same fallback.
            const float tg = rz * __builtin_amdgcn_rsqf(rho2);
            const int32_t gr = s_lut_row[(int32_t)__builtin_amdgcn_fmed3f((tg - S.lut_row_lo) * S.lut_row_scale, 0.f,
                                                                          (float)(S.n_lut_row - 1))];
            const float e0 = s_ts[gr], e1 = s_ts[gr + 1], e2 = s_ts[min(gr + 2, S.H)];
            const bool r0 = (gr == 0) | (sz >= rho2 * e0);
            const bool r1 = (gr + 1 < S.H) & (sz >= rho2 * e1);
            const bool r2 = (gr + 2 < S.H) & (sz >= rho2 * e2);
            int32_t row = gr + (int32_t)r1;
            const bool r_ok = r0 & !r2;
            if (!r_ok) {
                for (;;) {
                    if (row + 1 >= S.H || !(sz >= rho2 * s_ts[row + 1])) break;
                    ++row;
                }
                for (;;) {
                    if (row == 0 || sz >= rho2 * s_ts[row]) break;
                    --row;
                }
            }
            // (column < 4096 and H <= 2048: the product fits the 24-bit multiplier)
            const float D =
                as_global(dpan)[A.dpan_off + __umul24((uint32_t)wrap(A.c0 + col, S.W), (uint32_t)S.H) + (uint32_t)row];
            lim = D * D;
        }
    }
    return range2 <= lim;
}

// ---------------------------------------------------------------- ray traversal

// Launch shapes of the trace kernel (rays per workgroup, queued unknown
// voxels per wave), all compiled; shape 0 is the default.
struct Shape {
    int threads, queue;
};
constexpr Shape kShapes[] = {{256, 512}, {256, 384}, {256, 256}, {128, 512}, {128, 256}, {512, 256}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);


__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Queue entry: .x = x | y << 16, .y = z | bin << 16 | (m - 1) << 24, where m
// (1..64) is the number of ray incidences the entry stands for: neighbouring
// lanes that reach the same unknown voxel in the same step, with the same bin,
// share one entry (the ancestor test depends on the voxel alone).
__device__ __forceinline__ uint32_t entry_bin(uint32_t ey) { return (ey >> 16) & 0xffu; }

// Adds the incidences of the queued entries to their bins: per distinct bin,
// the sum of the entries' multiplicities is assembled from ballots bit by bit.
__device__ __forceinline__ void count_by_bin(const uint2* __restrict__ q, int32_t n, uint32_t* __restrict__ bins,
                                             int32_t lane) {
    for (int32_t base = 0; base < n; base += 64) {
        const int32_t i = base + lane;
        bool pending = i < n;
        const uint32_t ey = pending ? q[i].y : 0u;
        const uint32_t bin = entry_bin(ey);
        const uint32_t extra = ey >> 24;      // multiplicity - 1, 6 bits
        uint64_t left = ballot(pending);
        while (left) {
            const int32_t leader = __builtin_ctzll(left);
            const uint32_t b = __shfl(bin, leader, 64);
            const bool mine = pending && bin == b;
            const uint64_t same = ballot(mine);
            uint32_t sum = (uint32_t)__popcll(same);
#pragma unroll
            for (int32_t k = 0; k < 6; ++k) sum += (uint32_t)__popcll(ballot(mine && ((extra >> k) & 1u))) << k;
            if (lane == leader) atomicAdd(&bins[b], sum);
            pending = pending && bin != b;
            left &= ~same;
        }
    }
}

// Tests the n queued voxels against the ancestors, nearest first. Each pass
// tests every voxel still unobserved against one ancestor and compacts the
// survivors in place (a lane writes its survivor only after the whole chunk
// has been read, and survivors never overtake the read position). What is left
// after the last ancestor is new to the path and counts into the marginal bins.
__device__ __forceinline__ void drain_queue(uint2* __restrict__ q, int32_t n, const AncLDS* __restrict__ s_anc,
                                            int32_t na, const SensorDev& S, const float2* __restrict__ s_bv,
                                            const float* __restrict__ s_ts, const uint16_t* __restrict__ s_lut_col,
                                            const uint16_t* __restrict__ s_lut_row, const float* __restrict__ dpan,
                                            uint32_t* __restrict__ marg_bins, int32_t lane) {
    const float ts0 = s_ts[0], tsH = s_ts[S.H];
    for (int32_t k = 0; k < na && n > 0; ++k) {
        const AncLDS A = s_anc[k];
        int32_t m = 0;
        for (int32_t base = 0; base < n; base += 64) {
            const int32_t i = base + lane;
            const bool act = i < n;
            const uint2 e = act ? q[i] : make_uint2(0u, 0u);
            // (lanes without an entry run the cheap rejections on voxel 0 and
            // are masked out)
            const float cx = (float)(int32_t)(e.x & 0xffffu) + 0.5f;
            const float cy = (float)(int32_t)(e.x >> 16) + 0.5f;
            const float cz = (float)(int32_t)(e.y & 0xffffu) + 0.5f;
            const bool keep = !ancestor_sees(A, cx, cy, cz, act, S, s_bv, s_ts, ts0, tsH, s_lut_col, s_lut_row, dpan);
            const uint64_t bal = ballot(keep);
            if (keep) q[m + (int32_t)lane_prefix(bal)] = e;
            m += __popcll(bal);
        }
        n = m;
    }
    count_by_bin(q, n, marg_bins, lane);
}

struct TraceLDS {
    float2* bv;
    float* ts;
    uint32_t* bins;
    AncLDS* anc;
    uint2* queue;
    uint16_t* lut_col;
    uint16_t* lut_row;
};

// LDS carve-up: boundary table (twice over) | row table | bins [2B] | guess tables |
// per-wave queues | ancestors (as many as the launch provides for).
template <int kTh, int kQ>
__device__ __forceinline__ TraceLDS carve_lds(char* smem, const SensorDev& S) {
    TraceLDS L;
    L.bv = reinterpret_cast<float2*>(smem);                 // column boundaries twice over: [2W + 1]
    L.ts = reinterpret_cast<float*>(L.bv + 2 * S.W + 1);
    L.bins = reinterpret_cast<uint32_t*>(L.ts + S.H + 1);
    L.lut_col = reinterpret_cast<uint16_t*>(L.bins + 2 * S.B);
    L.lut_row = L.lut_col + S.n_lut_col;
    char* tail = smem + ((reinterpret_cast<char*>(L.lut_row + S.n_lut_row) - smem + 15) & ~static_cast<ptrdiff_t>(15));
    L.queue = reinterpret_cast<uint2*>(tail);
    L.anc = reinterpret_cast<AncLDS*>(L.queue + kQ * (kTh / 64));
    return L;
}

template <int kTh>
__device__ __forceinline__ void load_tables(const TraceLDS& L, const SensorDev& S) {
    for (int32_t i = threadIdx.x; i <= 2 * S.W; i += kTh) L.bv[i] = S.bv[i < S.W ? i : (i < 2 * S.W ? i - S.W : 0)];
    for (int32_t i = threadIdx.x; i <= S.H; i += kTh) L.ts[i] = S.ts[i];
    for (int32_t i = threadIdx.x; i < S.n_lut_col; i += kTh) L.lut_col[i] = S.lut_col[i];
    for (int32_t i = threadIdx.x; i < S.n_lut_row; i += kTh) L.lut_row[i] = S.lut_row[i];
}

// One workgroup = kTh consecutive rays (tile `tile`) of one node; each
// wave owns a queue in LDS. A lane walks its ray with the Amanatides-Woo 3D
// DDA (face-crossing parameters recomputed as (boundary - q) * (1/d); ties
// step x, then y, then z; a voxel is visited while its entry parameter is
// below the range and it is inside the grid). The grid byte of the next voxel
// is loaded one step ahead. An occupied voxel ends the ray and its entry
// parameter (or the range) is the ray's first hit; unknown voxels count into
// the absolute bin of the ray's column and, in marginal mode, are queued;
// whenever the queue could overflow it is drained against the ancestors.
// Requires the tables in LDS; ends with the tile's bins added to the node's
// global bins.
//
// kAhead = 2 keeps two voxels in flight per lane instead of one: the walk's
// front runs a step ahead of the voxel being examined, so a grid load has a
// whole step of work to hide behind. Launches with few waves per SIMD (the
// small levels near the root) are bound by that load latency rather than by
// instruction issue; results are the same either way.
template <bool kMarginal, int kTh, int kQ, int kAhead = 1>
__device__ __forceinline__ void trace_tile(const MapDev& M, const SensorDev& S, const TreeDev& Tr, int32_t node,
                                           int32_t tile, const TraceLDS& L) {
    const int32_t tid = threadIdx.x;
    const int32_t lane = tid & 63;
    int32_t na = 0;
    if (kMarginal) {
        const int32_t a0 = Tr.anc_ptr[node];
        na = min(Tr.anc_ptr[node + 1] - a0, Tr.anc_cap);     // the list is nearest first
        for (int32_t k = tid; k < na; k += kTh) {
            const int32_t a = Tr.anc_ids[a0 + k];
            const float4 qa = Tr.q4[a];
            const int32_t c0 = Tr.c0[a];
            int32_t c1 = c0 + S.WB;
            c1 = c1 >= S.W ? c1 - S.W : c1;
            const float2 b0 = S.bv[c0], b1 = S.bv[c1];   // global copy: LDS tables are not yet synchronised
            AncLDS A;
            A.qx = qa.x; A.qy = qa.y; A.qz = qa.z; A.c0 = c0;
            A.b0x = b0.x; A.b0y = b0.y; A.b1x = b1.x; A.b1y = b1.y;
            A.dpan_off = (uint32_t)a * (uint32_t)S.R;
            A.pad[0] = A.pad[1] = A.pad[2] = 0u;
            L.anc[k] = A;
        }
    }
    for (int32_t i = tid; i < 2 * S.B; i += kTh) L.bins[i] = 0u;
    __syncthreads();

    uint2* q = L.queue + (tid >> 6) * kQ;
    const int32_t r = tile * kTh + tid;
    const bool has_ray = r < S.R;
    const int32_t rr = has_ray ? r : 0;
    const int32_t bin = S.bin_of_col[rr / S.H];
    // lanes whose previous lane has the same bin (DPP wave shift right by one;
    // lane 0 receives -1)
    const bool bin_as_prev = __builtin_amdgcn_update_dpp(-1, bin, 0x138, 0xf, 0xf, false) == bin;
    const uint64_t bin_as_prev_mask = ballot(bin_as_prev);
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
    float tx = (bx - p.x) * fx;
    float ty = (by - p.y) * fy;
    float tz = (bz - p.z) * fz;
    float t = 0.f, h = S.rv;
    uint32_t n_abs = 0;
    const uint32_t ebin = (uint32_t)bin << 16;
    const gbytes_t grid = as_global(M.bricks);
    // the node lies inside the grid and t = 0 < rv, so its own voxel is
    // visited; a lane without a ray reads a padding byte and is done at once
    int32_t qn = 0;
    if constexpr (kAhead == 1) {
    uint32_t addr = has_ray ? voxel_addr(ix, iy, iz, M) : M.outside;   // address of the current voxel
    uint32_t st = grid[addr];
    uint64_t alive = ballot(has_ray);
    while (alive) {
        // Straight-line step without divergent branches: the current voxel's
        // byte is used first, then the next voxel is found and its byte
        // requested, so the load stays in flight until the next step uses it.
        // A lane that has finished (or left the grid) reads a padding byte,
        // which is neither unknown nor occupied. The first lane of each run
        // of equal unknown voxels writes the queue entry.
        do {
            const bool unk = st == kUnknown;
            const bool occ = st == kOccupied;
            h = occ ? t : h;
            if (!kMarginal) n_abs += unk ? 1u : 0u;
            // queueing (and the absolute count, which adds nothing in other
            // steps) runs only in steps where some lane of the wave is on an
            // unknown voxel (a wave-uniform branch)
            if (kMarginal && ballot(unk) != 0) {
                n_abs += unk ? 1u : 0u;
                // a lane whose unknown voxel and bin equal the previous lane's
                // joins that lane's entry; the first lane of each run appends
                // one entry carrying the run's length. Keys of other lanes are
                // distinct values above every address. (Lane 0 receives 0 from
                // the shift; it is never a duplicate, its bin_as_prev being
                // false.)
                const uint32_t key = unk ? addr : (0xffffffc0u | (uint32_t)lane);
                const uint32_t prev = (uint32_t)__builtin_amdgcn_mov_dpp((int32_t)key, 0x138, 0xf, 0xf, true);
                const uint64_t dups = ballot(prev == key) & bin_as_prev_mask;
                const uint64_t heads = ballot(unk) & ~dups;
                const bool head = unk & !((prev == key) & bin_as_prev);
                const uint32_t extra = (uint32_t)__builtin_ctzll(~((dups >> 1) >> lane));
                const int32_t below = (int32_t)lane_prefix(heads);
                if (head)
                    q[qn + below] =
                        make_uint2((uint32_t)ix | ((uint32_t)iy << 16), (uint32_t)iz | ebin | (extra << 24));
                qn = __builtin_amdgcn_readfirstlane(qn + __popcll(heads));
            }
            const bool mx = (tx <= ty) & (tx <= tz);
            const bool my = !mx & (ty <= tz);
            const bool mz = !mx & !my;
            const float tn = mx ? tx : (my ? ty : tz);
            ix += mx ? sx : 0;
            iy += my ? sy : 0;
            iz += mz ? sz : 0;
            // a lane that stops here (occupied, finished or outside) compares
            // +inf with the range: one comparison gives the mask, and the
            // ballot below takes it as it stands
            const float tn_go = st < kOccupied ? tn : __builtin_inff();
            const bool next_ok = tn_go < S.rv;
            alive = ballot(next_ok);
            addr = next_ok ? voxel_addr(ix, iy, iz, M) : M.outside;
            st = grid[addr];
            bx += mx ? dbx : 0.f;
            by += my ? dby : 0.f;
            bz += mz ? dbz : 0.f;
            tx = (bx - p.x) * fx;
            ty = (by - p.y) * fy;
            tz = (bz - p.z) * fz;
            t = tn;
        } while (alive && (!kMarginal || qn + 64 <= kQ));
        if (kMarginal) {
            drain_queue(q, qn, L.anc, na, S, L.bv, L.ts, L.lut_col, L.lut_row, Tr.dpan, L.bins + S.B, lane);
            qn = 0;
        }
    }
    } else {
    static_assert(kAhead == 2, "one or two voxels in flight");
    // Slot a and slot b hold the two voxels in flight (grid address, state,
    // entry parameter, coordinates packed as in a queue entry); they are
    // examined alternately, a first. `live`: the lane has not yet examined a
    // voxel that ends its ray, so a slot filled after that voxel is ignored.
    // The front (ix, iy, iz and the face parameters) is the newest voxel in
    // flight; refilling a slot takes the front one DDA step further. Once the
    // front has left the grid it takes at most one more step before the lane
    // examines the padding voxel it left through (which ends the ray) and
    // stops loading; coordinates -2 and n + 1 still give an address inside the
    // bricked grid (the coordinate bits are masked), whose byte is never
    // examined.
    bool live = has_ray;
    uint32_t addr_a = has_ray ? voxel_addr(ix, iy, iz, M) : M.outside;
    uint32_t st_a = grid[addr_a];
    float t_a = 0.f;
    uint32_t xy_a = (uint32_t)ix | ((uint32_t)iy << 16), z_a = (uint32_t)iz;
    uint32_t addr_b, st_b, xy_b, z_b;
    float t_b;
    auto advance = [&](uint32_t& addr_s, uint32_t& st_s, float& t_s, uint32_t& xy_s, uint32_t& z_s) {
        const bool mx = (tx <= ty) & (tx <= tz);
        const bool my = !mx & (ty <= tz);
        const bool mz = !mx & !my;
        const float tn = mx ? tx : (my ? ty : tz);
        ix += mx ? sx : 0;
        iy += my ? sy : 0;
        iz += mz ? sz : 0;
        const bool ok = live & (tn < S.rv);
        addr_s = ok ? voxel_addr(ix, iy, iz, M) : M.outside;
        st_s = grid[addr_s];
        bx += mx ? dbx : 0.f;
        by += my ? dby : 0.f;
        bz += mz ? dbz : 0.f;
        tx = (bx - p.x) * fx;
        ty = (by - p.y) * fy;
        tz = (bz - p.z) * fz;
        t_s = tn;
        xy_s = (uint32_t)ix | ((uint32_t)iy << 16);
        z_s = (uint32_t)iz;
    };
    auto examine = [&](uint32_t addr_s, uint32_t st_s, float t_s, uint32_t xy_s, uint32_t z_s) {
        const bool unk = live & (st_s == kUnknown);
        const bool occ = live & (st_s == kOccupied);
        h = occ ? t_s : h;
        if (!kMarginal) n_abs += unk ? 1u : 0u;
        if (kMarginal && ballot(unk) != 0) {
            n_abs += unk ? 1u : 0u;
            // the same run-merging append as with one voxel in flight
            const uint32_t key = unk ? addr_s : (0xffffffc0u | (uint32_t)lane);
            const uint32_t prev = (uint32_t)__builtin_amdgcn_mov_dpp((int32_t)key, 0x138, 0xf, 0xf, true);
            const uint64_t dups = ballot(prev == key) & bin_as_prev_mask;
            const uint64_t heads = ballot(unk) & ~dups;
            const bool head = unk & !((prev == key) & bin_as_prev);
            const uint32_t extra = (uint32_t)__builtin_ctzll(~((dups >> 1) >> lane));
            const int32_t below = (int32_t)lane_prefix(heads);
            if (head) q[qn + below] = make_uint2(xy_s, z_s | ebin | (extra << 24));
            qn = __builtin_amdgcn_readfirstlane(qn + __popcll(heads));
        }
        live = live & (st_s < kOccupied);
    };
    advance(addr_b, st_b, t_b, xy_b, z_b);
    uint64_t alive = ballot(live);
    while (alive) {
        do {
            examine(addr_a, st_a, t_a, xy_a, z_a);
            advance(addr_a, st_a, t_a, xy_a, z_a);
            examine(addr_b, st_b, t_b, xy_b, z_b);
            advance(addr_b, st_b, t_b, xy_b, z_b);
            alive = ballot(live);
        } while (alive && (!kMarginal || qn + 128 <= kQ));
        if (kMarginal) {
            drain_queue(q, qn, L.anc, na, S, L.bv, L.ts, L.lut_col, L.lut_row, Tr.dpan, L.bins + S.B, lane);
            qn = 0;
        }
    }
    }
    if (kMarginal && has_ray) Tr.dpan[(size_t)node * S.R + r] = h;
    if (n_abs) atomicAdd(&L.bins[bin], n_abs);
    __syncthreads();
    uint32_t* gb = Tr.bins + (size_t)node * 2 * S.B;
    for (int32_t i = tid; i < 2 * S.B; i += kTh) {
        const uint32_t v = L.bins[i];
        if (v) atomicAdd(&gb[i], v);
    }
}

template <bool kMarginal, int kAhead>
__global__ __launch_bounds__(kThreads) void k_trace(MapDev M, SensorDev S, TreeDev Tr,
                                                    const int32_t* __restrict__ nodes) {
    constexpr int kTh = kShapes[0].threads, kQ = kShapes[0].queue;
    static_assert(kTh == kThreads, "the per-tree path tiles rays by kThreads");
    extern __shared__ char smem[];
    const TraceLDS L = carve_lds<kTh, kQ>(smem, S);
    load_tables<kTh>(L, S);
    trace_tile<kMarginal, kTh, kQ, kAhead>(M, S, Tr, nodes[blockIdx.x / S.T], blockIdx.x % S.T, L);
}

// ---------------------------------------------------------------- window selection

// Window sums from a prefix sum over the bins taken circularly
// (P[i+1] = P[i] + bins[i mod B], S(k) = P[k+w] - P[k]), then the largest sum
// with the smallest k. Whole workgroup; returns (sum << 32) | (B - 1 - k) to
// every thread. Bins are read with atomic loads (they were accumulated with
// device-scope atomics, possibly by other workgroups).
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
    if (threadIdx.x == 0) {
        const int32_t k = S.B - 1 - (int32_t)(uint32_t)(best & 0xffffffffull);
        gain[node] = (uint32_t)(best >> 32);
        yaw[node] = k;
        if (marginal) Tr.c0[node] = S.c0_of_win[k];
    }
}

// ---------------------------------------------------------------- multi-tree, level by level

// Clears the bins of every tree in a batch. Grid: (blocks, n_trees).
__global__ void k_batch_zero(const BatchTree* __restrict__ trees, int32_t B2) {
    const BatchTree& T = trees[blockIdx.y];
    const size_t nb = (size_t)T.td.n * (size_t)B2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nb; i += (size_t)gridDim.x * blockDim.x)
        T.td.bins[i] = 0u;
}

// One depth level of all trees at once: work item = (tree, node) from
// `items` (tree << 32 | node), T workgroups per item.
template <int kTh, int kQ, int kAhead>
__global__ __launch_bounds__(kTh) void k_trace_multi(const BatchTree* __restrict__ trees,
                                                     const unsigned long long* __restrict__ items, SensorDev S) {
    extern __shared__ char smem[];
    const TraceLDS L = carve_lds<kTh, kQ>(smem, S);
    load_tables<kTh>(L, S);
    const unsigned long long it = items[blockIdx.x / S.T];
    const BatchTree& BT = trees[(uint32_t)(it >> 32)];
    SensorDev St = S;
    St.rv = BT.rv;
    St.rv2 = BT.rv2;
    const MapDev M = BT.map;     // copies: loaded once, not re-read through the descriptor
    const TreeDev Tr = BT.td;
    trace_tile<true, kTh, kQ, kAhead>(M, St, Tr, (int32_t)(uint32_t)it, blockIdx.x % S.T, L);
}

// Window selection for one depth level of all trees; writes each tree's
// outputs and, when asked, the node's depth buffer.
__global__ __launch_bounds__(kThreads) void k_finish_multi(const BatchTree* __restrict__ trees,
                                                           const unsigned long long* __restrict__ items, SensorDev S) {
    __shared__ uint32_t s_p[2 * kMaxBins + 1];
    __shared__ unsigned long long s_best[kThreads / 64];
    const unsigned long long it = items[blockIdx.x];
    const BatchTree& BT = trees[(uint32_t)(it >> 32)];
    const int32_t node = (int32_t)(uint32_t)it;
    const unsigned long long best = select_window(BT.td.bins + (size_t)node * 2 * S.B + S.B, S, s_p, s_best);
    const int32_t k = S.B - 1 - (int32_t)(uint32_t)(best & 0xffffffffull);
    const int32_t c0 = S.c0_of_win[k];
    if (threadIdx.x == 0) {
        BT.gain[node] = (uint32_t)(best >> 32);
        BT.yaw[node] = k;
        BT.td.c0[node] = c0;
    }
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

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

int shape_count() { return kNumShapes; }

void shape_of(int shape, int* threads, int* queue) {
    *threads = kShapes[shape].threads;
    *queue = kShapes[shape].queue;
}

size_t trace_lds_bytes(const SensorDev& sd, int shape, int32_t max_anc) {
    const size_t tables = sizeof(float2) * (2 * sd.W + 1) + sizeof(float) * (sd.H + 1) + sizeof(uint32_t) * 2 * sd.B +
                          sizeof(uint16_t) * (sd.n_lut_col + sd.n_lut_row);
    return ((tables + 15) & ~(size_t)15) + sizeof(uint2) * kShapes[shape].queue * (kShapes[shape].threads / 64) +
           sizeof(AncLDS) * (size_t)max_anc;
}

size_t lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64u * 1024u;
    return (size_t)v;
}

bool shape_fits(const SensorDev& sd, int shape, int32_t max_anc) {
    return trace_lds_bytes(sd, shape, max_anc) <= lds_limit();
}

int32_t tiles_per_node(const SensorDev& sd, int shape) {
    return (sd.R + kShapes[shape].threads - 1) / kShapes[shape].threads;
}

hipError_t launch_trace(const MapDev& m, const SensorDev& sd, const TreeDev& td, const int32_t* nodes,
                        int32_t n_nodes, bool marginal, int32_t max_anc, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    dim3 grid((unsigned)n_nodes * (unsigned)sd.T);
    size_t lds = trace_lds_bytes(sd, 0, marginal ? max_anc : 0);
    if (lds > lds_limit()) return hipErrorInvalidConfiguration;
    if (marginal && (int64_t)grid.x < kAheadWorkgroups)
        hipLaunchKernelGGL((k_trace<true, 2>), grid, dim3(kThreads), lds, s, m, sd, td, nodes);
    else if (marginal)
        hipLaunchKernelGGL((k_trace<true, 1>), grid, dim3(kThreads), lds, s, m, sd, td, nodes);
    else
        hipLaunchKernelGGL((k_trace<false, 1>), grid, dim3(kThreads), lds, s, m, sd, td, nodes);
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

template <int kTh, int kQ>
void launch_multi(const BatchTree* trees, const unsigned long long* items, int32_t n_items, const SensorDev& sd,
                  int32_t max_anc, hipStream_t s, hipEvent_t t0, hipEvent_t t1, int shape, bool ahead) {
    SensorDev st = sd;
    st.T = tiles_per_node(sd, shape);
    const dim3 grid((unsigned)n_items * (unsigned)st.T);
    const uint32_t lds = (uint32_t)trace_lds_bytes(sd, shape, max_anc);
    auto kern = ahead ? k_trace_multi<kTh, kQ, 2> : k_trace_multi<kTh, kQ, 1>;
    if (t0 && t1)
        hipExtLaunchKernelGGL(kern, grid, dim3(kTh), lds, s, t0, t1, 0u, trees, items, st);
    else
        hipLaunchKernelGGL(kern, grid, dim3(kTh), lds, s, trees, items, st);
}

template <int I>
void launch_multi_shape(int shape, const BatchTree* trees, const unsigned long long* items, int32_t n_items,
                        const SensorDev& sd, int32_t max_anc, hipStream_t s, hipEvent_t t0, hipEvent_t t1,
                        bool ahead) {
    if constexpr (I < kNumShapes) {
        if (shape == I)
            launch_multi<kShapes[I].threads, kShapes[I].queue>(trees, items, n_items, sd, max_anc, s, t0, t1, I,
                                                               ahead);
        else
            launch_multi_shape<I + 1>(shape, trees, items, n_items, sd, max_anc, s, t0, t1, ahead);
    }
}

}  // namespace

hipError_t launch_batch_level(const BatchTree* trees, const unsigned long long* items, int32_t n_items,
                              const SensorDev& sd, int32_t max_anc, hipStream_t s, int shape, hipEvent_t t0,
                              hipEvent_t t1, bool ahead) {
    if (n_items <= 0) return hipSuccess;
    if (shape < 0 || shape >= kNumShapes || max_anc < 0 || max_anc > kMaxAnc) return hipErrorInvalidValue;
    if (!shape_fits(sd, shape, max_anc)) return hipErrorInvalidConfiguration;
    launch_multi_shape<0>(shape, trees, items, n_items, sd, max_anc, s, t0, t1, ahead);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish_multi, dim3((unsigned)n_items), dim3(kThreads), 0, s, trees, items, sd);
    return hipGetLastError();
}

}  // namespace mgk
