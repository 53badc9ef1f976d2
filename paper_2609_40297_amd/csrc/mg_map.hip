// Map contents on the device: conversion of a truncated signed distance field
// (the volumetric map the paper's planners keep; Sec. IV turns it into a
// contiguous grid on the GPU) into the bricked occupancy grid, and in-place
// updates between replans (a box of the TSDF, or a list of voxels).
//
// Occupancy of a voxel from its TSDF distance d (metres) and weight w:
// unknown unless w >= w_min (never observed, or too little), occupied when
// d <= surface (inside the surface or within the band), free otherwise. Any
// comparison with a NaN is false, so a NaN weight is unknown and a NaN
// distance is free.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>

#include "mg_internal.h"

namespace mgk {

__device__ __forceinline__ uint8_t tsdf_state(float d, float w, float surface, float min_weight) {
    return !(w >= min_weight) ? (uint8_t)kUnknown : (d <= surface ? (uint8_t)kOccupied : (uint8_t)kFree);
}

// The summaries of the run's bricks assembled in LDS (the work of
// k_brick_flags, done here so that a whole-grid conversion needs no second
// pass): one wave per brick, each lane 8 of its 512 bytes; the unknown and free
// voxels get their block levels (mark_brick_row), and brick_unk records
// whether the brick holds no, some or only unknown voxels (bricks wholly in the
// padding have no entry). Whole workgroup of 256.
__device__ __forceinline__ void mark_run(uint8_t* tile, int32_t tb, int32_t bx0, int32_t by, int32_t bz,
                                         const MapDev& m) {
    const int32_t lane = (int32_t)threadIdx.x & 63, wave = (int32_t)threadIdx.x >> 6;
    for (int32_t k = wave; k < tb; k += 4) {
        uint64_t* p = reinterpret_cast<uint64_t*>(tile + k * 512) + lane;
        bool any_unk, all_unk, all_free;
        *p = mark_brick_row(*p, (uint32_t)lane, &any_unk, &all_unk, &all_free);
        const int32_t bx = bx0 + k;
        if (lane == 0 && (uint32_t)bx < m.mbx && (uint32_t)by < m.mby && (uint32_t)bz < m.mbz)
            m.brick_unk[(uint32_t)bx + m.mbx * ((uint32_t)by + m.mby * (uint32_t)bz)] =
                brick_summary(any_unk, all_unk, all_free);
    }
}

// Whole grid: one workgroup per run of up to 32 bricks along x at one (by, bz),
// over the bricks that hold grid voxels (bricks wholly in the padding keep
// kOutside from the map's creation). Each of the 64 (y, z) rows of the run is
// read coalesced along x, the states are assembled in LDS in brick order, the
// bricks' summaries are taken (mark_run), and the run's bricks (contiguous in
// memory) are written out in 16-byte stores. Padding voxels inside these
// bricks get kOutside.
constexpr int kTileBricks = 32;

__global__ __launch_bounds__(256) void k_tsdf_grid(const float* __restrict__ dist, const float* __restrict__ weight,
                                                   uint8_t* __restrict__ bricks, MapDev m, float surface,
                                                   float min_weight) {
    __shared__ __align__(16) uint8_t tile[kTileBricks * 512];
    const int32_t tb = m.nbx < kTileBricks ? m.nbx : kTileBricks;   // nbx is a power of two
    const int32_t bx0 = (int32_t)blockIdx.x * tb, by = (int32_t)blockIdx.y, bz = (int32_t)blockIdx.z;
    const int32_t tid = (int32_t)threadIdx.x;
    const int32_t x = bx0 * 8 + tid;
    const bool lane_in = tid < tb * 8;
    for (int32_t r = 0; r < 64; ++r) {
        const int32_t yy = r & 7, zz = r >> 3;
        const int32_t y = by * 8 + yy, z = bz * 8 + zz;
        if (lane_in) {
            uint8_t v = kOutside;
            if (x < m.nx && y < m.ny && z < m.nz) {
                const size_t i = (size_t)x + (size_t)m.nx * ((size_t)y + (size_t)m.ny * (size_t)z);
                v = tsdf_state(dist[i], weight[i], surface, min_weight);
            }
            tile[(tid >> 3) * 512 + (tid & 7) + (yy << 3) + (zz << 6)] = v;
        }
    }
    __syncthreads();
    mark_run(tile, tb, bx0, by, bz, m);
    __syncthreads();
    const size_t base = ((size_t)bx0 + (size_t)m.nbx * ((size_t)by + (size_t)m.nby * (size_t)bz)) * 512u;
    uint4* dst = (uint4*)(bricks + base);
    const uint4* src = (const uint4*)tile;
    for (int32_t o = tid; o < tb * 32; o += 256) dst[o] = src[o];
}

// The same with 16-byte loads: four consecutive voxels along x per thread
// (needs nx % 4 == 0, so every row starts 16-byte aligned); the 256 threads
// cover four rows of the run at a time.
__global__ __launch_bounds__(256) void k_tsdf_grid4(const float* __restrict__ dist, const float* __restrict__ weight,
                                                    uint8_t* __restrict__ bricks, MapDev m, float surface,
                                                    float min_weight) {
    __shared__ __align__(16) uint8_t tile[kTileBricks * 512];
    const int32_t tb = m.nbx < kTileBricks ? m.nbx : kTileBricks;
    const int32_t bx0 = (int32_t)blockIdx.x * tb, by = (int32_t)blockIdx.y, bz = (int32_t)blockIdx.z;
    const int32_t tid = (int32_t)threadIdx.x;
    const int32_t quad = tid & 63, sub = tid >> 6;          // 4 voxels along x, one of 4 rows
    const int32_t x = bx0 * 8 + quad * 4;
    const bool lane_in = quad < tb * 2;
    for (int32_t r0 = 0; r0 < 64; r0 += 4) {
        const int32_t r = r0 + sub;
        const int32_t yy = r & 7, zz = r >> 3;
        const int32_t y = by * 8 + yy, z = bz * 8 + zz;
        if (lane_in) {
            uint32_t v = kOutside * 0x01010101u;
            if (y < m.ny && z < m.nz && x < m.nx) {           // x < nx and nx % 4 == 0: all four inside
                const size_t i = (size_t)x + (size_t)m.nx * ((size_t)y + (size_t)m.ny * (size_t)z);
                const float4 d = *(const float4*)(dist + i);
                const float4 w = *(const float4*)(weight + i);
                v = (uint32_t)tsdf_state(d.x, w.x, surface, min_weight) |
                    ((uint32_t)tsdf_state(d.y, w.y, surface, min_weight) << 8) |
                    ((uint32_t)tsdf_state(d.z, w.z, surface, min_weight) << 16) |
                    ((uint32_t)tsdf_state(d.w, w.w, surface, min_weight) << 24);
            }
            *(uint32_t*)&tile[(quad >> 1) * 512 + (quad & 1) * 4 + (yy << 3) + (zz << 6)] = v;
        }
    }
    __syncthreads();
    mark_run(tile, tb, bx0, by, bz, m);
    __syncthreads();
    const size_t base = ((size_t)bx0 + (size_t)m.nbx * ((size_t)by + (size_t)m.nby * (size_t)bz)) * 512u;
    uint4* dst = (uint4*)(bricks + base);
    const uint4* src = (const uint4*)tile;
    for (int32_t o = tid; o < tb * 32; o += 256) dst[o] = src[o];
}

// A box of the grid (lo, size), its TSDF given box-local and x-fastest.
__global__ void k_tsdf_box(const float* __restrict__ dist, const float* __restrict__ weight,
                           uint8_t* __restrict__ bricks, MapDev m, int32_t lx, int32_t ly, int32_t lz, int32_t sx,
                           int32_t sy, size_t total, float surface, float min_weight) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t x = lx + (int32_t)(i % (size_t)sx);
        const int32_t y = ly + (int32_t)((i / (size_t)sx) % (size_t)sy);
        const int32_t z = lz + (int32_t)(i / ((size_t)sx * (size_t)sy));
        bricks[voxel_addr(x, y, z, m)] = tsdf_state(dist[i], weight[i], surface, min_weight);
    }
}

// New states for listed voxels (linear ids x + nx (y + ny z)); an id outside
// the grid or a state above 2 is skipped and counted in *rejected.
__global__ void k_map_scatter(const uint32_t* __restrict__ ids, const uint8_t* __restrict__ states, uint32_t count,
                              uint8_t* __restrict__ bricks, MapDev m, uint32_t* __restrict__ rejected) {
    const uint32_t nxy = (uint32_t)m.nx * (uint32_t)m.ny;
    const uint64_t nvox = (uint64_t)nxy * (uint64_t)m.nz;     // below 2^32 (map limit)
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
        const uint32_t id = ids[k];
        const uint8_t s = states[k];
        if (id >= nvox || s > kOccupied) {
            if (rejected) atomicAdd(rejected, 1u);
            continue;
        }
        const int32_t x = (int32_t)(id % (uint32_t)m.nx), y = (int32_t)((id / (uint32_t)m.nx) % (uint32_t)m.ny);
        const int32_t z = (int32_t)(id / nxy);
        bricks[voxel_addr(x, y, z, m)] = s;
    }
}

// Dense x-fastest copy of the grid's states.
__global__ void k_unbrick(const uint8_t* __restrict__ bricks, MapDev m, uint8_t* __restrict__ dense, uint32_t keep) {
    const size_t nxy = (size_t)m.nx * (size_t)m.ny;
    const size_t nvox = nxy * (size_t)m.nz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)(i % (size_t)m.nx), y = (int32_t)((i / (size_t)m.nx) % (size_t)m.ny);
        const int32_t z = (int32_t)(i / nxy);
        dense[i] = bricks[voxel_addr(x, y, z, m)] & keep;   // (the state, or the state with its block mark)
    }
}

namespace {
unsigned blocks_for(size_t n) {
    size_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}
}  // namespace

// Every byte of the padded grid set to kOutside (a new map, before conversion).
__global__ void k_fill_outside(uint4* __restrict__ p, size_t n16) {
    const uint32_t o = kOutside * 0x01010101u;
    const uint4 v = make_uint4(o, o, o, o);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_outside(const MapDev& m, hipStream_t s) {
    const size_t n16 = (size_t)m.nbx * m.nby * m.nbz * 32u;
    hipLaunchKernelGGL(k_fill_outside, dim3(blocks_for(n16)), dim3(256), 0, s, (uint4*)m.bricks, n16);
    return hipGetLastError();
}

hipError_t launch_tsdf_grid(const float* dist, const float* weight, const MapDev& m, float surface, float min_weight,
                            hipStream_t s) {
    const int32_t tb = m.nbx < kTileBricks ? m.nbx : kTileBricks;
    const int32_t ux = (m.nx + 7) / 8, uy = (m.ny + 7) / 8, uz = (m.nz + 7) / 8;   // bricks holding grid voxels
    const dim3 grid((unsigned)((ux + tb - 1) / tb), (unsigned)uy, (unsigned)uz);
    const bool aligned = m.nx % 4 == 0 && ((uintptr_t)dist % 16) == 0 && ((uintptr_t)weight % 16) == 0;
    if (aligned)
        hipLaunchKernelGGL(k_tsdf_grid4, grid, dim3(256), 0, s, dist, weight, (uint8_t*)m.bricks, m, surface,
                           min_weight);
    else
        hipLaunchKernelGGL(k_tsdf_grid, grid, dim3(256), 0, s, dist, weight, (uint8_t*)m.bricks, m, surface,
                           min_weight);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_blocks16(m, s) : e;            // (the bricks' summaries are taken above)
}

hipError_t launch_tsdf_box(const float* dist, const float* weight, const MapDev& m, const int32_t lo[3],
                           const int32_t size[3], float surface, float min_weight, hipStream_t s) {
    const size_t total = (size_t)size[0] * (size_t)size[1] * (size_t)size[2];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tsdf_box, dim3(blocks_for(total)), dim3(256), 0, s, dist, weight, (uint8_t*)m.bricks, m,
                       lo[0], lo[1], lo[2], size[0], size[1], total, surface, min_weight);
    return hipGetLastError();
}

hipError_t launch_map_scatter(const uint32_t* ids, const uint8_t* states, uint32_t count, const MapDev& m,
                              uint32_t* rejected, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_scatter, dim3(blocks_for(count)), dim3(256), 0, s, ids, states, count,
                       (uint8_t*)m.bricks, m, rejected);
    return hipGetLastError();
}

hipError_t launch_unbrick(const MapDev& m, uint8_t* dense, hipStream_t s, bool marks) {
    const size_t nvox = (size_t)m.nx * m.ny * m.nz;
    hipLaunchKernelGGL(k_unbrick, dim3(blocks_for(nvox)), dim3(256), 0, s, m.bricks, m, dense, marks ? 0xffu : 3u);
    return hipGetLastError();
}

}  // namespace mgk
