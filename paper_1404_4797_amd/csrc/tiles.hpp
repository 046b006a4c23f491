// Slot tiles for slot-parallel kernels over a CSR: each workgroup takes
// kTile consecutive adjacency slots and recovers the source row of every
// slot in LDS (row starts scattered into the tile, then a max-scan), so rows
// of any length are split evenly over the grid without a per-slot search.
#pragma once

#include "common.hpp"

namespace sclap {
namespace {

constexpr int kTileThreads = 256;
constexpr int kTilePer = 8;
constexpr int kTile = kTileThreads * kTilePer;

__device__ int32_t upper_node(const int64_t* __restrict__ xadj, int32_t n, int64_t slot) {
    // largest u in [0, n) with xadj[u] <= slot
    int32_t lo = 0, hi = n;  // invariant: xadj[lo] <= slot, answer in [lo, hi)
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (xadj[mid] <= slot) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Fills owner[0 .. i1-i0) with the source node of each slot of [i0, i1).
__device__ void tile_owners(const int64_t* __restrict__ xadj, int32_t n, int64_t i0, int64_t i1, int32_t* owner) {
    __shared__ int32_t s_u[2];
    __shared__ int32_t s_carry[kTileThreads / kWave];
    const int tid = threadIdx.x;
    for (int j = tid; j < kTile; j += kTileThreads) owner[j] = -1;
    if (tid == 0) s_u[0] = upper_node(xadj, n, i0);
    if (tid == 1) s_u[1] = upper_node(xadj, n, i1 - 1);
    __syncthreads();
    const int32_t u0 = s_u[0], u1 = s_u[1];
    if (tid == 0) atomicMax(&owner[0], u0);
    for (int64_t u = static_cast<int64_t>(u0) + 1 + tid; u <= u1; u += kTileThreads) {
        const int64_t st = xadj[u];
        if (st >= i0 && st < i1) atomicMax(&owner[st - i0], static_cast<int32_t>(u));
    }
    __syncthreads();
    // inclusive max-scan over the tile: 8 consecutive entries per thread
    int32_t loc[kTilePer];
    int32_t m = -1;
#pragma unroll
    for (int j = 0; j < kTilePer; ++j) {
        loc[j] = owner[tid * kTilePer + j];
        m = loc[j] > m ? loc[j] : m;
    }
    int32_t incl = m;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= o) incl = t > incl ? t : incl;
    }
    if (lane_id() == kWave - 1) s_carry[tid / kWave] = incl;
    __syncthreads();
    int32_t run = __shfl_up(incl, 1, 64);
    if (lane_id() == 0) run = -1;
    for (int w = 0; w < tid / kWave; ++w) run = s_carry[w] > run ? s_carry[w] : run;
#pragma unroll
    for (int j = 0; j < kTilePer; ++j) {
        run = loc[j] > run ? loc[j] : run;
        owner[tid * kTilePer + j] = run;
    }
    __syncthreads();
}

}  // namespace
}  // namespace sclap
