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

// Source row of the first slot of every tile, and at [ntiles] the row of the
// last slot: tile t then holds the row starts of rows trow[t]+1 .. trow[t+1]
// (those that start inside it).  One search per tile, all in parallel, once
// per graph, instead of two dependent searches at the start of every tile.
__global__ void tile_rows_kernel(const int64_t* __restrict__ xadj, int32_t n, int64_t S, int64_t ntiles,
                                 int32_t* __restrict__ trow) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t > ntiles) return;
    const int64_t slot = t * kTile < S ? t * kTile : S - 1;
    trow[t] = upper_node(xadj, n, slot);
}

// Tiles of the S slots over the rows [0, n) of xadj (offsets monotone; no
// tiles when S = 0).
struct TileRows {
    int64_t ntiles = 0;
    DBuf<int32_t> trow;
    TileRows(const int64_t* xadj, int32_t n, int64_t S, hipStream_t s) {
        ntiles = S > 0 ? (S + kTile - 1) / kTile : 0;
        trow.alloc(static_cast<size_t>(ntiles) + 1, s);
        if (ntiles == 0) return;
        tile_rows_kernel<<<grid_for(ntiles + 1, 256), 256, 0, s>>>(xadj, n, S, ntiles, trow.get());
        LAUNCHCHK();
    }
};

// Fills owner[0 .. i1-i0) with the source node of each slot of tile `tile`
// ([i0, i1)), from the tile's first row trow[tile].
__device__ void tile_owners(const int64_t* __restrict__ xadj, const int32_t* __restrict__ trow, int64_t tile,
                            int64_t i0, int64_t i1, int32_t* owner) {
    __shared__ int32_t s_carry[kTileThreads / kWave];
    const int tid = threadIdx.x;
    for (int j = tid; j < kTile; j += kTileThreads) owner[j] = -1;
    const int32_t u0 = trow[tile], u1 = trow[tile + 1];
    __syncthreads();
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
