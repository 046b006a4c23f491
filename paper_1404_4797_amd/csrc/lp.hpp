// Size-constrained label propagation (SCLaP) on gfx950: one level, one phase.
#pragma once

#include "common.hpp"
#include "primitives.hpp"

namespace sclap {

// kInitial: label propagation of the device initial partitioner; refinement
// rules, its own hash phase.
enum Phase : int32_t { kCluster = 0, kRefine = 1, kInitial = 2 };

struct DevGraph {
    int32_t n = 0;
    int64_t S = 0;
    const int64_t* xadj = nullptr;
    const int32_t* adj = nullptr;
    const int32_t* ew = nullptr;  // null => unit edge weights
    const int32_t* vw = nullptr;  // null => unit node weights
};

struct LPTuning {
    int32_t lane_max = 16;    // <= 16
    int32_t wave_max = 256;   // <= 256
    int32_t block_max = 8192; // <= 8192
    int32_t hub_part_limit = 4096;  // <= 4096; larger hub partitions use the HBM table
    int32_t hub_region_cap = 0;     // 0: about twice a partition's expected share
    int32_t select_small_max = 4096;  // larger overflow segments: multi-workgroup selection
    int32_t select_launches = 0;      // multi-workgroup selection launches per sub-round (0: default)
    int32_t skip_quiet = 0;           // 1: skip nodes whose decision cannot have changed; -1: never; 0: caller's choice
    int32_t capture = 0;              // 1: record each call's rounds in a HIP graph; else launch directly
    int32_t fuse = 0;                 // >= 0: the small buckets of a small colour in one launch; -1: one launch each
    int32_t block_table = 10240;      // LDS table entries of the longest-row workgroup bucket: 10240 or 16384
};

// Several disjoint graphs in one CSR (node ranges per graph, no edge between
// ranges).  Every hash and order uses graph-local ids and the graph's own
// seed and bound, so each graph's result equals its result alone.
struct MultiGraph {
    int32_t G = 0;
    const int32_t* gid = nullptr;     // [n] graph of each node
    const int32_t* lgid = nullptr;    // [nw] graph of each label
    const int32_t* nbase = nullptr;   // [G] first node of each graph
    const int32_t* lbase = nullptr;   // [G] first label of each graph
    const int64_t* bound = nullptr;   // [G] bound of each graph's labels
    const uint64_t* seed = nullptr;   // [G]
    const uint8_t* active = nullptr;  // [G] nodes of inactive graphs never move
    int32_t max_labels = 0;           // refinement: the most blocks of any graph (0: unknown)
};

struct LPResult {
    int32_t rounds_run = 0;
    int64_t visits = 0;
    int64_t moves = 0;
};

// Runs SCLaP rounds for one (level, phase) in place on `label` (n entries,
// values in [0, nw)) and `w` (nw entries, w[x] = total node weight of label
// x).  `color_override` is a device array or null.
LPResult run_lp(const DevGraph& g, int32_t phase, int32_t level, uint64_t seed, int32_t nsub, int32_t rounds,
                int64_t bound, int32_t* label, int32_t* w, int32_t nw, const int32_t* color_override,
                const LPTuning& tune, hipStream_t s, const MultiGraph* mg = nullptr);

// w[x] = sum of c(v) over label(v) = x, for x in [0, nw).
void label_weights(const DevGraph& g, const int32_t* label, int32_t* w, int32_t nw, hipStream_t s);

}  // namespace sclap
