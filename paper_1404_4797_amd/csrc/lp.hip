// Size-constrained label propagation (SCLaP) kernels for gfx950.
//
// Follows Section 3.1 (Label Propagation with Size Constraints) of
// Meyerhenke, Sanders, Schulz (2014): a visited node moves to the eligible
// neighbouring label (cluster or block) of strongest connection, eligible
// meaning the label stays within the bound after the move; during refinement
// a node of an overloaded block moves to the best eligible block regardless
// of its own.  The paper's asynchronous visiting is realised as hash-coloured
// sub-rounds: every node of colour s is evaluated against the state at the
// start of sub-round s, then each target admits its candidates in
// (gain desc, node asc) order while it stays within the bound, then the moves
// are applied.  All arithmetic is integer, so the result does not depend on
// thread order.
//
// Node evaluation is bucketed by degree:
//   lane   one lane per node, neighbour labels kept in registers (deg <= 16)
//   wave   one wave64 per node, open-addressing table in LDS (deg <= 256)
//   block  one workgroup per node with an LDS table of 16, 64 or 128 KB
//          (deg <= 1024, 4096, 8192)
//   hub    the row is cut into 8192-slot chunks; each workgroup sums its
//          chunk in an LDS table and appends the chunk's distinct labels to
//          the hub's entry list; one workgroup per hub then sums that list in
//          LDS, or, when it is longer than 8192 entries, through an
//          open-addressing table in HBM that a further pass scans
// The per-node connection table maps a neighbour label to the summed weight
// of the edges to it (Section 4.1 uses hashing with linear probing for this).
//
// Evaluation writes each node's result at the node's position in the
// sub-round's schedule, so no counter is shared.  Per-label sums use
// LDS-private histograms when the label space is small (refinement: k blocks).
#include <climits>
#include <cstdio>
#include <cstdlib>

#include "lp.hpp"
#include "profile.hpp"

namespace sclap {

namespace {

constexpr int kNB = 7;  // buckets: lane4, lane16, wave, block (3 table sizes), hub
constexpr int kHubBucket = kNB - 1;
constexpr int kLaneSmall = 4;
constexpr int kLaneMax = 16;
constexpr int kWaveTable = 512;
constexpr int kWaveMaxDeg = kWaveTable / 2;
constexpr int kBlockTable = 16384;
constexpr int kBlockMaxDeg = kBlockTable / 2;
constexpr int kBlock1Max = 1024;  // 256 threads, 16 KB table
constexpr int kBlock2Max = 4096;  // 512 threads, 64 KB table
constexpr int kHubChunk = kBlockMaxDeg;  // slots per hub workgroup (table load <= 1/2)
constexpr int kHubTChunk = 4096;         // HBM table entries per scan workgroup
constexpr int kSmallLabels = 4096;       // LDS-private histograms up to this many labels
constexpr int kMaxBlocks = 1024;         // grid cap of the grid-stride candidate kernels

struct Counters {
    uint32_t ncand;
    uint32_t nslow;
    int32_t gmin;
    int32_t gmax;
    uint32_t bad_color;
    uint32_t pad[3];
};

struct EvalArgs {
    const int64_t* xadj;
    const int32_t* adj;
    const int32_t* ew;
    const int32_t* vw;
    const int32_t* label;
    const int32_t* w;
    int64_t bound;
    uint64_t tp;  // H(seed, 2, level, phase, round)
    int32_t refine;
    const int32_t* nodes;  // schedule entries of this launch
    int32_t count;
    int32_t* ct;  // per entry: target label or -1
    int32_t* cg;  // per entry: gain
};

// ------------------------------------------------------- selection helpers

// Best eligible label seen so far under the total order
// (conn desc, tie(x) asc, x asc); tie(x) = mix(tp ^ x) is computed lazily,
// only when two labels have equal connection.
struct Best {
    int32_t conn;
    int32_t x;
    uint64_t tie;
    bool tv;
};

__device__ __forceinline__ void best_init(Best& b) {
    b.conn = -1;
    b.x = -1;
    b.tie = 0;
    b.tv = false;
}

__device__ __forceinline__ uint64_t tie_of(uint64_t tp, int32_t x) {
    return mix64(tp ^ static_cast<uint64_t>(static_cast<uint32_t>(x)));
}

__device__ __forceinline__ void best_consider(Best& b, int32_t x, int32_t conn, uint64_t tp) {
    if (b.x < 0 || conn > b.conn) {
        b.conn = conn;
        b.x = x;
        b.tv = false;
        return;
    }
    if (conn < b.conn) return;
    const uint64_t tx = tie_of(tp, x);
    if (!b.tv) {
        b.tie = tie_of(tp, b.x);
        b.tv = true;
    }
    if (tx < b.tie || (tx == b.tie && x < b.x)) {
        b.x = x;
        b.tie = tx;
    }
}

__device__ __forceinline__ uint64_t best_tie(const Best& b, uint64_t tp) { return b.tv ? b.tie : tie_of(tp, b.x); }

// Wave-wide argmax; every lane gets the winning (x, conn) or x = -1.
__device__ __forceinline__ void wave_argmax(const Best& b, uint64_t tp, int32_t& out_x, int32_t& out_conn) {
    const int32_t bc = b.x >= 0 ? b.conn : -1;
    const int32_t maxc = wave_max(bc);
    if (maxc < 0) {
        out_x = -1;
        out_conn = -1;
        return;
    }
    const bool top = b.x >= 0 && bc == maxc;
    const uint64_t tk = top ? best_tie(b, tp) : ~0ULL;
    const uint64_t mt = wave_min_u64(tk);
    const int32_t xx = (top && tk == mt) ? b.x : INT_MAX;
    out_x = wave_min(xx);
    out_conn = maxc;
}

// Combines one candidate per wave (written to LDS by each wave's lane 0).
__device__ __forceinline__ void combine_into(int32_t& bc, uint64_t& bt, int32_t& bx, int32_t c2, uint64_t t2,
                                             int32_t x2) {
    if (x2 < 0) return;
    if (bx < 0 || c2 > bc || (c2 == bc && (t2 < bt || (t2 == bt && x2 < bx)))) {
        bc = c2;
        bt = t2;
        bx = x2;
    }
}

__device__ __forceinline__ bool eligible(const EvalArgs& A, int32_t x, int32_t c) {
    return static_cast<int64_t>(A.w[x]) + c <= A.bound;
}

// Decision for a node given its best eligible label (x, conn) and the
// connection to its own label: a move needs a positive gain, or an overloaded
// own block during refinement.
__device__ __forceinline__ void store_result(const EvalArgs& A, int32_t i, int32_t x, int32_t conn, int32_t own,
                                             bool over) {
    int32_t t = -1, gain = 0;
    if (x >= 0) {
        gain = conn - own;
        if (over || gain > 0) t = x;
    }
    A.ct[i] = t;
    A.cg[i] = gain;
}

__device__ __forceinline__ uint32_t table_size_for(int32_t d, uint32_t lo, uint32_t hi) {
    uint32_t t = lo;
    while (t < 2u * static_cast<uint32_t>(d) && t < hi) t <<= 1;
    return t;
}

// Linear-probing insert of (x, wt) into a table of 2^k entries (key -1 =
// empty), in LDS or HBM.  The table always has a free entry for a new key.
__device__ __forceinline__ void table_add(int32_t* keys, int32_t* vals, uint32_t mask, int32_t x, int32_t wt) {
    uint32_t h = slot_hash(static_cast<uint32_t>(x)) & mask;
    while (true) {
        const int32_t prev = atomicCAS(&keys[h], -1, x);
        if (prev == -1 || prev == x) {
            atomicAdd(&vals[h], wt);
            return;
        }
        h = (h + 1) & mask;
    }
}

// Adds the slots [b, b+d) of a row to a table; each thread keeps U gathers
// in flight before inserting.
template <int NT, int U>
__device__ __forceinline__ void insert_slots(const EvalArgs& A, int64_t b, int32_t d, int32_t* keys, int32_t* vals,
                                             uint32_t mask, int tid) {
    for (int32_t j0 = tid; j0 < d; j0 += NT * U) {
        int32_t x[U], wt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t j = j0 + u * NT;
            x[u] = j < d ? A.adj[b + j] : 0;
            wt[u] = j < d ? (A.ew ? A.ew[b + j] : 1) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t j = j0 + u * NT;
            x[u] = j < d ? A.label[x[u]] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (x[u] >= 0) table_add(keys, vals, mask, x[u], wt[u]);
    }
}

// ------------------------------------------------------------ lane bucket

template <int MAXD>
__global__ void __launch_bounds__(256) eval_lane_kernel(EvalArgs A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= A.count) return;
    const int32_t v = A.nodes[i];
    const int64_t b = A.xadj[v];
    const int d = static_cast<int>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    int32_t lab[MAXD], wt[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        if (j < d) {
            lab[j] = A.label[A.adj[b + j]];
            wt[j] = A.ew ? A.ew[b + j] : 1;
        } else {
            lab[j] = -1;
            wt[j] = 0;
        }
    }
    int32_t own = 0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j) own += (lab[j] == a) ? wt[j] : 0;
    const bool over = A.refine && A.w[a] > A.bound;
    Best best;
    best_init(best);
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        const int32_t x = lab[j];
        bool skip = (x < 0) || (x == a);
#pragma unroll
        for (int j2 = 0; j2 < j; ++j2) skip |= (lab[j2] == x);
        if (skip) continue;
        int32_t conn = 0;
#pragma unroll
        for (int j2 = j; j2 < MAXD; ++j2) conn += (lab[j2] == x) ? wt[j2] : 0;
        if (!over && conn <= own) continue;  // cannot give a positive gain
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c)) continue;
        best_consider(best, x, conn, A.tp);
    }
    store_result(A, i, best.x, best.conn, own, over);
}

// ------------------------------------------------------------ wave bucket

__global__ void __launch_bounds__(256) eval_wave_kernel(EvalArgs A) {
    __shared__ int32_t tkeys[4][kWaveTable];
    __shared__ int32_t tvals[4][kWaveTable];
    const int wid = threadIdx.x >> 6;
    const int lane = lane_id();
    const int node_i = blockIdx.x * 4 + wid;
    if (node_i >= A.count) return;
    int32_t* keys = tkeys[wid];
    int32_t* vals = tvals[wid];
    const int32_t v = A.nodes[node_i];
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    const uint32_t tsz = table_size_for(d, 64, kWaveTable);
    const uint32_t mask = tsz - 1;
    for (uint32_t j = lane; j < tsz; j += 64) {
        keys[j] = -1;
        vals[j] = 0;
    }
    wave_sync();
    insert_slots<64, 4>(A, b, d, keys, vals, mask, lane);
    wave_sync();
    int32_t ownp = 0;
    for (uint32_t j = lane; j < tsz; j += 64)
        if (keys[j] == a) ownp = vals[j];
    const int32_t own = wave_max(ownp);
    const bool over = A.refine && A.w[a] > A.bound;
    Best best;
    best_init(best);
    for (uint32_t j = lane; j < tsz; j += 64) {
        const int32_t x = keys[j];
        if (x < 0 || x == a) continue;
        const int32_t conn = vals[j];
        if (!over && conn <= own) continue;
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c)) continue;
        best_consider(best, x, conn, A.tp);
    }
    int32_t bx, bconn;
    wave_argmax(best, A.tp, bx, bconn);
    if (lane == 0) store_result(A, node_i, bx, bconn, own, over);
}

// ----------------------------------------------------------- block bucket

template <int NT, int TABLE>
__global__ void __launch_bounds__(NT) eval_block_kernel(EvalArgs A) {
    __shared__ int32_t keys[TABLE];
    __shared__ int32_t vals[TABLE];
    __shared__ int32_t s_own;
    __shared__ int32_t s_conn[NT / 64];
    __shared__ int32_t s_x[NT / 64];
    __shared__ uint64_t s_tie[NT / 64];
    const int tid = threadIdx.x;
    const int wid = tid >> 6;
    const int lane = lane_id();
    const int32_t v = A.nodes[blockIdx.x];
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    const uint32_t tsz = table_size_for(d, 512, TABLE);
    const uint32_t mask = tsz - 1;
    for (uint32_t j = tid; j < tsz; j += NT) {
        keys[j] = -1;
        vals[j] = 0;
    }
    if (tid == 0) s_own = 0;
    __syncthreads();
    insert_slots<NT, 4>(A, b, d, keys, vals, mask, tid);
    __syncthreads();
    for (uint32_t j = tid; j < tsz; j += NT)
        if (keys[j] == a) s_own = vals[j];
    __syncthreads();
    const int32_t own = s_own;
    const bool over = A.refine && A.w[a] > A.bound;
    Best best;
    best_init(best);
    for (uint32_t j = tid; j < tsz; j += NT) {
        const int32_t x = keys[j];
        if (x < 0 || x == a) continue;
        const int32_t conn = vals[j];
        if (!over && conn <= own) continue;
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c)) continue;
        best_consider(best, x, conn, A.tp);
    }
    int32_t bx, bconn;
    wave_argmax(best, A.tp, bx, bconn);
    if (lane == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(A.tp, bx) : ~0ULL;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < NT / 64; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        store_result(A, blockIdx.x, fx, fc, own, over);
    }
}

// ------------------------------------------------------------- hub bucket

struct HubArgs {
    const int32_t* hub_nodes;    // [H]
    const int32_t* hub_plog;     // [H] log2 of the hub's partition count
    const int32_t* hub_pbase;    // [H+1] first partition of each hub
    const int32_t* hub_cap;      // [H] entries per partition region
    const int32_t* hub_tfirst;   // [H+1] first HBM table chunk of each hub
    const int32_t* chunk_hub;    // [nchunks]
    const int32_t* part_hub;     // [nparts]
    const int32_t* tchunk_hub;   // [ntchunks]
    const int64_t* hub_rbase;    // [H] first region entry of the hub
    const int64_t* hub_obase;    // [H] first overflow entry of the hub
    const int64_t* hub_toff;     // [H] HBM table offset
    const int64_t* chunk_begin;  // [nchunks] first slot of the chunk
    const int64_t* tchunk_begin; // [ntchunks] first table entry (absolute)
    const uint32_t* hub_tmask;   // [H] HBM table size - 1
    int32_t* rcount;   // [nparts] entries reserved per partition    } zeroed
    int32_t* ocount;   // [H] overflow entries                      } per
    int32_t* big;      // [H] hub needs the HBM table               } sub-
    int32_t* hub_own;  // [H] connection to the own label           } round
    int32_t* ekeys;    // partition regions (label, summed weight)
    int32_t* evals;
    int32_t* okeys;    // overflow of full regions
    int32_t* ovals;
    int32_t* gkeys;    // HBM tables
    int32_t* gvals;
    int32_t* w_conn;   // winners per partition, then per table chunk
    uint64_t* w_tie;
    int32_t* w_x;
    int32_t part_limit;  // partitions with more entries take the HBM table path
};

constexpr int kHubThreads = 1024;
constexpr int kPartThreads = 256;
constexpr int kPartTable = 8192;  // 64 KB LDS table of a partition workgroup
constexpr int kMaxPartLog = 10;   // at most 1024 partitions per hub

__device__ __forceinline__ uint32_t part_of(int32_t x, int32_t plog) {
    return plog == 0 ? 0u : (slot_hash(static_cast<uint32_t>(x)) >> (32 - plog));
}

// Sums one chunk of a hub row in an LDS table, then scatters the chunk's
// distinct (label, weight) entries into the hub's label partitions.
__global__ void __launch_bounds__(kHubThreads) hub_chunk_kernel(EvalArgs A, HubArgs H) {
    __shared__ int32_t keys[kBlockTable];
    __shared__ int32_t vals[kBlockTable];
    __shared__ uint32_t pcount[1 << kMaxPartLog];
    __shared__ int32_t pbase[1 << kMaxPartLog];
    constexpr int kPer = kBlockTable / kHubThreads;
    const int tid = threadIdx.x;
    const int32_t h = H.chunk_hub[blockIdx.x];
    const int32_t v = H.hub_nodes[h];
    const int64_t begin = H.chunk_begin[blockIdx.x];
    const int64_t row_end = A.xadj[v + 1];
    const int64_t end = begin + kHubChunk < row_end ? begin + kHubChunk : row_end;
    const uint32_t tsz = table_size_for(static_cast<int32_t>(end - begin), 1024, kBlockTable);
    const uint32_t mask = tsz - 1;
    const int32_t plog = H.hub_plog[h];
    const int32_t P = 1 << plog;
    for (uint32_t j = tid; j < tsz; j += kHubThreads) {
        keys[j] = -1;
        vals[j] = 0;
    }
    for (int32_t j = tid; j < P; j += kHubThreads) pcount[j] = 0;
    __syncthreads();
    insert_slots<kHubThreads, 4>(A, begin, static_cast<int32_t>(end - begin), keys, vals, mask, tid);
    __syncthreads();
    for (int j = 0; j < kPer; ++j) {
        const uint32_t e = static_cast<uint32_t>(tid) * kPer + j;
        if (e < tsz && keys[e] >= 0) atomicAdd(&pcount[part_of(keys[e], plog)], 1u);
    }
    __syncthreads();
    for (int32_t j = tid; j < P; j += kHubThreads) {
        const uint32_t c = pcount[j];
        pbase[j] = c ? atomicAdd(&H.rcount[H.hub_pbase[h] + j], static_cast<int32_t>(c)) : 0;
        pcount[j] = 0;
    }
    __syncthreads();
    const int32_t cap = H.hub_cap[h];
    const int64_t rb = H.hub_rbase[h];
    for (int j = 0; j < kPer; ++j) {
        const uint32_t e = static_cast<uint32_t>(tid) * kPer + j;
        if (e >= tsz || keys[e] < 0) continue;
        const uint32_t p = part_of(keys[e], plog);
        const int32_t idx = pbase[p] + static_cast<int32_t>(atomicAdd(&pcount[p], 1u));
        if (idx < cap) {
            const int64_t at = rb + static_cast<int64_t>(p) * cap + idx;
            H.ekeys[at] = keys[e];
            H.evals[at] = vals[e];
        } else {  // region full: the rest of the partition goes to the hub's overflow list
            const int64_t at = H.hub_obase[h] + atomicAdd(&H.ocount[h], 1);
            H.okeys[at] = keys[e];
            H.ovals[at] = vals[e];
        }
    }
}

__device__ __forceinline__ int32_t block_sum_part(int32_t v, int32_t* s_red) {
    v = wave_sum(v);
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t t = 0;
    for (int w = 0; w < kPartThreads / 64; ++w) t += s_red[w];
    __syncthreads();
    return t;
}

// One workgroup per label partition of a hub: sums the partition's entries
// in LDS and writes the partition's best eligible label.  A partition with
// more than part_limit entries marks its hub for the HBM table path.
__global__ void __launch_bounds__(kPartThreads) hub_part_kernel(EvalArgs A, HubArgs H) {
    __shared__ int32_t keys[kPartTable];
    __shared__ int32_t vals[kPartTable];
    __shared__ int32_t s_red[kPartThreads / 64];
    __shared__ int32_t s_conn[kPartThreads / 64];
    __shared__ int32_t s_x[kPartThreads / 64];
    __shared__ uint64_t s_tie[kPartThreads / 64];
    const int tid = threadIdx.x;
    const int32_t gp = blockIdx.x;
    const int32_t h = H.part_hub[gp];
    const int32_t p = gp - H.hub_pbase[h];
    const int32_t plog = H.hub_plog[h];
    const int32_t cap = H.hub_cap[h];
    const int32_t in_region = H.rcount[gp] < cap ? H.rcount[gp] : cap;
    const int32_t ov = H.ocount[h];
    const int64_t ob = H.hub_obase[h];
    int32_t mine = 0;
    for (int32_t j = tid; j < ov; j += kPartThreads) mine += part_of(H.okeys[ob + j], plog) == static_cast<uint32_t>(p);
    const int32_t total = in_region + (ov > 0 ? block_sum_part(mine, s_red) : 0);
    if (total > H.part_limit) {
        if (tid == 0) H.big[h] = 1;
        return;
    }
    const uint32_t tsz = table_size_for(total, 256, kPartTable);
    const uint32_t mask = tsz - 1;
    for (uint32_t j = tid; j < tsz; j += kPartThreads) {
        keys[j] = -1;
        vals[j] = 0;
    }
    __syncthreads();
    const int64_t r0 = H.hub_rbase[h] + static_cast<int64_t>(p) * cap;
    for (int32_t j = tid; j < in_region; j += kPartThreads) table_add(keys, vals, mask, H.ekeys[r0 + j], H.evals[r0 + j]);
    for (int32_t j = tid; j < ov; j += kPartThreads) {
        const int32_t x = H.okeys[ob + j];
        if (part_of(x, plog) == static_cast<uint32_t>(p)) table_add(keys, vals, mask, x, H.ovals[ob + j]);
    }
    __syncthreads();
    const int32_t v = H.hub_nodes[h];
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    Best best;
    best_init(best);
    for (uint32_t j = tid; j < tsz; j += kPartThreads) {
        const int32_t x = keys[j];
        if (x < 0) continue;
        const int32_t conn = vals[j];
        if (x == a) {
            H.hub_own[h] = conn;  // only the partition of a holds a, in one entry
            continue;
        }
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c)) continue;
        best_consider(best, x, conn, A.tp);
    }
    int32_t bx, bconn;
    wave_argmax(best, A.tp, bx, bconn);
    const int wid = tid >> 6;
    if (lane_id() == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(A.tp, bx) : ~0ULL;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < kPartThreads / 64; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        H.w_conn[gp] = fc;
        H.w_tie[gp] = ft;
        H.w_x[gp] = fx;
    }
}

// Decision of a hub from the winners in [first[h], first[h+1]).
__device__ __forceinline__ void hub_decide(const EvalArgs& A, const HubArgs& H, int32_t h, const int32_t* first) {
    const int32_t v = H.hub_nodes[h];
    const int32_t a = A.label[v];
    int32_t fc = -1, fx = -1;
    uint64_t ft = ~0ULL;
    for (int32_t j = first[h] + lane_id(); j < first[h + 1]; j += 64)
        combine_into(fc, ft, fx, H.w_conn[j], H.w_tie[j], H.w_x[j]);
    const int32_t maxc = wave_max(fx >= 0 ? fc : -1);
    int32_t bx = -1;
    if (maxc >= 0) {
        const bool top = fx >= 0 && fc == maxc;
        const uint64_t mt = wave_min_u64(top ? ft : ~0ULL);
        bx = wave_min((top && ft == mt) ? fx : INT_MAX);
    }
    const bool over = A.refine && A.w[a] > A.bound;
    if (lane_id() == 0) store_result(A, h, bx, maxc, H.hub_own[h], over);
}

__global__ void __launch_bounds__(64) hub_finish_kernel(EvalArgs A, HubArgs H) {
    if (H.big[blockIdx.x]) return;
    hub_decide(A, H, blockIdx.x, H.hub_pbase);
}

// HBM table path for marked hubs: clear the table ...
__global__ void __launch_bounds__(256) hub_clear_kernel(HubArgs H) {
    const int32_t h = H.tchunk_hub[blockIdx.x];
    if (!H.big[h]) return;
    const int64_t begin = H.tchunk_begin[blockIdx.x];
    const int64_t tend = H.hub_toff[h] + static_cast<int64_t>(H.hub_tmask[h]) + 1;
    const int64_t end = begin + kHubTChunk < tend ? begin + kHubTChunk : tend;
    for (int64_t j = begin + threadIdx.x; j < end; j += 256) {
        H.gkeys[j] = -1;
        H.gvals[j] = 0;
    }
}

// ... add every partition region (and, from partition 0, the overflow list) ...
__global__ void __launch_bounds__(256) hub_table_insert_kernel(HubArgs H) {
    const int32_t gp = blockIdx.x;
    const int32_t h = H.part_hub[gp];
    if (!H.big[h]) return;
    const int32_t p = gp - H.hub_pbase[h];
    const int32_t cap = H.hub_cap[h];
    const int32_t in_region = H.rcount[gp] < cap ? H.rcount[gp] : cap;
    int32_t* gk = H.gkeys + H.hub_toff[h];
    int32_t* gv = H.gvals + H.hub_toff[h];
    const uint32_t gmask = H.hub_tmask[h];
    const int64_t r0 = H.hub_rbase[h] + static_cast<int64_t>(p) * cap;
    for (int32_t j = threadIdx.x; j < in_region; j += 256) table_add(gk, gv, gmask, H.ekeys[r0 + j], H.evals[r0 + j]);
    if (p == 0) {
        const int64_t ob = H.hub_obase[h];
        for (int32_t j = threadIdx.x; j < H.ocount[h]; j += 256) table_add(gk, gv, gmask, H.okeys[ob + j], H.ovals[ob + j]);
    }
}

// ... pick the best entry of each table chunk ...
__global__ void __launch_bounds__(256) hub_scan_kernel(EvalArgs A, HubArgs H, int32_t wbase) {
    __shared__ int32_t s_conn[4];
    __shared__ int32_t s_x[4];
    __shared__ uint64_t s_tie[4];
    const int32_t h = H.tchunk_hub[blockIdx.x];
    if (!H.big[h]) return;
    const int32_t v = H.hub_nodes[h];
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    const int64_t begin = H.tchunk_begin[blockIdx.x];
    const int64_t tend = H.hub_toff[h] + static_cast<int64_t>(H.hub_tmask[h]) + 1;
    const int64_t end = begin + kHubTChunk < tend ? begin + kHubTChunk : tend;
    Best best;
    best_init(best);
    for (int64_t j = begin + threadIdx.x; j < end; j += 256) {
        const int32_t x = H.gkeys[j];
        if (x < 0) continue;
        const int32_t conn = H.gvals[j];
        if (x == a) {
            H.hub_own[h] = conn;
            continue;
        }
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c)) continue;
        best_consider(best, x, conn, A.tp);
    }
    int32_t bx, bconn;
    wave_argmax(best, A.tp, bx, bconn);
    const int wid = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(A.tp, bx) : ~0ULL;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < 4; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        H.w_conn[wbase + blockIdx.x] = fc;
        H.w_tie[wbase + blockIdx.x] = ft;
        H.w_x[wbase + blockIdx.x] = fx;
    }
}

// ... and decide from the chunk winners (stored after the partition winners).
__global__ void __launch_bounds__(64) hub_big_finish_kernel(EvalArgs A, HubArgs H, const int32_t* tfirst_shifted) {
    if (!H.big[blockIdx.x]) return;
    hub_decide(A, H, blockIdx.x, tfirst_shifted);
}

// ------------------------------------------------------- block utilities

// One atomic per block: returns the position of this thread's item among all
// flagged items of the grid (order within the grid unspecified).
__device__ __forceinline__ uint32_t block_append(bool flag, uint32_t* counter) {
    __shared__ uint32_t s_cnt[4];
    __shared__ uint32_t s_base;
    const int wid = threadIdx.x >> 6;
    const uint64_t m = __ballot(flag);
    if (lane_id() == 0) s_cnt[wid] = static_cast<uint32_t>(__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < 4; ++w) {
            const uint32_t c = s_cnt[w];
            s_cnt[w] = run;
            run += c;
        }
        s_base = run ? atomicAdd(counter, run) : 0;
    }
    __syncthreads();
    const uint32_t idx = s_base + s_cnt[wid] + static_cast<uint32_t>(__popcll(m & lanemask_lt()));
    __syncthreads();
    return idx;
}

__device__ __forceinline__ int32_t block_sum_i32(int32_t v) {
    __shared__ int32_t s[4];
    v = wave_sum(v);
    if (lane_id() == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    const int32_t t = s[0] + s[1] + s[2] + s[3];
    __syncthreads();
    return t;
}

// ------------------------------------------------- candidates and admission

// tsum[t] += c(v) over the candidates of the sub-round; counts them.
template <bool kSmall>
__global__ void __launch_bounds__(256) cand_accum_kernel(const int32_t* __restrict__ ct,
                                                         const int32_t* __restrict__ nodes, int32_t count,
                                                         const int32_t* __restrict__ vw, int32_t* __restrict__ tsum,
                                                         int32_t nw, Counters* ctr) {
    __shared__ int32_t loc[kSmall ? kSmallLabels : 1];
    if (kSmall) {
        for (int j = threadIdx.x; j < nw; j += 256) loc[j] = 0;
        __syncthreads();
    }
    int32_t found = 0;
    for (int32_t p = blockIdx.x * 256 + threadIdx.x; p < count; p += gridDim.x * 256) {
        const int32_t t = ct[p];
        if (t < 0) continue;
        ++found;
        const int32_t c = vw ? vw[nodes[p]] : 1;
        if (c) {
            if (kSmall) atomicAdd(&loc[t], c);
            else atomicAdd(&tsum[t], c);
        }
    }
    if (kSmall) {
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256)
            if (loc[j]) atomicAdd(&tsum[j], loc[j]);
    }
    const int32_t tot = block_sum_i32(found);
    if (threadIdx.x == 0 && tot) atomicAdd(&ctr->ncand, static_cast<uint32_t>(tot));
}

// Fast path of admission: if everything aimed at t fits, admit it all;
// otherwise the candidate goes to the slow list.
__global__ void __launch_bounds__(256) admit_kernel(const int32_t* __restrict__ ct, const int32_t* __restrict__ cg,
                                                    int32_t count, const int32_t* __restrict__ w,
                                                    const int32_t* __restrict__ tsum, int64_t bound,
                                                    uint8_t* __restrict__ ok, uint32_t* __restrict__ slow_idx,
                                                    Counters* ctr) {
    __shared__ int32_t s_min[4], s_max[4];
    const int32_t stride = gridDim.x * 256;
    const int32_t iters = (count + stride - 1) / stride;
    int32_t gmin = INT_MAX, gmax = INT_MIN;
    for (int32_t it = 0; it < iters; ++it) {
        const int32_t p = it * stride + blockIdx.x * 256 + threadIdx.x;
        bool slow = false;
        if (p < count) {
            const int32_t t = ct[p];
            uint8_t o = 0;
            if (t >= 0) {
                if (static_cast<int64_t>(w[t]) + tsum[t] <= bound) {
                    o = 1;
                } else {
                    slow = true;
                    const int32_t gain = cg[p];
                    gmin = gain < gmin ? gain : gmin;
                    gmax = gain > gmax ? gain : gmax;
                }
            }
            ok[p] = o;
        }
        const uint32_t j = block_append(slow, &ctr->nslow);
        if (slow) slow_idx[j] = static_cast<uint32_t>(p);
    }
    gmin = wave_min(gmin);
    gmax = wave_max(gmax);
    if (lane_id() == 0) {
        s_min[threadIdx.x >> 6] = gmin;
        s_max[threadIdx.x >> 6] = gmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t a = INT_MAX, b = INT_MIN;
        for (int w2 = 0; w2 < 4; ++w2) {
            a = s_min[w2] < a ? s_min[w2] : a;
            b = s_max[w2] > b ? s_max[w2] : b;
        }
        if (a != INT_MAX) atomicMin(&ctr->gmin, a);
        if (b != INT_MIN) atomicMax(&ctr->gmax, b);
    }
}

// key = [t][gmax - gain][v] packed into the low bits; value = schedule entry.
__global__ void slow_keys_kernel(const uint32_t* __restrict__ slow_idx, uint32_t m, const int32_t* __restrict__ nodes,
                                 const int32_t* __restrict__ ct, const int32_t* __restrict__ cg, int32_t gmax,
                                 int bits_v, int shift_t, int with_t, uint64_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t p = slow_idx[j];
    uint64_t k = (static_cast<uint64_t>(static_cast<int64_t>(gmax) - cg[p]) << bits_v) |
                 static_cast<uint64_t>(static_cast<uint32_t>(nodes[p]));
    if (with_t) k |= static_cast<uint64_t>(static_cast<uint32_t>(ct[p])) << shift_t;
    keys[j] = k;
    vals[j] = p;
}

__global__ void slow_keys_t_kernel(const uint32_t* __restrict__ vals, uint32_t m, const int32_t* __restrict__ ct,
                                   uint64_t* __restrict__ keys) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    keys[j] = static_cast<uint64_t>(static_cast<uint32_t>(ct[vals[j]]));
}

__global__ void slow_gather_kernel(const uint32_t* __restrict__ vals, uint32_t m, const int32_t* __restrict__ nodes,
                                   const int32_t* __restrict__ ct, const int32_t* __restrict__ vw,
                                   int64_t* __restrict__ csum, int32_t* __restrict__ head) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t p = vals[j];
    csum[j] = vw ? vw[nodes[p]] : 1;
    head[j] = (j == 0 || ct[vals[j - 1]] != ct[p]) ? static_cast<int32_t>(j) : 0;
}

// Sorted by (target, gain desc, node asc): admit while the running weight of
// the target's candidates keeps it within the bound (node weights are >= 0,
// so the admitted set is a prefix).
__global__ void slow_admit_kernel(const uint32_t* __restrict__ vals, uint32_t m, const int32_t* __restrict__ ct,
                                  const int32_t* __restrict__ w, const int64_t* __restrict__ psum,
                                  const int32_t* __restrict__ segstart, int64_t bound, uint8_t* __restrict__ ok) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t p = vals[j];
    const int32_t s0 = segstart[j];
    const int64_t pre = psum[j] - (s0 > 0 ? psum[s0 - 1] : 0);
    ok[p] = (static_cast<int64_t>(w[ct[p]]) + pre <= bound) ? 1 : 0;
}

template <bool kSmall>
__global__ void __launch_bounds__(256) apply_kernel(const int32_t* __restrict__ ct, const uint8_t* __restrict__ ok,
                                                    const int32_t* __restrict__ nodes, int32_t count,
                                                    const int32_t* __restrict__ vw, int32_t* __restrict__ label,
                                                    int32_t* __restrict__ w, int32_t* __restrict__ tsum, int32_t nw) {
    __shared__ int32_t delta[kSmall ? kSmallLabels : 1];
    if (kSmall) {
        for (int j = threadIdx.x; j < nw; j += 256) delta[j] = 0;
        __syncthreads();
    }
    for (int32_t p = blockIdx.x * 256 + threadIdx.x; p < count; p += gridDim.x * 256) {
        const int32_t t = ct[p];
        if (t < 0) continue;
        if (!kSmall) tsum[t] = 0;
        if (!ok[p]) continue;
        const int32_t v = nodes[p];
        const int32_t a = label[v];
        const int32_t c = vw ? vw[v] : 1;
        label[v] = t;
        if (c) {
            if (kSmall) {
                atomicAdd(&delta[t], c);
                atomicSub(&delta[a], c);
            } else {
                atomicAdd(&w[t], c);
                atomicSub(&w[a], c);
            }
        }
    }
    if (kSmall) {
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256)
            if (delta[j]) atomicAdd(&w[j], delta[j]);
    }
}

__global__ void reset_counters_kernel(Counters* ctr) {
    ctr->ncand = 0;
    ctr->nslow = 0;
    ctr->gmin = INT_MAX;
    ctr->gmax = INT_MIN;
}

// --------------------------------------------------------------- schedule

// Category of a node: colour * kNB + degree bucket; degree-0 nodes never move
// and go to the extra category ncat.
__global__ void __launch_bounds__(256) classify_kernel(int32_t n, const int64_t* __restrict__ xadj,
                                                       const int32_t* __restrict__ color_override, uint64_t hc,
                                                       int32_t nsub, int32_t th0, int32_t th1, int32_t th2,
                                                       int32_t th3, int32_t th4, int32_t th5,
                                                       uint64_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals, uint32_t* __restrict__ cat_count,
                                                       unsigned long long* __restrict__ cat_slots, Counters* ctr) {
    __shared__ uint32_t hist[16 * kNB + 1];
    __shared__ unsigned long long shist[16 * kNB + 1];
    const int ncat = nsub * kNB;
    for (int j = threadIdx.x; j <= ncat; j += 256) {
        hist[j] = 0;
        shist[j] = 0;
    }
    __syncthreads();
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) {
        const int64_t d = xadj[v + 1] - xadj[v];
        int32_t col;
        if (color_override) {
            col = color_override[v];
            if (col < 0 || col >= nsub) {
                atomicOr(&ctr->bad_color, 1u);
                col = 0;
            }
        } else {
            col = static_cast<int32_t>(mix64(hc ^ static_cast<uint64_t>(static_cast<uint32_t>(v))) %
                                       static_cast<uint64_t>(nsub));
        }
        const int32_t bucket = d <= th0   ? 0
                               : d <= th1 ? 1
                               : d <= th2 ? 2
                               : d <= th3 ? 3
                               : d <= th4 ? 4
                               : d <= th5 ? 5
                                          : kHubBucket;
        const int32_t cat = d == 0 ? ncat : col * kNB + bucket;
        keys[v] = static_cast<uint64_t>(cat);
        vals[v] = static_cast<uint32_t>(v);
        atomicAdd(&hist[cat], 1u);
        if (d) atomicAdd(&shist[cat], static_cast<unsigned long long>(d));
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= ncat; j += 256) {
        if (hist[j]) atomicAdd(&cat_count[j], hist[j]);
        if (shist[j]) atomicAdd(&cat_slots[j], shist[j]);
    }
}

// rows[2i] = first slot of nodes[i], rows[2i+1] = its degree
__global__ void gather_rows_kernel(const int32_t* __restrict__ nodes, int32_t count, const int64_t* __restrict__ xadj,
                                   int64_t* __restrict__ rows) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) {
        rows[2 * i] = xadj[nodes[i]];
        rows[2 * i + 1] = xadj[nodes[i] + 1] - xadj[nodes[i]];
    }
}

template <bool kSmall>
__global__ void __launch_bounds__(256) label_weights_kernel(int32_t n, const int32_t* __restrict__ label,
                                                            const int32_t* __restrict__ vw, int32_t* __restrict__ w,
                                                            int32_t nw) {
    __shared__ int32_t loc[kSmall ? kSmallLabels : 1];
    if (kSmall) {
        for (int j = threadIdx.x; j < nw; j += 256) loc[j] = 0;
        __syncthreads();
    }
    for (int32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int32_t c = vw ? vw[v] : 1;
        if (!c) continue;
        if (kSmall) atomicAdd(&loc[label[v]], c);
        else atomicAdd(&w[label[v]], c);
    }
    if (kSmall) {
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256)
            if (loc[j]) atomicAdd(&w[j], loc[j]);
    }
}

// Per-colour hub metadata built on the host after the schedule is known.
struct HubPlan {
    int32_t count = 0;
    int32_t nchunks = 0;
    int32_t nparts = 0;
    int32_t ntchunks = 0;
    int64_t region_entries = 0;
    int64_t overflow_entries = 0;
    int64_t table_entries = 0;
    // hub_nodes | plog | pbase[H+1] | cap | tfirst_shifted[H+1] | chunk_hub | part_hub | tchunk_hub
    DBuf<int32_t> i32;
    // rbase | obase | toff | chunk_begin | tchunk_begin
    DBuf<int64_t> i64;
    DBuf<uint32_t> u32;  // tmask
};

thread_local Counters* t_host_ctr = nullptr;

Counters* host_counters() {
    if (!t_host_ctr) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&t_host_ctr), sizeof(Counters), hipHostMallocDefault));
    return t_host_ctr;
}

unsigned capped_grid(int64_t items) {
    const int64_t g = (items + 255) / 256;
    return static_cast<unsigned>(g < 1 ? 1 : (g > kMaxBlocks ? kMaxBlocks : g));
}

}  // namespace

void label_weights(const DevGraph& g, const int32_t* label, int32_t* w, int32_t nw, hipStream_t s) {
    fill_i32(w, 0, nw, s);
    if (g.n > 0) {
        if (nw <= kSmallLabels)
            label_weights_kernel<true><<<capped_grid(g.n), 256, 0, s>>>(g.n, label, g.vw, w, nw);
        else
            label_weights_kernel<false><<<grid_for(g.n, 256), 256, 0, s>>>(g.n, label, g.vw, w, nw);
        LAUNCHCHK();
    }
}

LPResult run_lp(const DevGraph& g, int32_t phase, int32_t level, uint64_t seed, int32_t nsub, int32_t rounds,
                int64_t bound, int32_t* label, int32_t* w, int32_t nw, const int32_t* color_override,
                const LPTuning& tune, hipStream_t s) {
    LPResult res;
    const int32_t n = g.n;
    if (n == 0 || rounds <= 0) return res;
    if (nsub < 1 || nsub > 16) fail(-1, "subrounds must be in 1..16");
    const bool small = nw <= kSmallLabels;
    static const bool trace = std::getenv("SCLAP_TRACE") != nullptr;  // per sub-round counts on stderr

    // --- schedule: nodes grouped by (colour, degree bucket), ascending ids
    const int32_t ncat = nsub * kNB;
    const int32_t th1 = std::max(1, std::min(tune.lane_max, kLaneMax));
    const int32_t th0 = std::min(kLaneSmall, th1);
    const int32_t th2 = std::max(th1, std::min(tune.wave_max, kWaveMaxDeg));
    const int32_t tb = std::max(th2, std::min(tune.block_max, kBlockMaxDeg));
    const int32_t th3 = std::min(tb, std::max(th2, kBlock1Max));
    const int32_t th4 = std::min(tb, std::max(th3, kBlock2Max));
    const int32_t th5 = tb;
    DBuf<uint64_t> ckeys(n, s), ckeys_tmp(n, s);
    DBuf<uint32_t> order(n, s), order_tmp(n, s);
    DBuf<uint32_t> cat_count(ncat + 1, s);
    DBuf<unsigned long long> cat_slots(ncat + 1, s);
    DBuf<Counters> ctr(1, s);
    fill_u32(cat_count.get(), 0, ncat + 1, s);
    HIPCHK(hipMemsetAsync(cat_slots.get(), 0, (ncat + 1) * sizeof(unsigned long long), s));
    HIPCHK(hipMemsetAsync(ctr.get(), 0, sizeof(Counters), s));
    const uint64_t hc = hash_prefix({seed, 1, static_cast<uint64_t>(static_cast<uint32_t>(level)),
                                     static_cast<uint64_t>(static_cast<uint32_t>(phase))});
    {
        ProfScope ps("lp_schedule", 0, s);
        classify_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g.xadj, color_override, hc, nsub, th0, th1, th2, th3, th4, th5,
                                                         ckeys.get(), order.get(), cat_count.get(), cat_slots.get(),
                                                         ctr.get());
        LAUNCHCHK();
    }
    RadixScratch rs;
    radix_sort_pairs(ckeys.get(), order.get(), ckeys_tmp.get(), order_tmp.get(), n, 0, bits_for(ncat), rs, s);
    ckeys.release();
    ckeys_tmp.release();
    order_tmp.release();
    std::vector<uint32_t> cnt(ncat + 1);
    std::vector<unsigned long long> cslots(ncat + 1);
    HIPCHK(hipMemcpyAsync(cnt.data(), cat_count.get(), (ncat + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(cslots.data(), cat_slots.get(), (ncat + 1) * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    Counters* hctr = host_counters();
    HIPCHK(hipMemcpyAsync(hctr, ctr.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hctr->bad_color) fail(-1, "color_override value outside [0, subrounds)");
    std::vector<int64_t> off(ncat + 2, 0);
    for (int32_t j = 0; j <= ncat; ++j) off[j + 1] = off[j] + cnt[j];
    const int32_t* nodes = reinterpret_cast<const int32_t*>(order.get());

    // --- hub plans per colour
    std::vector<HubPlan> plans(nsub);
    int64_t max_region = 0, max_over = 0, max_table = 0, max_win = 0, max_hub_ints = 0;
    for (int32_t sc = 0; sc < nsub; ++sc) {
        const int32_t cat = sc * kNB + kHubBucket;
        const int32_t H = static_cast<int32_t>(cnt[cat]);
        HubPlan& P = plans[sc];
        P.count = H;
        if (H == 0) continue;
        std::vector<int32_t> hn(H);
        std::vector<int64_t> rows(2 * static_cast<size_t>(H)), hd(H), xs(H);
        HIPCHK(hipMemcpyAsync(hn.data(), nodes + off[cat], H * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        {
            DBuf<int64_t> drows(2 * static_cast<size_t>(H), s);
            gather_rows_kernel<<<grid_for(H, 256), 256, 0, s>>>(nodes + off[cat], H, g.xadj, drows.get());
            LAUNCHCHK();
            HIPCHK(hipMemcpyAsync(rows.data(), drows.get(), 2 * H * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        for (int32_t h = 0; h < H; ++h) {
            xs[h] = rows[2 * h];
            hd[h] = rows[2 * h + 1];
        }
        std::vector<int32_t> plog(H), pbase(H + 1), cap(H), tfirst(H + 1), chub, phub, thub;
        std::vector<int64_t> rbase(H), obase(H), toff(H), cbeg, tbeg;
        std::vector<uint32_t> tmask(H);
        int64_t rtot = 0, otot = 0, ttot = 0;
        int32_t np = 0, ntc = 0;
        for (int32_t h = 0; h < H; ++h) {
            // about 2048 entries per label partition, at most 1024 partitions
            int32_t lg = 0;
            while (lg < kMaxPartLog && (static_cast<int64_t>(2048) << lg) < hd[h]) ++lg;
            plog[h] = lg;
            const int64_t per = (hd[h] + (1LL << lg) - 1) >> lg;
            cap[h] = static_cast<int32_t>(std::min<int64_t>(2 * per + 64, hd[h]));
            if (tune.hub_region_cap > 0) cap[h] = std::min(cap[h], tune.hub_region_cap);
            pbase[h] = np;
            for (int32_t p = 0; p < (1 << lg); ++p) phub.push_back(h);
            np += 1 << lg;
            rbase[h] = rtot;
            rtot += static_cast<int64_t>(cap[h]) << lg;
            obase[h] = otot;
            otot += hd[h];
            uint64_t tsz = 1;
            while (tsz < 2 * static_cast<uint64_t>(hd[h])) tsz <<= 1;
            toff[h] = ttot;
            tmask[h] = static_cast<uint32_t>(tsz - 1);
            for (int64_t sl = 0; sl < hd[h]; sl += kHubChunk) {
                chub.push_back(h);
                cbeg.push_back(xs[h] + sl);
            }
            tfirst[h] = ntc;
            for (int64_t e = 0; e < static_cast<int64_t>(tsz); e += kHubTChunk) {
                thub.push_back(h);
                tbeg.push_back(ttot + e);
                ++ntc;
            }
            ttot += static_cast<int64_t>(tsz);
        }
        pbase[H] = np;
        tfirst[H] = ntc;
        P.nchunks = static_cast<int32_t>(chub.size());
        P.nparts = np;
        P.ntchunks = ntc;
        P.region_entries = rtot;
        P.overflow_entries = otot;
        P.table_entries = ttot;
        // table-chunk winners are stored after the partition winners
        for (int32_t h = 0; h <= H; ++h) tfirst[h] += np;
        std::vector<int32_t> i32;
        for (const auto* vec : {&hn, &plog, &pbase, &cap, &tfirst, &chub, &phub, &thub})
            i32.insert(i32.end(), vec->begin(), vec->end());
        std::vector<int64_t> i64;
        for (const auto* vec : {&rbase, &obase, &toff, &cbeg, &tbeg}) i64.insert(i64.end(), vec->begin(), vec->end());
        P.i32.alloc(i32.size(), s);
        P.i64.alloc(i64.size(), s);
        P.u32.alloc(tmask.size(), s);
        HIPCHK(hipMemcpyAsync(P.i32.get(), i32.data(), i32.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P.i64.get(), i64.data(), i64.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P.u32.get(), tmask.data(), tmask.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // host vectors go out of scope
        max_region = std::max(max_region, rtot);
        max_over = std::max(max_over, otot);
        max_table = std::max(max_table, ttot);
        max_win = std::max(max_win, static_cast<int64_t>(np) + ntc);
        max_hub_ints = std::max(max_hub_ints, static_cast<int64_t>(np) + 3 * static_cast<int64_t>(H));
    }
    DBuf<int32_t> ekeys, evals, okeys, ovals, gkeys, gvals, hub_ints, w_conn, w_x;
    DBuf<uint64_t> w_tie;
    if (max_win > 0) {
        ekeys.alloc(max_region, s);
        evals.alloc(max_region, s);
        okeys.alloc(max_over, s);
        ovals.alloc(max_over, s);
        gkeys.alloc(max_table, s);
        gvals.alloc(max_table, s);
        hub_ints.alloc(max_hub_ints, s);
        w_conn.alloc(max_win, s);
        w_x.alloc(max_win, s);
        w_tie.alloc(max_win, s);
    }

    // --- per-entry candidate buffers: at most the nodes of one colour
    int64_t max_color = 0;
    for (int32_t sc = 0; sc < nsub; ++sc) max_color = std::max(max_color, off[(sc + 1) * kNB] - off[sc * kNB]);
    const int64_t cap = std::max<int64_t>(max_color, 1);
    DBuf<int32_t> ct(cap, s), cg(cap, s), tsum(nw, s);
    DBuf<uint8_t> ok(cap, s);
    DBuf<uint32_t> slow_idx(cap, s);
    fill_i32(tsum.get(), 0, nw, s);

    EvalArgs A;
    A.xadj = g.xadj;
    A.adj = g.adj;
    A.ew = g.ew;
    A.vw = g.vw;
    A.label = label;
    A.w = w;
    A.bound = bound;
    A.refine = phase == kRefine ? 1 : 0;

    // Algorithmic bytes of one evaluation launch: per node its schedule entry,
    // row offsets, own label and weight (and w(own) when refining) and its
    // result (target, gain); per slot the neighbour id, edge weight and
    // neighbour label.
    const double node_bytes = 4.0 + 16.0 + 4.0 + (g.vw ? 4.0 : 0.0) + (phase == kRefine ? 4.0 : 0.0) + 8.0;
    const double slot_bytes = 8.0 + (g.ew ? 4.0 : 0.0);
    auto eval_bytes = [&](int64_t nodes_in, unsigned long long slots_in) {
        return node_bytes * static_cast<double>(nodes_in) + slot_bytes * static_cast<double>(slots_in);
    };
    reset_counters_kernel<<<1, 1, 0, s>>>(ctr.get());
    LAUNCHCHK();
    DBuf<uint64_t> sk, sk_tmp;
    DBuf<uint32_t> sv_tmp;
    DBuf<int64_t> psum;
    DBuf<int32_t> heads;
    const int bits_v = bits_for(static_cast<uint64_t>(n - 1));
    const int bits_t = bits_for(static_cast<uint64_t>(nw > 0 ? nw - 1 : 0));

    for (int32_t r = 0; r < rounds; ++r) {
        A.tp = hash_prefix({seed, 2, static_cast<uint64_t>(static_cast<uint32_t>(level)),
                            static_cast<uint64_t>(static_cast<uint32_t>(phase)),
                            static_cast<uint64_t>(static_cast<uint32_t>(r))});
        int64_t round_cands = 0;
        for (int32_t sc = 0; sc < nsub; ++sc) {
            const int32_t c0 = sc * kNB;
            const int64_t ccount = off[c0 + kNB] - off[c0];
            if (ccount == 0) continue;
            const int32_t* cnodes = nodes + off[c0];
            // evaluation: one result per schedule entry of this colour
            for (int32_t bk = 0; bk < kHubBucket; ++bk) {
                const int64_t count = off[c0 + bk + 1] - off[c0 + bk];
                if (count == 0) continue;
                A.nodes = nodes + off[c0 + bk];
                A.count = static_cast<int32_t>(count);
                A.ct = ct.get() + (off[c0 + bk] - off[c0]);
                A.cg = cg.get() + (off[c0 + bk] - off[c0]);
                static const char* const kNames[kHubBucket] = {"lp_eval_lane4", "lp_eval_lane16", "lp_eval_wave",
                                                               "lp_eval_block1k", "lp_eval_block4k",
                                                               "lp_eval_block8k"};
                ProfScope ps(kNames[bk], eval_bytes(count, cslots[c0 + bk]), s);
                const unsigned nb = static_cast<unsigned>(count);
                if (bk == 0) {
                    eval_lane_kernel<kLaneSmall><<<grid_for(count, 256), 256, 0, s>>>(A);
                } else if (bk == 1) {
                    eval_lane_kernel<kLaneMax><<<grid_for(count, 256), 256, 0, s>>>(A);
                } else if (bk == 2) {
                    eval_wave_kernel<<<grid_for(count, 4), 256, 0, s>>>(A);
                } else if (bk == 3) {
                    eval_block_kernel<256, 2 * kBlock1Max><<<nb, 256, 0, s>>>(A);
                } else if (bk == 4) {
                    eval_block_kernel<512, 2 * kBlock2Max><<<nb, 512, 0, s>>>(A);
                } else {
                    eval_block_kernel<1024, kBlockTable><<<nb, 1024, 0, s>>>(A);
                }
                LAUNCHCHK();
            }
            const HubPlan& P = plans[sc];
            if (P.count > 0) {
                const int32_t Hn = P.count;
                HubArgs H;
                const int32_t* i32 = P.i32.get();
                H.hub_nodes = i32;
                H.hub_plog = i32 + Hn;
                H.hub_pbase = i32 + 2 * Hn;
                H.hub_cap = i32 + 3 * Hn + 1;
                const int32_t* tfirst_shifted = i32 + 4 * Hn + 1;
                H.hub_tfirst = tfirst_shifted;
                H.chunk_hub = i32 + 5 * Hn + 2;
                H.part_hub = H.chunk_hub + P.nchunks;
                H.tchunk_hub = H.part_hub + P.nparts;
                const int64_t* i64 = P.i64.get();
                H.hub_rbase = i64;
                H.hub_obase = i64 + Hn;
                H.hub_toff = i64 + 2 * Hn;
                H.chunk_begin = i64 + 3 * Hn;
                H.tchunk_begin = H.chunk_begin + P.nchunks;
                H.hub_tmask = P.u32.get();
                H.rcount = hub_ints.get();
                H.ocount = H.rcount + P.nparts;
                H.big = H.ocount + Hn;
                H.hub_own = H.big + Hn;
                H.ekeys = ekeys.get();
                H.evals = evals.get();
                H.okeys = okeys.get();
                H.ovals = ovals.get();
                H.gkeys = gkeys.get();
                H.gvals = gvals.get();
                H.w_conn = w_conn.get();
                H.w_tie = w_tie.get();
                H.w_x = w_x.get();
                H.part_limit = std::max(1, std::min(tune.hub_part_limit, kPartTable / 2));
                fill_i32(H.rcount, 0, static_cast<int64_t>(P.nparts) + 3 * Hn, s);
                A.nodes = H.hub_nodes;
                A.count = Hn;
                A.ct = ct.get() + (off[c0 + kHubBucket] - off[c0]);
                A.cg = cg.get() + (off[c0 + kHubBucket] - off[c0]);
                {
                    ProfScope ps("lp_eval_hub_chunk", eval_bytes(Hn, cslots[c0 + kHubBucket]), s);
                    hub_chunk_kernel<<<P.nchunks, kHubThreads, 0, s>>>(A, H);
                    LAUNCHCHK();
                }
                {
                    ProfScope ps("lp_eval_hub_part", 0, s);
                    hub_part_kernel<<<P.nparts, kPartThreads, 0, s>>>(A, H);
                    LAUNCHCHK();
                    hub_finish_kernel<<<Hn, 64, 0, s>>>(A, H);
                    LAUNCHCHK();
                }
                {
                    ProfScope ps("lp_eval_hub_table", 0, s);
                    hub_clear_kernel<<<P.ntchunks, 256, 0, s>>>(H);
                    LAUNCHCHK();
                    hub_table_insert_kernel<<<P.nparts, 256, 0, s>>>(H);
                    LAUNCHCHK();
                    hub_scan_kernel<<<P.ntchunks, 256, 0, s>>>(A, H, P.nparts);
                    LAUNCHCHK();
                    hub_big_finish_kernel<<<Hn, 64, 0, s>>>(A, H, tfirst_shifted);
                    LAUNCHCHK();
                }
            }
            // per-target candidate weight, then admission (fast path)
            {
                ProfScope ps("lp_admit", 0, s);
                if (small)
                    cand_accum_kernel<true><<<capped_grid(ccount), 256, 0, s>>>(ct.get(), cnodes, ccount, g.vw,
                                                                                tsum.get(), nw, ctr.get());
                else
                    cand_accum_kernel<false><<<capped_grid(ccount), 256, 0, s>>>(ct.get(), cnodes, ccount, g.vw,
                                                                                 tsum.get(), nw, ctr.get());
                LAUNCHCHK();
                admit_kernel<<<capped_grid(ccount), 256, 0, s>>>(ct.get(), cg.get(), ccount, w, tsum.get(), bound,
                                                                 ok.get(), slow_idx.get(), ctr.get());
                LAUNCHCHK();
            }
            HIPCHK(hipMemcpyAsync(hctr, ctr.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (profiler().on) profiler().collect();
            const uint32_t ncand = hctr->ncand;
            const uint32_t m = hctr->nslow;
            if (trace)
                fprintf(stderr, "[sclap] %s L%d r%d s%d n=%lld cand=%u slow=%u gain=[%d,%d] hubs=%d hub_slots=%llu\n",
                        phase == kRefine ? "refine" : "cluster", level, r, sc, static_cast<long long>(ccount), ncand,
                        m, m ? hctr->gmin : 0, m ? hctr->gmax : 0, plans[sc].count, cslots[c0 + kHubBucket]);
            if (m > 0) {
                // slow path: sort candidates of overflowing targets by
                // (target, gain desc, node asc) and admit the prefix that fits
                ProfScope ps("lp_admit_sorted", 0, s);
                const int bits_g = bits_for(static_cast<uint64_t>(static_cast<int64_t>(hctr->gmax) - hctr->gmin));
                const int low_bits = bits_g + bits_v;
                const bool single = low_bits + bits_t <= 64;
                sk.reserve(m, s);
                sk_tmp.reserve(m, s);
                sv_tmp.reserve(m, s);
                psum.reserve(m, s);
                heads.reserve(m, s);
                uint32_t* sv = slow_idx.get();  // values, sorted in place
                slow_keys_kernel<<<grid_for(m, 256), 256, 0, s>>>(slow_idx.get(), m, cnodes, ct.get(), cg.get(),
                                                                  hctr->gmax, bits_v, low_bits, single ? 1 : 0,
                                                                  sk.get(), sv);
                LAUNCHCHK();
                if (single) {
                    radix_sort_pairs(sk.get(), sv, sk_tmp.get(), sv_tmp.get(), m, 0, low_bits + bits_t, rs, s);
                } else {
                    radix_sort_pairs(sk.get(), sv, sk_tmp.get(), sv_tmp.get(), m, 0, low_bits, rs, s);
                    slow_keys_t_kernel<<<grid_for(m, 256), 256, 0, s>>>(sv, m, ct.get(), sk.get());
                    LAUNCHCHK();
                    radix_sort_pairs(sk.get(), sv, sk_tmp.get(), sv_tmp.get(), m, 0, bits_t, rs, s);
                }
                slow_gather_kernel<<<grid_for(m, 256), 256, 0, s>>>(sv, m, cnodes, ct.get(), g.vw, psum.get(),
                                                                    heads.get());
                LAUNCHCHK();
                inclusive_scan_i64(psum.get(), psum.get(), m, s);
                inclusive_max_i32(heads.get(), heads.get(), m, s);
                slow_admit_kernel<<<grid_for(m, 256), 256, 0, s>>>(sv, m, ct.get(), w, psum.get(), heads.get(), bound,
                                                                   ok.get());
                LAUNCHCHK();
            }
            if (ncand > 0) {
                ProfScope ps("lp_apply", 0, s);
                if (small) {
                    apply_kernel<true><<<capped_grid(ccount), 256, 0, s>>>(ct.get(), ok.get(), cnodes, ccount, g.vw,
                                                                           label, w, tsum.get(), nw);
                    LAUNCHCHK();
                    fill_i32(tsum.get(), 0, nw, s);
                } else {
                    apply_kernel<false><<<grid_for(ccount, 256), 256, 0, s>>>(ct.get(), ok.get(), cnodes, ccount,
                                                                              g.vw, label, w, tsum.get(), nw);
                    LAUNCHCHK();
                }
            }
            reset_counters_kernel<<<1, 1, 0, s>>>(ctr.get());
            LAUNCHCHK();
            round_cands += ncand;  // the first candidate of every target is always admitted
        }
        res.rounds_run = r + 1;
        res.moves += round_cands;
        if (round_cands == 0) break;
    }
    res.visits = static_cast<int64_t>(res.rounds_run) * g.S;
    HIPCHK(hipStreamSynchronize(s));
    if (profiler().on) profiler().collect();
    return res;
}

}  // namespace sclap
