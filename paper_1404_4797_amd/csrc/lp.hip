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

// buckets: lane4, lane16, group16 (16 lanes per node), group32, wave,
// block (3 table sizes), hub
constexpr int kNB = 9;
constexpr int kHubBucket = kNB - 1;
constexpr int kLaneSmall = 4;
constexpr int kLaneMax = 16;
constexpr int kG16Max = 32;  // 16 lanes and a 64-entry table per node
constexpr int kG32Max = 64;  // 32 lanes and a 128-entry table per node
constexpr int kWaveTable = 512;
constexpr int kWaveMaxDeg = kWaveTable / 2;
// the workgroup bucket with the longest rows (up to kBlockMaxDeg slots): a
// 10240-entry table (80 KB, probed modulo its size) by default, which leaves
// room on the compute unit for a workgroup with a 64 KB table; the 16384-entry
// power-of-two table (128 KB) as a tuning choice
constexpr int kBlockTable = 10240;
constexpr int kBlockTablePow2 = 16384;
constexpr int kBlockMaxDeg = kBlockTablePow2 / 2;
constexpr int kBlock1Max = 1024;  // 256 threads, 16 KB table
constexpr int kBlock2Max = 4096;  // 512 threads, 64 KB table
constexpr int kHubTable = 8192;          // LDS table of a hub chunk workgroup (64 KB: two per CU)
constexpr int kHubChunk = kHubTable / 2; // slots per hub workgroup (table load <= 1/2)
constexpr int kHubDenseChunk = 8192;     // slots per hub workgroup with dense block arrays
constexpr int kHubTChunk = 4096;         // HBM table entries per scan workgroup
constexpr int kSmallLabels = 4096;       // LDS-private histograms up to this many labels
constexpr int kMaxBlocks = 512;          // grid cap of the grid-stride candidate kernels
constexpr int kSmallSeg = 4096;          // segments up to this length: one selecting workgroup
constexpr int kSegChunk = 16384;         // entries per workgroup in the multi-workgroup selection
constexpr int kLargeBlocks = 256;        // grid of the multi-workgroup selection kernel
constexpr int kLargeThreads = 1024;      // and its workgroup size

struct Counters {
    uint32_t ncand;        // candidates of the sub-round
    uint32_t nslow;        // candidates aimed at targets that cannot take them all
    int32_t gmin;          // gain range of those candidates
    int32_t gmax;
    uint32_t bad_color;
    uint32_t nseg;         // targets that cannot take all their candidates
    uint32_t slow_total;   // entries reserved in their segments
    uint32_t unused;
    uint32_t nlarge;       // segments longer than kSmallSeg
    uint32_t nlchunks;     // kSegChunk-entry chunks of those segments
    int32_t gkey;          // gmax of the sub-round's keys, kept past the counter reset
    uint32_t pad;
};

struct EvalArgs {
    const int64_t* xadj;
    const int32_t* adj;
    int64_t S;  // slots of the graph (bound of the vector loads of short rows)
    const int32_t* ew;
    const int32_t* vw;
    const int32_t* label;
    // Narrow copies of label for the neighbour gathers when every label fits
    // 8 or 16 bits (refinement: blocks): a cache line then holds 4 or 2
    // times as many neighbours' labels.  Null when not kept.
    const uint8_t* label8;
    const uint16_t* label16;
    const int32_t* w;
    int64_t bound;
    uint64_t tp;  // H(seed, 2, level, phase, round)
    int32_t refine;
    // several graphs in one launch; gid == null: one graph, the scalars above
    const int32_t* gid;      // [n] graph of each node
    const uint64_t* g_tp;    // [G] tie prefix of each graph for this round
    const int64_t* g_bound;  // [G] bound of each graph's labels
    const int32_t* g_lbase;  // [G] first label of each graph
    // Quiet nodes: evaluated with no neighbouring label connected more strongly
    // than their own, not overloaded, and no neighbour has moved since.  Such a
    // node emits nothing while it stays quiet and its block is not overloaded
    // (its connections are unchanged), so it need not be evaluated again.
    uint8_t* quiet;     // [n] flags (null: not tracked); see quiet_mode()
    const uint32_t* rcnt;  // candidates of each round so far (device)
    int32_t round;         // this round
    int32_t quiet_n;       // nodes of the graph (the tracking threshold is 1/8 of them)
    int32_t dense_k;    // > 0: every node's labels are lbase + [0, dense_k) (refinement blocks)
    // the previous round's candidate count (null in the first round): after a
    // round without candidates the state is a fixed point and the evaluation
    // of the later rounds is skipped
    const uint32_t* gate;
    const int32_t* nodes;  // schedule entries of this launch
    int32_t count;
    int32_t* ct;  // per entry: target label or -1
    int32_t* cg;  // per entry: gain
};

// A round runs only while the previous one had candidates (gate: that
// round's candidate count, null for the first round).  Rounds are enqueued
// before the previous round's count is known (ahead of the host, or all of
// a level's rounds at once in a captured graph), so every kernel checks the
// gate: after a round without candidates the following ones do nothing.
__device__ __forceinline__ bool stopped(const uint32_t* gate) { return gate && *gate == 0; }

// Quiet-node tracking: marks are written from two rounds after the first
// round with at most n/8 candidates on, and used to skip nodes one round
// later (1: mark, 2: mark and skip, 0: off).  Derived from the per-round
// candidate counts on the device, so it needs no host decision per round.
__device__ __forceinline__ int quiet_mode(const uint8_t* quiet, const uint32_t* rcnt, int32_t round, int32_t n) {
    if (!quiet) return 0;
    for (int32_t q = 0; q + 2 <= round; ++q)
        if (static_cast<int64_t>(rcnt[q]) * 8 <= n) return q + 2 < round ? 2 : 1;
    return 0;
}

__device__ __forceinline__ int quiet_mode(const EvalArgs& A) { return quiet_mode(A.quiet, A.rcnt, A.round, A.quiet_n); }

// ------------------------------------------------------- selection helpers

__device__ __forceinline__ int32_t nbr_label(const EvalArgs& A, int32_t u) {
    if (A.label8) return A.label8[u];
    if (A.label16) return A.label16[u];
    return A.label[u];
}

// Per-node constants: the tie prefix and bound of the node's graph and the
// graph's first label (ties hash graph-local label ids).
struct Ctx {
    uint64_t tp;
    int64_t bound;
    int32_t lbase;
};

__device__ __forceinline__ Ctx ctx_of(const EvalArgs& A, int32_t v) {
    if (A.gid) {
        const int32_t g = A.gid[v];
        return Ctx{A.g_tp[g], A.g_bound[g], A.g_lbase[g]};
    }
    return Ctx{A.tp, A.bound, 0};
}

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

__device__ __forceinline__ uint64_t tie_of(const Ctx& kx, int32_t x) {
    return mix64(kx.tp ^ static_cast<uint64_t>(static_cast<uint32_t>(x - kx.lbase)));
}

__device__ __forceinline__ void best_consider(Best& b, int32_t x, int32_t conn, const Ctx& kx) {
    if (b.x < 0 || conn > b.conn) {
        b.conn = conn;
        b.x = x;
        b.tv = false;
        return;
    }
    if (conn < b.conn) return;
    const uint64_t tx = tie_of(kx, x);
    if (!b.tv) {
        b.tie = tie_of(kx, b.x);
        b.tv = true;
    }
    if (tx < b.tie || (tx == b.tie && x < b.x)) {
        b.x = x;
        b.tie = tx;
    }
}

__device__ __forceinline__ uint64_t best_tie(const Best& b, const Ctx& kx) { return b.tv ? b.tie : tie_of(kx, b.x); }

// Wave-wide argmax; every lane gets the winning (x, conn) or x = -1.
__device__ __forceinline__ void wave_argmax(const Best& b, const Ctx& kx, int32_t& out_x, int32_t& out_conn) {
    const int32_t bc = b.x >= 0 ? b.conn : -1;
    const int32_t maxc = wave_max(bc);
    if (maxc < 0) {
        out_x = -1;
        out_conn = -1;
        return;
    }
    const bool top = b.x >= 0 && bc == maxc;
    const uint64_t tk = top ? best_tie(b, kx) : ~0ULL;
    const uint64_t mt = wave_min_u64(tk);
    const int32_t xx = (top && tk == mt) ? b.x : INT_MAX;
    out_x = wave_min(xx);
    out_conn = maxc;
}

// Reductions over aligned groups of G lanes of a wave (G a power of two <= 64).
template <int G>
__device__ __forceinline__ int32_t group_max(int32_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ int32_t group_min(int32_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ uint64_t group_min_u64(uint64_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), o, 64);
        const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), o, 64);
        const uint64_t u = (static_cast<uint64_t>(hi) << 32) | lo;
        v = u < v ? u : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ bool group_any(bool b) {
    const uint64_t m = __ballot(b);
    if (G == 64) return m != 0;
    const int base = lane_id() & ~(G - 1);
    return ((m >> base) & ((1ULL << G) - 1)) != 0;
}

// Group-wide argmax; every lane of the group gets the winning (x, conn).
template <int G>
__device__ __forceinline__ void group_argmax(const Best& b, const Ctx& kx, int32_t& out_x, int32_t& out_conn) {
    const int32_t bc = b.x >= 0 ? b.conn : -1;
    const int32_t maxc = group_max<G>(bc);
    if (maxc < 0) {
        out_x = -1;
        out_conn = -1;
        return;
    }
    const bool top = b.x >= 0 && bc == maxc;
    const uint64_t tk = top ? best_tie(b, kx) : ~0ULL;
    const uint64_t mt = group_min_u64<G>(tk);
    const int32_t xx = (top && tk == mt) ? b.x : INT_MAX;
    out_x = group_min<G>(xx);
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

__device__ __forceinline__ bool eligible(const EvalArgs& A, int32_t x, int32_t c, const Ctx& kx) {
    return static_cast<int64_t>(A.w[x]) + c <= kx.bound;
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

// True if v is quiet and may skip evaluation (its block is not overloaded).
__device__ __forceinline__ bool skip_quiet(const EvalArgs& A, int qm, int32_t v, const Ctx& kx) {
    if (qm < 2 || !A.quiet[v]) return false;
    return !A.refine || A.w[A.label[v]] <= kx.bound;
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

// The same for a table of any size tsz: the first probe is the hash scaled
// to [0, tsz), and probing wraps at tsz.
__device__ __forceinline__ void table_add_sized(int32_t* keys, int32_t* vals, uint32_t tsz, int32_t x, int32_t wt) {
    uint32_t h = static_cast<uint32_t>((static_cast<uint64_t>(slot_hash(static_cast<uint32_t>(x))) * tsz) >> 32);
    while (true) {
        const int32_t prev = atomicCAS(&keys[h], -1, x);
        if (prev == -1 || prev == x) {
            atomicAdd(&vals[h], wt);
            return;
        }
        h = h + 1 == tsz ? 0u : h + 1;
    }
}

// Adds the slots [b, b+d) of a row to a table of tsz entries; each thread
// keeps U gathers in flight before inserting.  kPow2: tsz is a power of two
// (masked probes), else any size (table_add_sized).
template <int NT, int U, bool kPow2 = true>
__device__ __forceinline__ void insert_slots(const EvalArgs& A, int64_t b, int32_t d, int32_t* keys, int32_t* vals,
                                             uint32_t tsz, int tid) {
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
            x[u] = j < d ? nbr_label(A, x[u]) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (x[u] < 0) continue;
            if (kPow2) table_add(keys, vals, tsz - 1, x[u], wt[u]);
            else table_add_sized(keys, vals, tsz, x[u], wt[u]);
        }
    }
}

// ------------------------------------------------------------ lane bucket

// A short row's neighbour ids and weights, then the neighbours' labels.
// The row is read with 16-byte loads from the aligned address at or below
// its start when the aligned window lies inside the arrays (one lane per
// row: a wave's scalar loads each touch 64 rows, so fewer, wider loads
// spend less of the load unit's time); -1 and 0 past the row's end.
template <int MAXD>
__device__ __forceinline__ void lane_words(const int32_t* base, int64_t b, int d, int64_t S, int32_t* out, bool& vec) {
    constexpr int NQ = MAXD / 4 + 1;
    const int off = static_cast<int>((reinterpret_cast<uintptr_t>(base + b) & 15u) >> 2);
    const int64_t b0 = b - off;
    const int nq = (off + d + 3) >> 2;
    vec = b0 >= 0 && b0 + 4 * static_cast<int64_t>(nq) <= S;
    if (!vec) return;
    int32_t r[4 * NQ];
    const int4* q = reinterpret_cast<const int4*>(base + b0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        int4 w = make_int4(0, 0, 0, 0);
        if (k < nq) w = q[k];
        r[4 * k] = w.x;
        r[4 * k + 1] = w.y;
        r[4 * k + 2] = w.z;
        r[4 * k + 3] = w.w;
    }
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        const int32_t x0 = r[j], x1 = r[j + 1], x2 = r[j + 2], x3 = r[j + 3];
        out[j] = off == 0 ? x0 : off == 1 ? x1 : off == 2 ? x2 : x3;
    }
}

template <int MAXD>
__device__ __forceinline__ void lane_row(const EvalArgs& A, int64_t b, int d, int32_t* lab, int32_t* wt) {
    bool vec;
    lane_words<MAXD>(A.adj, b, d, A.S, lab, vec);
    if (vec) {
        if (A.ew) {
            bool vec_w;
            lane_words<MAXD>(A.ew, b, d, A.S, wt, vec_w);
            if (!vec_w)
#pragma unroll
                for (int j = 0; j < MAXD; ++j) wt[j] = j < d ? A.ew[b + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < MAXD; ++j) {
            lab[j] = j < d ? nbr_label(A, lab[j]) : -1;
            if (!A.ew) wt[j] = j < d ? 1 : 0;
            else if (j >= d) wt[j] = 0;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        if (j < d) {
            lab[j] = nbr_label(A, A.adj[b + j]);
            wt[j] = A.ew ? A.ew[b + j] : 1;
        } else {
            lab[j] = -1;
            wt[j] = 0;
        }
    }
}

template <int MAXD>
__device__ __forceinline__ void eval_lane_body(const EvalArgs& A, int32_t bid) {
    const int i = bid * 256 + threadIdx.x;
    if (i >= A.count || stopped(A.gate)) return;
    const int qm = quiet_mode(A);
    const int32_t v = A.nodes[i];
    const Ctx kx = ctx_of(A, v);
    if (skip_quiet(A, qm, v, kx)) {
        store_result(A, i, -1, 0, 0, false);
        return;
    }
    const int64_t b = A.xadj[v];
    const int d = static_cast<int>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    int32_t lab[MAXD], wt[MAXD];
    lane_row<MAXD>(A, b, d, lab, wt);
    int32_t own = 0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j) own += (lab[j] == a) ? wt[j] : 0;
    const bool over = A.refine && A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;  // some other neighbouring label is connected more strongly
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
        blocked |= conn > own;
        if (!over && conn <= own) continue;  // cannot give a positive gain
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, conn, kx);
    }
    store_result(A, i, best.x, best.conn, own, over);
    if (qm) A.quiet[v] = (!over && !blocked) ? 1 : 0;
}

template <int MAXD>
__global__ void __launch_bounds__(256) eval_lane_kernel(EvalArgs A) {
    eval_lane_body<MAXD>(A, blockIdx.x);
}

// --------------------------------------------------- group and wave buckets

// G lanes per node (G = 16, 32 or 64: 256 / G nodes per workgroup), each
// group with an open-addressing table of T entries in LDS.
// LDS: 2 * (256 / G) * T int32 (the groups' key tables, then their sums).
template <int G, int T>
__device__ __forceinline__ void eval_group_body(const EvalArgs& A, int32_t bid, int32_t* lds) {
    constexpr int NG = 256 / G;
    const int grp = threadIdx.x / G;
    const int gl = threadIdx.x % G;
    const int node_i = bid * NG + grp;
    if (node_i >= A.count || stopped(A.gate)) return;  // uniform per group
    const int qm = quiet_mode(A);
    int32_t* keys = lds + grp * T;
    int32_t* vals = lds + (NG + grp) * T;
    const int32_t v = A.nodes[node_i];
    const Ctx kx = ctx_of(A, v);
    if (skip_quiet(A, qm, v, kx)) {
        if (gl == 0) store_result(A, node_i, -1, 0, 0, false);
        return;
    }
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    const uint32_t tsz = table_size_for(d, T < 64 ? T : 64, T);
    for (uint32_t j = gl; j < tsz; j += G) {
        keys[j] = -1;
        vals[j] = 0;
    }
    wave_sync();
    insert_slots<G, 4>(A, b, d, keys, vals, tsz, gl);
    wave_sync();
    int32_t ownp = 0;
    for (uint32_t j = gl; j < tsz; j += G)
        if (keys[j] == a) ownp = vals[j];
    const int32_t own = group_max<G>(ownp);
    const bool over = A.refine && A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;  // some other neighbouring label is connected more strongly
    for (uint32_t j = gl; j < tsz; j += G) {
        const int32_t x = keys[j];
        if (x < 0 || x == a) continue;
        const int32_t conn = vals[j];
        blocked |= conn > own;
        if (!over && conn <= own) continue;
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, conn, kx);
    }
    int32_t bx, bconn;
    group_argmax<G>(best, kx, bx, bconn);
    const bool any_blocked = group_any<G>(blocked);
    if (gl == 0) {
        store_result(A, node_i, bx, bconn, own, over);
        if (qm) A.quiet[v] = (!over && !any_blocked) ? 1 : 0;
    }
}

template <int G, int T>
__global__ void __launch_bounds__(256) eval_group_kernel(EvalArgs A) {
    __shared__ int32_t lds[2 * (256 / G) * T];
    eval_group_body<G, T>(A, blockIdx.x, lds);
}

// ----------------------------------------------------------- block bucket

// LDS of the block bodies: per-wave winners (tie keys, labels, sums) then
// the body's table.
template <int NT>
struct BlockScratch {
    uint64_t tie[NT / 64];
    int32_t conn[NT / 64];
    int32_t x[NT / 64];
    int32_t own;
    int32_t pad;
};

// LDS: BlockScratch<NT> then 2 * TABLE int32 (keys, then sums).
template <int NT, int TABLE>
__device__ __forceinline__ void eval_block_body(const EvalArgs& A, int32_t bid, unsigned char* lds) {
    BlockScratch<NT>& S = *reinterpret_cast<BlockScratch<NT>*>(lds);
    int32_t* keys = reinterpret_cast<int32_t*>(lds + sizeof(BlockScratch<NT>));
    int32_t* vals = keys + TABLE;
    int32_t& s_own = S.own;
    int32_t* s_conn = S.conn;
    int32_t* s_x = S.x;
    uint64_t* s_tie = S.tie;
    const int tid = threadIdx.x;
    const int wid = tid >> 6;
    const int lane = lane_id();
    if (stopped(A.gate)) return;  // uniform over the grid
    const int qm = quiet_mode(A);
    const int32_t v = A.nodes[bid];
    const Ctx kx = ctx_of(A, v);
    if (skip_quiet(A, qm, v, kx)) {  // uniform over the workgroup
        if (tid == 0) store_result(A, bid, -1, 0, 0, false);
        return;
    }
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    constexpr bool kPow2 = (TABLE & (TABLE - 1)) == 0;
    const uint32_t tsz = kPow2 ? table_size_for(d, 512, TABLE) : static_cast<uint32_t>(TABLE);
    for (uint32_t j = tid; j < tsz; j += NT) {
        keys[j] = -1;
        vals[j] = 0;
    }
    if (tid == 0) s_own = 0;
    __syncthreads();
    insert_slots<NT, 4, kPow2>(A, b, d, keys, vals, tsz, tid);
    __syncthreads();
    for (uint32_t j = tid; j < tsz; j += NT)
        if (keys[j] == a) s_own = vals[j];
    __syncthreads();
    const int32_t own = s_own;
    const bool over = A.refine && A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;
    for (uint32_t j = tid; j < tsz; j += NT) {
        const int32_t x = keys[j];
        if (x < 0 || x == a) continue;
        const int32_t conn = vals[j];
        blocked |= conn > own;
        if (!over && conn <= own) continue;
        if (best.x >= 0 && conn < best.conn) continue;
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, conn, kx);
    }
    int32_t bx, bconn;
    wave_argmax(best, kx, bx, bconn);
    if (lane == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(kx, bx) : ~0ULL;
    }
    const int any_blocked = __syncthreads_or(blocked);
    if (tid == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < NT / 64; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        store_result(A, bid, fx, fc, own, over);
        if (qm) A.quiet[v] = (!over && !any_blocked) ? 1 : 0;
    }
}

template <int NT, int TABLE>
__global__ void __launch_bounds__(NT) eval_block_kernel(EvalArgs A) {
    __shared__ __align__(16) unsigned char lds[sizeof(BlockScratch<NT>) + 2 * TABLE * sizeof(int32_t)];
    eval_block_body<NT, TABLE>(A, blockIdx.x, lds);
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
constexpr int kPartTable = 4096;  // 32 KB LDS table of a partition workgroup (four per CU)
constexpr int kMaxPartLog = 11;   // at most 2048 partitions per hub

__device__ __forceinline__ uint32_t part_of(int32_t x, int32_t plog) {
    return plog == 0 ? 0u : (slot_hash(static_cast<uint32_t>(x)) >> (32 - plog));
}

// Sums one chunk of a hub row in an LDS table, then scatters the chunk's
// distinct (label, weight) entries into the hub's label partitions.
__global__ void __launch_bounds__(kHubThreads) hub_chunk_kernel(EvalArgs A, HubArgs H) {
    __shared__ int32_t keys[kHubTable];
    __shared__ int32_t vals[kHubTable];
    __shared__ uint32_t pcount[1 << kMaxPartLog];
    __shared__ int32_t pbase[1 << kMaxPartLog];
    constexpr int kPer = kHubTable / kHubThreads;
    if (stopped(A.gate)) return;  // uniform over the grid
    const int tid = threadIdx.x;
    const int32_t h = H.chunk_hub[blockIdx.x];
    const int32_t v = H.hub_nodes[h];
    const int64_t begin = H.chunk_begin[blockIdx.x];
    const int64_t row_end = A.xadj[v + 1];
    const int64_t end = begin + kHubChunk < row_end ? begin + kHubChunk : row_end;
    const uint32_t tsz = table_size_for(static_cast<int32_t>(end - begin), 1024, kHubTable);
    const int32_t plog = H.hub_plog[h];
    const int32_t P = 1 << plog;
    for (uint32_t j = tid; j < tsz; j += kHubThreads) {
        keys[j] = -1;
        vals[j] = 0;
    }
    for (int32_t j = tid; j < P; j += kHubThreads) pcount[j] = 0;
    __syncthreads();
    insert_slots<kHubThreads, 4>(A, begin, static_cast<int32_t>(end - begin), keys, vals, tsz, tid);
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
    if (stopped(A.gate)) return;  // uniform over the grid
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
    const Ctx kx = ctx_of(A, v);
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
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, conn, kx);
    }
    int32_t bx, bconn;
    wave_argmax(best, kx, bx, bconn);
    const int wid = tid >> 6;
    if (lane_id() == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(kx, bx) : ~0ULL;
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
    const Ctx kx = ctx_of(A, v);
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
    const bool over = A.refine && A.w[a] > kx.bound;
    if (lane_id() == 0) store_result(A, h, bx, maxc, H.hub_own[h], over);
}

__global__ void __launch_bounds__(64) hub_finish_kernel(EvalArgs A, HubArgs H) {
    if (stopped(A.gate) || H.big[blockIdx.x]) return;
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
    if (stopped(A.gate) || !H.big[h]) return;
    const int32_t v = H.hub_nodes[h];
    const Ctx kx = ctx_of(A, v);
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
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, conn, kx);
    }
    int32_t bx, bconn;
    wave_argmax(best, kx, bx, bconn);
    const int wid = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(kx, bx) : ~0ULL;
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
    if (stopped(A.gate) || !H.big[blockIdx.x]) return;
    hub_decide(A, H, blockIdx.x, tfirst_shifted);
}

// ------------------------------------------------ dense refinement buckets
//
// During refinement a node's labels are its graph's blocks, so connections
// are summed in a dense array of dense_k entries (one LDS atomic add per
// slot, no probing) instead of a hash table.

constexpr int kDenseMax = 256;

// Adds the slots [b, b+d) of a row to conn with LDS atomics (STRIDE lanes,
// U batches of loads in flight).
template <int STRIDE>
__device__ __forceinline__ void dense_slots(const EvalArgs& A, const Ctx& kx, int64_t b, int32_t d, int32_t* conn,
                                            int lane_in_set) {
    constexpr int U = 4;
    for (int32_t j0 = lane_in_set; j0 < d; j0 += STRIDE * U) {
        int32_t x[U], wt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t j = j0 + u * STRIDE;
            x[u] = j < d ? A.adj[b + j] : -1;
            wt[u] = j < d ? (A.ew ? A.ew[b + j] : 1) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = x[u] >= 0 ? nbr_label(A, x[u]) - kx.lbase : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (x[u] >= 0) atomicAdd(&conn[x[u]], wt[u]);
    }
}

// Best eligible block of a node from its dense connections (lane j of the
// set scans entries j, j + NT, ...).
__device__ __forceinline__ void dense_best(const EvalArgs& A, const Ctx& kx, const int32_t* conn, int32_t a,
                                           int32_t c, int32_t own, bool over, int first, int step, Best& best,
                                           bool& blocked) {
    const int32_t la = a - kx.lbase;
    for (int32_t j = first; j < A.dense_k; j += step) {
        const int32_t cn = conn[j];
        if (cn == 0 || j == la) continue;  // not a neighbouring block, or the own one
        blocked |= cn > own;
        if (!over && cn <= own) continue;
        if (best.x >= 0 && cn < best.conn) continue;
        const int32_t x = j + kx.lbase;
        if (!eligible(A, x, c, kx)) continue;
        best_consider(best, x, cn, kx);
    }
}

// LDS: (256 / G) * kDenseMax int32 (each group's block sums).
template <int G>
__device__ __forceinline__ void eval_dense_group_body(const EvalArgs& A, int32_t bid, int32_t* lds) {
    constexpr int NG = 256 / G;
    const int grp = threadIdx.x / G;
    const int gl = threadIdx.x % G;
    const int node_i = bid * NG + grp;
    if (node_i >= A.count || stopped(A.gate)) return;  // uniform per group
    const int qm = quiet_mode(A);
    int32_t* conn = lds + grp * kDenseMax;
    const int32_t v = A.nodes[node_i];
    const Ctx kx = ctx_of(A, v);
    if (skip_quiet(A, qm, v, kx)) {
        if (gl == 0) store_result(A, node_i, -1, 0, 0, false);
        return;
    }
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    for (int32_t j = gl; j < A.dense_k; j += G) conn[j] = 0;
    wave_sync();
    dense_slots<G>(A, kx, b, d, conn, gl);
    wave_sync();
    const int32_t own = conn[a - kx.lbase];
    const bool over = A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;
    dense_best(A, kx, conn, a, c, own, over, gl, G, best, blocked);
    int32_t bx, bconn;
    group_argmax<G>(best, kx, bx, bconn);
    const bool any_blocked = group_any<G>(blocked);
    if (gl == 0) {
        store_result(A, node_i, bx, bconn, own, over);
        if (qm) A.quiet[v] = (!over && !any_blocked) ? 1 : 0;
    }
}

template <int G>
__global__ void __launch_bounds__(256) eval_dense_group_kernel(EvalArgs A) {
    __shared__ int32_t lds[(256 / G) * kDenseMax];
    eval_dense_group_body<G>(A, blockIdx.x, lds);
}

// LDS: BlockScratch<NT> then kDenseMax int32 (the node's block sums).
template <int NT>
__device__ __forceinline__ void eval_dense_block_body(const EvalArgs& A, int32_t bid, unsigned char* lds) {
    BlockScratch<NT>& S = *reinterpret_cast<BlockScratch<NT>*>(lds);
    int32_t* conn = reinterpret_cast<int32_t*>(lds + sizeof(BlockScratch<NT>));
    int32_t* s_conn = S.conn;
    int32_t* s_x = S.x;
    uint64_t* s_tie = S.tie;
    const int tid = threadIdx.x;
    const int wid = tid >> 6;
    if (stopped(A.gate)) return;  // uniform over the grid
    const int qm = quiet_mode(A);
    const int32_t v = A.nodes[bid];
    const Ctx kx = ctx_of(A, v);
    if (skip_quiet(A, qm, v, kx)) {  // uniform over the workgroup
        if (tid == 0) store_result(A, bid, -1, 0, 0, false);
        return;
    }
    const int64_t b = A.xadj[v];
    const int32_t d = static_cast<int32_t>(A.xadj[v + 1] - b);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    for (int32_t j = tid; j < A.dense_k; j += NT) conn[j] = 0;
    __syncthreads();
    dense_slots<NT>(A, kx, b, d, conn, tid);
    __syncthreads();
    const int32_t own = conn[a - kx.lbase];
    const bool over = A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;
    dense_best(A, kx, conn, a, c, own, over, tid, NT, best, blocked);
    int32_t bx, bconn;
    wave_argmax(best, kx, bx, bconn);
    if (lane_id() == 0) {
        s_conn[wid] = bconn;
        s_x[wid] = bx;
        s_tie[wid] = bx >= 0 ? tie_of(kx, bx) : ~0ULL;
    }
    const int any_blocked = __syncthreads_or(blocked);
    if (tid == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < NT / 64; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        store_result(A, bid, fx, fc, own, over);
        if (qm) A.quiet[v] = (!over && !any_blocked) ? 1 : 0;
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) eval_dense_block_kernel(EvalArgs A) {
    __shared__ __align__(16) unsigned char lds[sizeof(BlockScratch<NT>) + kDenseMax * sizeof(int32_t)];
    eval_dense_block_body<NT>(A, blockIdx.x, lds);
}

// ------------------------------------------------- small buckets, fused

// The buckets of up to 1 024 slots (one lane, 16, 32 or 64 lanes, or one
// 256-thread workgroup per node) of a small colour in one launch: consecutive
// workgroup ranges belong to the buckets in order, and each workgroup runs its
// bucket's body on an LDS buffer sized for the largest.  A small colour
// otherwise pays one launch per bucket on one stream.
constexpr int kFusedBuckets = 6;

struct FusedBuckets {
    const int32_t* nodes[kFusedBuckets];
    int32_t* ct[kFusedBuckets];
    int32_t* cg[kFusedBuckets];
    int32_t count[kFusedBuckets];
    int32_t first[kFusedBuckets + 1];  // first workgroup of each bucket, then the total
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kFusedLds =
    cmax(cmax(2 * 16 * (2 * kG16Max) * sizeof(int32_t), 2 * 8 * (2 * kG32Max) * sizeof(int32_t)),
         cmax(cmax(2 * 4 * kWaveTable * sizeof(int32_t), sizeof(BlockScratch<256>) + 2 * (2 * kBlock1Max) * sizeof(int32_t)),
              cmax(16 * kDenseMax * sizeof(int32_t), sizeof(BlockScratch<256>) + kDenseMax * sizeof(int32_t))));

template <bool kDense>
__global__ void __launch_bounds__(256) eval_fused_kernel(EvalArgs A, FusedBuckets F) {
    __shared__ __align__(16) unsigned char lds[kFusedLds];
    int b = 0;
    while (b + 1 < kFusedBuckets && static_cast<int32_t>(blockIdx.x) >= F.first[b + 1]) ++b;
    const int32_t bid = static_cast<int32_t>(blockIdx.x) - F.first[b];
    A.nodes = F.nodes[b];
    A.count = F.count[b];
    A.ct = F.ct[b];
    A.cg = F.cg[b];
    int32_t* l32 = reinterpret_cast<int32_t*>(lds);
    switch (b) {  // uniform over the workgroup
        case 0:
            eval_lane_body<kLaneSmall>(A, bid);
            break;
        case 1:
            eval_lane_body<kLaneMax>(A, bid);
            break;
        case 2:
            if (kDense) eval_dense_group_body<16>(A, bid, l32);
            else eval_group_body<16, 2 * kG16Max>(A, bid, l32);
            break;
        case 3:
            if (kDense) eval_dense_group_body<32>(A, bid, l32);
            else eval_group_body<32, 2 * kG32Max>(A, bid, l32);
            break;
        case 4:
            if (kDense) eval_dense_group_body<64>(A, bid, l32);
            else eval_group_body<64, kWaveTable>(A, bid, l32);
            break;
        default:
            if (kDense) eval_dense_block_body<256>(A, bid, lds);
            else eval_block_body<256, 2 * kBlock1Max>(A, bid, lds);
            break;
    }
}

// Hubs: every chunk of a hub's row adds its dense sums to the hub's row of
// hub_sum (dense_k entries per hub) ...
__global__ void __launch_bounds__(kHubThreads) hub_dense_chunk_kernel(EvalArgs A, HubArgs H,
                                                                      int32_t* __restrict__ hub_sum) {
    __shared__ int32_t conn[kDenseMax];
    if (stopped(A.gate)) return;  // uniform over the grid
    const int tid = threadIdx.x;
    const int32_t h = H.chunk_hub[blockIdx.x];
    const int32_t v = H.hub_nodes[h];
    const Ctx kx = ctx_of(A, v);
    const int64_t begin = H.chunk_begin[blockIdx.x];
    const int64_t row_end = A.xadj[v + 1];
    const int64_t end = begin + kHubDenseChunk < row_end ? begin + kHubDenseChunk : row_end;
    for (int32_t j = tid; j < A.dense_k; j += kHubThreads) conn[j] = 0;
    __syncthreads();
    dense_slots<kHubThreads>(A, kx, begin, static_cast<int32_t>(end - begin), conn, tid);
    __syncthreads();
    for (int32_t j = tid; j < A.dense_k; j += kHubThreads)
        if (conn[j]) atomicAdd(&hub_sum[static_cast<int64_t>(h) * A.dense_k + j], conn[j]);
}

// ... then one workgroup per hub decides and clears the hub's row.
__global__ void __launch_bounds__(256) hub_dense_finish_kernel(EvalArgs A, HubArgs H, int32_t* __restrict__ hub_sum) {
    __shared__ int32_t s_conn[4];
    __shared__ int32_t s_x[4];
    __shared__ uint64_t s_tie[4];
    if (stopped(A.gate)) return;  // uniform over the grid
    const int tid = threadIdx.x;
    const int32_t h = blockIdx.x;
    const int32_t v = H.hub_nodes[h];
    const Ctx kx = ctx_of(A, v);
    const int32_t a = A.label[v];
    const int32_t c = A.vw ? A.vw[v] : 1;
    int32_t* conn = hub_sum + static_cast<int64_t>(h) * A.dense_k;
    const int32_t own = conn[a - kx.lbase];
    const bool over = A.w[a] > kx.bound;
    Best best;
    best_init(best);
    bool blocked = false;
    dense_best(A, kx, conn, a, c, own, over, tid, 256, best, blocked);
    int32_t bx, bconn;
    wave_argmax(best, kx, bx, bconn);
    if (lane_id() == 0) {
        s_conn[tid >> 6] = bconn;
        s_x[tid >> 6] = bx;
        s_tie[tid >> 6] = bx >= 0 ? tie_of(kx, bx) : ~0ULL;
    }
    __syncthreads();
    for (int32_t j = tid; j < A.dense_k; j += 256) conn[j] = 0;
    if (tid == 0) {
        int32_t fc = -1, fx = -1;
        uint64_t ft = ~0ULL;
        for (int w = 0; w < 4; ++w) combine_into(fc, ft, fx, s_conn[w], s_tie[w], s_x[w]);
        store_result(A, h, fx, fc, own, over);
    }
}

// ------------------------------------------------------- block utilities

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

// Bound of a target label: one scalar, or per graph through the label's graph.
struct Bounds {
    int64_t bound;
    const int32_t* lgid;     // [nw] graph of each label, or null
    const int64_t* g_bound;  // [G]
};

__device__ __forceinline__ int64_t bound_of(const Bounds& B, int32_t t) {
    return B.lgid ? B.g_bound[B.lgid[t]] : B.bound;
}

// Block-local LDS index of label t: t itself for small label spaces, else an
// open-addressing slot (kAggTable entries, at most kAggChunk keys per chunk,
// so the table is never more than half full).
constexpr int kAggChunk = 2048;
constexpr int kAggTable = 4096;


template <bool kSmall>
__device__ __forceinline__ int32_t agg_slot(int32_t* keys, int32_t t, bool insert) {
    if (kSmall) return t;
    uint32_t h = slot_hash(static_cast<uint32_t>(t)) & (kAggTable - 1);
    while (true) {
        const int32_t k = insert ? atomicCAS(&keys[h], -1, t) : keys[h];
        if (k == t || (insert && k == -1)) return static_cast<int32_t>(h);
        h = (h + 1) & (kAggTable - 1);
    }
}

// tsum[t] += c(v) and cnt[t] += 1 over the candidates of the sub-round, summed
// per block in LDS first so that a label many nodes aim at (a hub's cluster)
// costs one global atomic per block and chunk, not one per candidate.
template <bool kSmall, int R>
__global__ void __launch_bounds__(256) cand_accum_kernel(const int32_t* __restrict__ ct,
                                                         const int32_t* __restrict__ nodes, int32_t count,
                                                         const int32_t* __restrict__ vw, int32_t* __restrict__ tsum,
                                                         int32_t* __restrict__ cnt, int32_t nw, Counters* ctr,
                                                         const uint32_t* __restrict__ gate,
                                                         uint32_t* __restrict__ round_cnt) {
    if (stopped(gate)) return;  // uniform over the grid
    constexpr int kSlots = kSmall ? kSmallLabels : kAggTable;
    __shared__ int32_t keys[kSmall ? 1 : kAggTable];
    __shared__ int32_t lsum[kSlots];
    __shared__ int32_t lcnt[kSlots];
    const int32_t nslots = kSmall ? nw : kAggTable;
    for (int j = threadIdx.x; j < nslots; j += 256) {
        if (!kSmall) keys[j] = -1;
        lsum[j] = 0;
        lcnt[j] = 0;
    }
    __syncthreads();
    int32_t found = 0;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * (R * 256); base < count;
         base += static_cast<int64_t>(gridDim.x) * (R * 256)) {
        // all of the thread's loads of the chunk first, then the LDS updates
        int32_t tr[R], cr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t p = base + r * 256 + threadIdx.x;
            tr[r] = p < count ? ct[p] : -1;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t p = base + r * 256 + threadIdx.x;
            cr[r] = tr[r] >= 0 ? (vw ? vw[nodes[p]] : 1) : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (tr[r] < 0) continue;
            ++found;
            const int32_t i = agg_slot<kSmall>(keys, tr[r], true);
            if (cr[r]) atomicAdd(&lsum[i], cr[r]);
            atomicAdd(&lcnt[i], 1);
        }
        if (!kSmall) {  // flush this chunk's labels
            __syncthreads();
            for (int j = threadIdx.x; j < kAggTable; j += 256) {
                const int32_t t = keys[j];
                if (t >= 0) {
                    if (lsum[j]) atomicAdd(&tsum[t], lsum[j]);
                    atomicAdd(&cnt[t], lcnt[j]);
                    keys[j] = -1;
                    lsum[j] = 0;
                    lcnt[j] = 0;
                }
            }
            __syncthreads();
        }
    }
    if (kSmall) {
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256) {
            if (lsum[j]) atomicAdd(&tsum[j], lsum[j]);
            if (lcnt[j]) atomicAdd(&cnt[j], lcnt[j]);
        }
    }
    const int32_t tot = block_sum_i32(found);
    if (threadIdx.x == 0 && tot) {
        atomicAdd(&ctr->ncand, static_cast<uint32_t>(tot));
        atomicAdd(round_cnt, static_cast<uint32_t>(tot));
    }
}

// ------------------------------------------------------------- admission
//
// Outcome of a candidate in ok[p]: 0 not a candidate (or rejected), 1
// admitted, kOkSlow aimed at a target that cannot take all its candidates.
// The apply kernel decides those from the target's boundary key bnd[t]: a
// candidate is admitted when its key [gmax - gain][node] is below it.
constexpr uint8_t kOkSlow = 2;

// Multi-workgroup selection for segments longer than the single-workgroup
// limit: the same most-significant-digit-first selection with kLDigit-bit
// digits and per-segment histograms in HBM. A segment is registered when its
// target claims it: it takes the next large index l and a run of
// kSegChunk-entry chunks.
constexpr int kLDigit = 12;
constexpr int kLBins = 1 << kLDigit;

struct LargeSel {
    int32_t* target;    // [nlarge] target of each large segment
    int32_t* base;      // [nlarge] its first entry
    int32_t* len;       // [nlarge] its entries
    int32_t* chunk0;    // [nlarge] its first chunk
    int32_t* owner;     // [nlchunks] large segment of each chunk
    uint32_t* hist;     // [nlarge][kLBins] weight per digit
    uint64_t* prefix;   // [nlarge] digits fixed so far
    int64_t* room;      // [nlarge] weight still admissible below the prefix
    uint32_t* done;     // [nlarge] chunks finished with the current digit
};

__device__ __forceinline__ int32_t seg_chunks(int32_t len) { return (len + kSegChunk - 1) / kSegChunk; }

// Gives target t (room = bound - w(t)) a segment of cnt[t] entries, and a
// large index when that is longer than small_max.
__device__ void claim_segment(int32_t t, int32_t len, int64_t room, int32_t* seg_off, int32_t* seg_list,
                              const LargeSel& L, int32_t small_max, Counters* ctr) {
    const int32_t base = static_cast<int32_t>(atomicAdd(&ctr->slow_total, static_cast<uint32_t>(len)));
    seg_off[t] = base;
    seg_list[atomicAdd(&ctr->nseg, 1u)] = t;
    if (len <= small_max) return;
    const uint32_t l = atomicAdd(&ctr->nlarge, 1u);
    const int32_t nch = seg_chunks(len);
    const int32_t c0 = static_cast<int32_t>(atomicAdd(&ctr->nlchunks, static_cast<uint32_t>(nch)));
    L.target[l] = t;
    L.base[l] = base;
    L.len[l] = len;
    L.chunk0[l] = c0;
    L.prefix[l] = 0;
    L.room[l] = room;
    for (int32_t c = 0; c < nch; ++c) L.owner[c0 + c] = static_cast<int32_t>(l);
}

// Fast path of admission: if everything aimed at t fits, admit it all;
// otherwise the candidate goes to the slow list and its target gets a
// segment (small label spaces: the grid walks the labels; otherwise the first
// slow candidate of a target claims it).
template <bool kSmall, int kAdmitIters>
__global__ void __launch_bounds__(256) admit_kernel(const int32_t* __restrict__ ct, const int32_t* __restrict__ cg,
                                                    int32_t count, const int32_t* __restrict__ w,
                                                    const int32_t* __restrict__ tsum,
                                                    const int32_t* __restrict__ cnt, Bounds B,
                                                    uint8_t* __restrict__ ok, uint32_t* __restrict__ slow_idx,
                                                    int32_t* __restrict__ seg_off, int32_t* __restrict__ seg_list,
                                                    LargeSel L, int32_t small_max, int32_t nw, Counters* ctr,
                                                    const uint32_t* __restrict__ gate) {
    __shared__ int32_t s_min[4], s_max[4];
    if (stopped(gate)) return;  // uniform over the grid
    if (kSmall) {
        for (int32_t t = blockIdx.x * 256 + threadIdx.x; t < nw; t += gridDim.x * 256) {
            if (cnt[t] == 0) continue;
            const int64_t room = bound_of(B, t) - static_cast<int64_t>(w[t]);
            if (tsum[t] > room) claim_segment(t, cnt[t], room, seg_off, seg_list, L, small_max, ctr);
        }
    }
    // each block takes kAdmitIters * 256 consecutive candidates at a time
    // and appends its slow ones with one atomic
    int32_t gmin = INT_MAX, gmax = INT_MIN;
    for (int32_t base = blockIdx.x * (kAdmitIters * 256); base < count; base += gridDim.x * (kAdmitIters * 256)) {
        uint32_t mask = 0;
        // the thread's targets and gains first (loads in flight together),
        // then the decisions
        int32_t tt[kAdmitIters], gg[kAdmitIters];
#pragma unroll
        for (int it = 0; it < kAdmitIters; ++it) {
            const int32_t p = base + it * 256 + static_cast<int32_t>(threadIdx.x);
            tt[it] = p < count ? ct[p] : -2;
            gg[it] = p < count ? cg[p] : 0;
        }
#pragma unroll
        for (int it = 0; it < kAdmitIters; ++it) {
            const int32_t p = base + it * 256 + static_cast<int32_t>(threadIdx.x);
            const int32_t t = tt[it];
            if (t == -2) continue;  // past the end
            uint8_t o = 0;
            if (t >= 0) {
                const int64_t room = bound_of(B, t) - static_cast<int64_t>(w[t]);
                if (tsum[t] <= room) {
                    o = 1;
                } else {
                    o = kOkSlow;
                    mask |= 1u << it;
                    const int32_t gain = gg[it];
                    gmin = gain < gmin ? gain : gmin;
                    gmax = gain > gmax ? gain : gmax;
                    if (!kSmall && seg_off[t] == -1 && atomicCAS(&seg_off[t], -1, -2) == -1)
                        claim_segment(t, cnt[t], room, seg_off, seg_list, L, small_max, ctr);
                }
            }
            ok[p] = o;
        }
        uint32_t j = block_append_count(static_cast<uint32_t>(__popc(mask)), &ctr->nslow);
        while (mask) {
            const int it = __ffs(mask) - 1;
            mask &= mask - 1;
            slow_idx[j++] = static_cast<uint32_t>(base + it * 256 + static_cast<int32_t>(threadIdx.x));
        }
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

// Writes every slow candidate into its target's segment as the key
// [gmax - gain][node] (ascending key = gain desc, node asc), with its weight.
// Space is reserved once per label per block chunk.
template <bool kSmall, int R>
__global__ void __launch_bounds__(256) scatter_kernel(const uint32_t* __restrict__ slow_idx,
                                                      const int32_t* __restrict__ nodes, const int32_t* __restrict__ ct,
                                                      const int32_t* __restrict__ cg, const int32_t* __restrict__ vw,
                                                      int bits_v, int32_t nw, const int32_t* __restrict__ seg_off,
                                                      int32_t* __restrict__ seg_fill, uint64_t* __restrict__ skey,
                                                      int32_t* __restrict__ swt, const Counters* ctr) {
    constexpr int kSlots = kSmall ? kSmallLabels : kAggTable;
    __shared__ int32_t keys[kSmall ? 1 : kAggTable];
    __shared__ int32_t lcnt[kSlots];
    __shared__ int32_t lbase[kSlots];
    const int32_t nslots = kSmall ? nw : kAggTable;
    const uint32_t m = ctr->nslow;
    const int32_t gmax = ctr->gmax;
    for (int j = threadIdx.x; j < nslots; j += 256) {
        if (!kSmall) keys[j] = -1;
        lcnt[j] = 0;
    }
    __syncthreads();
    for (uint32_t base = blockIdx.x * (R * 256); base < m; base += gridDim.x * (R * 256)) {
        // the thread's slow candidates, their targets, nodes and gains, all
        // loaded before the LDS work
        uint32_t pr[R];
        int32_t tr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t j = base + r * 256 + threadIdx.x;
            pr[r] = j < m ? slow_idx[j] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) tr[r] = pr[r] != 0xFFFFFFFFu ? ct[pr[r]] : -1;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (tr[r] >= 0) atomicAdd(&lcnt[agg_slot<kSmall>(keys, tr[r], true)], 1);
        __syncthreads();
        for (int i = threadIdx.x; i < nslots; i += 256) {
            const int32_t t = kSmall ? i : keys[i];
            lbase[i] = (t >= 0 && lcnt[i]) ? atomicAdd(&seg_fill[t], lcnt[i]) : 0;
            lcnt[i] = 0;
        }
        __syncthreads();
        int32_t vr[R], gr[R], cr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            vr[r] = tr[r] >= 0 ? nodes[pr[r]] : 0;
            gr[r] = tr[r] >= 0 ? cg[pr[r]] : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) cr[r] = tr[r] >= 0 ? (vw ? vw[vr[r]] : 1) : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (tr[r] < 0) continue;
            const int32_t t = tr[r];
            const int32_t i = agg_slot<kSmall>(keys, t, false);
            const int32_t at = seg_off[t] + lbase[i] + atomicAdd(&lcnt[i], 1);
            skey[at] = (static_cast<uint64_t>(static_cast<int64_t>(gmax) - gr[r]) << bits_v) |
                       static_cast<uint64_t>(static_cast<uint32_t>(vr[r]));
            swt[at] = cr[r];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nslots; i += 256) {
            if (!kSmall) keys[i] = -1;
            lcnt[i] = 0;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bits_of(uint64_t x) { return x ? 64 - __clzll(static_cast<long long>(x)) : 0; }

__device__ __forceinline__ int64_t shfl_up_i64(int64_t v, int o) {
    const uint32_t lo = __shfl_up(static_cast<uint32_t>(static_cast<uint64_t>(v)), o, 64);
    const uint32_t hi = __shfl_up(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32), o, 64);
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// One workgroup per overflowing target (grid-stride over the segments):
// finds the smallest key whose inclusive weight prefix, in key order, exceeds
// the target's room bound - w(t), by a most-significant-digit-first radix
// selection on weight histograms, and stores it as the target's boundary:
// every candidate with a smaller key is admitted (node weights are >= 0, so
// that is exactly the admitted prefix).  Block 0 also keeps the sub-round's
// gmax for the apply kernel.
__global__ void __launch_bounds__(256) select_kernel(const int32_t* __restrict__ seg_list,
                                                     int32_t* __restrict__ seg_off, int32_t* __restrict__ seg_fill,
                                                     const int32_t* __restrict__ cnt, const int32_t* __restrict__ w,
                                                     Bounds B, int bits_v, const uint64_t* __restrict__ skey,
                                                     const int32_t* __restrict__ swt, uint64_t* __restrict__ bnd,
                                                     int32_t small_max, Counters* ctr) {
    __shared__ unsigned long long hist[256];
    __shared__ uint64_t s_prefix, s_mask;
    __shared__ int64_t s_room;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->gkey = ctr->gmax;
    const uint32_t nseg = ctr->nseg;
    const int total_bits = bits_of(static_cast<uint64_t>(static_cast<int64_t>(ctr->gmax) - ctr->gmin)) + bits_v;
    const int passes = total_bits > 0 ? (total_bits + 7) / 8 : 1;
    for (uint32_t sid = blockIdx.x; sid < nseg; sid += gridDim.x) {
        const int32_t t = seg_list[sid];
        const int32_t base = seg_off[t];
        const int32_t len = cnt[t];
        if (len > small_max) {  // selected by the multi-workgroup kernels, which keep their own copy of the range
            if (threadIdx.x == 0) {
                seg_off[t] = -1;
                seg_fill[t] = 0;
            }
            continue;
        }
        if (threadIdx.x == 0) {
            s_prefix = 0;
            s_mask = 0;
            s_room = bound_of(B, t) - static_cast<int64_t>(w[t]);
        }
        __syncthreads();
        for (int pass = passes - 1; pass >= 0; --pass) {
            const int shift = 8 * pass;
            hist[threadIdx.x] = 0;
            __syncthreads();
            const uint64_t prefix = s_prefix, pmask = s_mask;
            for (int32_t i = threadIdx.x; i < len; i += 256) {
                const uint64_t k = skey[base + i];
                const int32_t c = swt[base + i];
                if ((k & pmask) == prefix && c) atomicAdd(&hist[(k >> shift) & 255], static_cast<unsigned long long>(c));
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                // boundary digit: the first whose cumulative weight exceeds the
                // room (digit 255 when none of 0..254 does); lane j holds digits
                // 4j .. 4j+3
                const int lane = threadIdx.x;
                const int64_t room = s_room;
                int64_t h[4], local = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h[q] = static_cast<int64_t>(hist[4 * lane + q]);
                    local += h[q];
                }
                int64_t incl = local;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int64_t u = shfl_up_i64(incl, o);
                    if (lane >= o) incl += u;
                }
                int64_t run = incl - local;
                int d = 256;
                int64_t rund = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (d != 256) continue;
                    if (run + h[q] > room) {
                        d = 4 * lane + q;
                        rund = run;
                    } else {
                        run += h[q];
                    }
                }
                const int dmin = wave_min(d);
                const bool mine = dmin == 256 ? lane == 63 : d == dmin;
                if (mine) {
                    const int dd = dmin == 256 ? 255 : dmin;
                    const int64_t before = dmin == 256 ? incl - h[3] : rund;
                    s_room = room - before;
                    s_prefix = prefix | (static_cast<uint64_t>(dd) << shift);
                    s_mask = pmask | (255ULL << shift);
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            bnd[t] = s_prefix;  // smallest key that does not fit
            seg_off[t] = -1;
            seg_fill[t] = 0;
        }
    }
}

// Boundary digit of a histogram held as kPerT consecutive digits per thread
// (hv, summing to local): the first digit whose cumulative weight exceeds
// room (the last digit when none below it does); *s_d and *s_run (the weight
// of the digits before it) are set for the whole block.
template <int NT, int kPerT>
__device__ __forceinline__ void block_pick_digit(const int64_t* hv, int64_t local, int64_t room, int64_t* sc,
                                                 int* s_d, int64_t* s_run) {
    const int j = threadIdx.x;
    sc[j] = local;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {  // inclusive scan
        const int64_t add = j >= o ? sc[j - o] : 0;
        __syncthreads();
        sc[j] += add;
        __syncthreads();
    }
    const int64_t incl = sc[j];
    const int64_t excl = incl - local;
    if (j == NT - 1) {  // no digit below the last one exceeds the room
        *s_d = NT * kPerT - 1;
        *s_run = incl - hv[kPerT - 1];
    }
    __syncthreads();
    // the digit where the admissible weight runs out (monotone: one thread)
    if (incl > room && excl <= room) {
        int64_t run = excl;
        int d = kPerT * j + kPerT - 1;
        for (int q = 0; q < kPerT - 1; ++q) {
            if (run + hv[q] > room) {
                d = kPerT * j + q;
                break;
            }
            run += hv[q];
        }
        *s_d = d;
        *s_run = run;
    }
    __syncthreads();
}

// One digit of the multi-workgroup selection per launch, most significant
// first: launch j of nlaunch handles digit passes - 1 - j.  Every block adds
// its chunk's weight histogram to the segment's histogram in HBM; the last
// block to finish a segment picks that segment's boundary digit (no block
// waits for another).  Keys rarely need more digits than the host launches;
// when they do, the last block of each segment in the final launch finishes
// the remaining digits alone, over the whole segment.  After the last digit
// the segment's boundary key is stored.
__global__ void __launch_bounds__(kLargeThreads) large_pass_kernel(LargeSel L, int launch, int nlaunch, int bits_v,
                                                                   const uint64_t* __restrict__ skey,
                                                                   const int32_t* __restrict__ swt,
                                                                   uint64_t* __restrict__ bnd, const Counters* ctr) {
    constexpr int NT = kLargeThreads;
    constexpr int kPerT = kLBins / NT;
    constexpr int U = 4;
    __shared__ uint32_t h[kLBins];
    __shared__ int64_t sc[NT];
    __shared__ int s_last, s_d;
    __shared__ int64_t s_run;
    const int total_bits = bits_of(static_cast<uint64_t>(static_cast<int64_t>(ctr->gmax) - ctr->gmin)) + bits_v;
    const int passes = total_bits > 0 ? (total_bits + kLDigit - 1) / kLDigit : 1;
    const int pass = passes - 1 - launch;
    const uint32_t nlarge = ctr->nlarge;
    if (pass < 0 || nlarge == 0) return;  // uniform over the grid
    const bool finish = launch == nlaunch - 1;
    const int shift = kLDigit * pass;
    const uint64_t above = shift + kLDigit >= 64 ? 0ULL : ~0ULL << (shift + kLDigit);  // digits already fixed
    const int32_t nch = static_cast<int32_t>(ctr->nlchunks);
    const int j = threadIdx.x;
    // adds the weights of entries [i0, i1) of a segment whose key matches
    // prefix on the digits above `sh` to the LDS histogram of digit `sh`
    auto accumulate = [&](int32_t base, int32_t i0, int32_t i1, uint64_t prefix, uint64_t ab, int sh) {
        for (int32_t i = i0 + j; i < i1; i += NT * U) {
            uint64_t k[U];
            int32_t wt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t x = i + u * NT;
                k[u] = x < i1 ? skey[base + x] : 0;
                wt[u] = x < i1 ? swt[base + x] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if ((k[u] & ab) == prefix && wt[u]) atomicAdd(&h[(k[u] >> sh) & (kLBins - 1)], static_cast<uint32_t>(wt[u]));
        }
    };
    for (int32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int32_t l = L.owner[c];
        const int32_t base = L.base[l];
        const int32_t len = L.len[l];
        const int32_t i0 = (c - L.chunk0[l]) * kSegChunk;
        const int32_t i1 = i0 + kSegChunk < len ? i0 + kSegChunk : len;
        const uint64_t prefix = L.prefix[l];
        uint32_t* hl = L.hist + static_cast<size_t>(l) * kLBins;
        for (int q = j; q < kLBins; q += NT) h[q] = 0;
        __syncthreads();
        accumulate(base, i0, i1, prefix, above, shift);
        __syncthreads();
        for (int q = j; q < kLBins; q += NT)
            if (h[q]) atomicAdd(&hl[q], h[q]);
        // the barrier orders every thread's adds before thread 0's release
        // fence, and thread 0's acquire fence before every thread's reads (a
        // device-scope fence writes back and invalidates the L2, so one
        // thread issues it, not every wave)
        __syncthreads();
        if (j == 0) {
            const uint32_t nchunks = static_cast<uint32_t>(seg_chunks(len));
            __threadfence();
            const bool last = atomicAdd(&L.done[l], 1u) == nchunks - 1;
            if (last) __threadfence();
            s_last = last;
        }
        __syncthreads();
        if (s_last) {  // block-uniform
            // thread j holds digits kPerT*j .. kPerT*j + kPerT-1
            int64_t hv[kPerT];
            int64_t local = 0;
#pragma unroll
            for (int q = 0; q < kPerT; ++q) {
                hv[q] = __hip_atomic_load(&hl[kPerT * j + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                local += hv[q];
            }
            int64_t room = L.room[l];
            block_pick_digit<NT, kPerT>(hv, local, room, sc, &s_d, &s_run);
#pragma unroll
            for (int q = 0; q < kPerT; ++q) hl[kPerT * j + q] = 0;
            uint64_t np = prefix | (static_cast<uint64_t>(s_d) << shift);
            room -= s_run;
            if (finish) {
                for (int q2 = pass - 1; q2 >= 0; --q2) {  // remaining digits, this block alone
                    const int sh = kLDigit * q2;
                    __syncthreads();
                    for (int q = j; q < kLBins; q += NT) h[q] = 0;
                    __syncthreads();
                    accumulate(base, 0, len, np, ~0ULL << (sh + kLDigit), sh);
                    __syncthreads();
                    local = 0;
#pragma unroll
                    for (int q = 0; q < kPerT; ++q) {
                        hv[q] = h[kPerT * j + q];
                        local += hv[q];
                    }
                    block_pick_digit<NT, kPerT>(hv, local, room, sc, &s_d, &s_run);
                    np |= static_cast<uint64_t>(s_d) << sh;
                    room -= s_run;
                }
            }
            if (j == 0) {
                L.room[l] = room;
                L.prefix[l] = np;
                L.done[l] = 0;
                if (pass == 0 || finish) bnd[L.target[l]] = np;  // smallest key that does not fit
            }
        }
        __syncthreads();
    }
}

// The per-sub-round counters back to their empty state (the round's
// candidate count and the kept gmax are not touched).
__device__ __forceinline__ void clear_subround(Counters* ctr) {
    ctr->ncand = 0;
    ctr->nslow = 0;
    ctr->gmin = INT_MAX;
    ctr->gmax = INT_MIN;
    ctr->nseg = 0;
    ctr->slow_total = 0;
    ctr->nlarge = 0;
    ctr->nlchunks = 0;
}

// Decides the slow candidates from their targets' boundary keys, moves the
// admitted candidates and updates the label weights; also clears the
// per-target candidate sums and counts and the sub-round counters for the
// next sub-round (no kernel of this one reads them any more).
template <bool kSmall>
__global__ void __launch_bounds__(256) apply_kernel(const int32_t* __restrict__ ct, uint8_t* __restrict__ ok,
                                                    const int32_t* __restrict__ nodes, int32_t count,
                                                    const int32_t* __restrict__ cg, int bits_v,
                                                    const uint64_t* __restrict__ bnd,
                                                    const int32_t* __restrict__ vw, int32_t* __restrict__ label,
                                                    uint8_t* __restrict__ label8, uint16_t* __restrict__ label16,
                                                    int32_t* __restrict__ w, int32_t* __restrict__ tsum,
                                                    int32_t* __restrict__ cnt, int32_t nw, Counters* ctr,
                                                    const uint32_t* __restrict__ gate) {
    __shared__ int32_t delta[kSmall ? kSmallLabels : 1];
    const int32_t gkey = ctr->gkey;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) clear_subround(ctr);
        if (kSmall)
            for (int j = threadIdx.x; j < nw; j += 256) {
                tsum[j] = 0;
                cnt[j] = 0;
            }
    }
    if (stopped(gate)) return;  // uniform over the grid
    if (kSmall) {
        for (int j = threadIdx.x; j < nw; j += 256) delta[j] = 0;
        __syncthreads();
    }
    // U grid-stride positions per thread at a time: their loads are issued
    // together, level by level, before the updates
    constexpr int U = 4;
    const int32_t stride = gridDim.x * 256;
    for (int32_t p0 = blockIdx.x * 256 + threadIdx.x; p0 < count; p0 += stride * U) {
        int32_t tq[U], vq[U], aq[U], cq[U];
        uint8_t oq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = p0 + u * stride;
            tq[u] = p < count ? ct[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = p0 + u * stride;
            oq[u] = tq[u] >= 0 ? ok[p] : 0;
            vq[u] = tq[u] >= 0 ? nodes[p] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = p0 + u * stride;
            if (oq[u] == kOkSlow) {
                const uint64_t key = (static_cast<uint64_t>(static_cast<int64_t>(gkey) - cg[p]) << bits_v) |
                                     static_cast<uint64_t>(static_cast<uint32_t>(vq[u]));
                oq[u] = key < bnd[tq[u]] ? 1 : 0;
                ok[p] = oq[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            aq[u] = oq[u] ? label[vq[u]] : 0;
            cq[u] = oq[u] ? (vw ? vw[vq[u]] : 1) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t t = tq[u];
            if (t < 0) continue;
            if (!kSmall) {
                tsum[t] = 0;
                cnt[t] = 0;
            }
            if (!oq[u]) continue;
            const int32_t v = vq[u];
            const int32_t a = aq[u];
            const int32_t c = cq[u];
            label[v] = t;
            if (label8) label8[v] = static_cast<uint8_t>(t);
            if (label16) label16[v] = static_cast<uint16_t>(t);
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
    }
    if (kSmall) {
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256)
            if (delta[j]) atomicAdd(&w[j], delta[j]);
    }
}

template <typename T>
__global__ void narrow_kernel(const int32_t* __restrict__ label, int32_t n, T* __restrict__ out) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) out[v] = static_cast<T>(label[v]);
}

// After a sub-round: every neighbour of a node that moved is no longer quiet.
// One wave per 64 schedule positions; the wave walks each mover's row.
__global__ void __launch_bounds__(256) unquiet_kernel(const int32_t* __restrict__ ct, const uint8_t* __restrict__ ok,
                                                      const int32_t* __restrict__ nodes, int32_t count,
                                                      const int64_t* __restrict__ xadj,
                                                      const int32_t* __restrict__ adj, uint8_t* __restrict__ quiet,
                                                      const uint32_t* __restrict__ gate,
                                                      const uint32_t* __restrict__ rcnt, int32_t round, int32_t qn) {
    if (stopped(gate) || quiet_mode(quiet, rcnt, round, qn) == 0) return;
    const int64_t base = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) & ~63LL;
    const int lane = lane_id();
    const int64_t p = base + lane;
    const bool mover = p < count && ct[p] >= 0 && ok[p];
    uint64_t m = __ballot(mover);
    while (m) {
        const int i = __ffsll(static_cast<long long>(m)) - 1;
        m &= m - 1;
        const int32_t u = nodes[base + i];
        const int64_t e = xadj[u + 1];
        for (int64_t j = xadj[u] + lane; j < e; j += 64) quiet[adj[j]] = 0;
    }
}

__global__ void reset_counters_kernel(Counters* ctr) { clear_subround(ctr); }

// --------------------------------------------------------------- schedule

// Upper degree of each bucket but the hub bucket (non-decreasing).
struct Thresholds {
    int32_t t[kNB - 1];
};

// Category of a node: colour * kNB + degree bucket; degree-0 nodes never move
// and go to the extra category ncat.
__global__ void __launch_bounds__(256) classify_kernel(int32_t n, const int64_t* __restrict__ xadj,
                                                       const int32_t* __restrict__ color_override, uint64_t hc,
                                                       const int32_t* __restrict__ gid, const uint64_t* __restrict__ g_hc,
                                                       const int32_t* __restrict__ g_nbase,
                                                       const uint8_t* __restrict__ g_active,
                                                       int32_t nsub, Thresholds th,
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
    // grid-stride: few workgroups, so the per-category totals cost few global
    // atomics on their handful of addresses
    for (int32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int64_t d = xadj[v + 1] - xadj[v];
        uint64_t hcv = hc;
        int32_t lv = v;  // graph-local id
        bool act = true;
        if (gid) {
            const int32_t g = gid[v];
            hcv = g_hc[g];
            lv = v - g_nbase[g];
            act = g_active[g] != 0;
        }
        int32_t col;
        if (color_override) {
            col = color_override[v];
            if (col < 0 || col >= nsub) {
                atomicOr(&ctr->bad_color, 1u);
                col = 0;
            }
        } else {
            col = static_cast<int32_t>(mix64(hcv ^ static_cast<uint64_t>(static_cast<uint32_t>(lv))) %
                                       static_cast<uint64_t>(nsub));
        }
        int32_t bucket = kHubBucket;
#pragma unroll
        for (int j = kHubBucket - 1; j >= 0; --j)
            if (d <= th.t[j]) bucket = j;
        const int32_t cat = (d == 0 || !act) ? ncat : col * kNB + bucket;
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

// Per-graph hash prefixes H(seed_g, tag, level, phase[, round]).
__global__ void graph_prefix_kernel(int32_t G, const uint64_t* __restrict__ seed, uint64_t tag, uint64_t level,
                                    uint64_t phase, int64_t round, uint64_t* __restrict__ out) {
    const int32_t g = blockIdx.x * 256 + threadIdx.x;
    if (g >= G) return;
    uint64_t h = mix64(seed[g]);
    h = mix64(h ^ tag);
    h = mix64(h ^ level);
    h = mix64(h ^ phase);
    if (round >= 0) h = mix64(h ^ static_cast<uint64_t>(round));
    out[g] = h;
}

constexpr int kLWChunk = 2048;  // nodes per block and step of label_weights_kernel<false>

template <bool kSmall>
__global__ void __launch_bounds__(256) label_weights_kernel(int32_t n, const int32_t* __restrict__ label,
                                                            const int32_t* __restrict__ vw, int32_t* __restrict__ w,
                                                            int32_t nw) {
    __shared__ int32_t loc[kSmallLabels];
    if (kSmall) {
        for (int j = threadIdx.x; j < nw; j += 256) loc[j] = 0;
        __syncthreads();
        for (int32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
            const int32_t c = vw ? vw[v] : 1;
            if (c) atomicAdd(&loc[label[v]], c);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < nw; j += 256)
            if (loc[j]) atomicAdd(&w[j], loc[j]);
        return;
    }
    // Large label spaces, kLWChunk consecutive nodes per block at a time: when
    // their labels span fewer than kSmallLabels ids (the blocks of the few
    // graphs a chunk of a batch covers, or a run of singleton clusters), they
    // are summed in LDS first, so a label many nodes share costs one global
    // atomic per chunk; otherwise every node adds to HBM directly.
    constexpr int R = kLWChunk / 256;
    __shared__ int32_t s_lo[4], s_hi[4];
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * kLWChunk; base < n;
         base += static_cast<int64_t>(gridDim.x) * kLWChunk) {
        int32_t lab[R], cw[R];
        int32_t lo = INT_MAX, hi = INT_MIN;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t v = base + r * 256 + threadIdx.x;
            lab[r] = v < n ? label[v] : -1;
            cw[r] = v < n ? (vw ? vw[v] : 1) : 0;
            if (lab[r] >= 0) {
                lo = lab[r] < lo ? lab[r] : lo;
                hi = lab[r] > hi ? lab[r] : hi;
            }
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane_id() == 0) {
            s_lo[threadIdx.x >> 6] = lo;
            s_hi[threadIdx.x >> 6] = hi;
        }
        __syncthreads();
        lo = min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3]));
        hi = max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3]));
        const int64_t span = static_cast<int64_t>(hi) - lo + 1;
        if (span > 0 && span <= kSmallLabels) {
            for (int j = threadIdx.x; j < span; j += 256) loc[j] = 0;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (cw[r]) atomicAdd(&loc[lab[r] - lo], cw[r]);
            __syncthreads();
            for (int j = threadIdx.x; j < span; j += 256)
                if (loc[j]) atomicAdd(&w[lo + j], loc[j]);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (cw[r]) atomicAdd(&w[lab[r]], cw[r]);
        }
        __syncthreads();  // s_lo, s_hi and loc are reused by the next chunk
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

// Side streams for the independent evaluation launches of a sub-round
// (default priority, created once per thread).  fork() makes them wait for
// the work already on the caller's stream, join() makes the caller's stream
// wait for them.  The hub chain, usually the longest, stays on the caller's
// stream, so the join mostly waits on work that has already finished (a
// cross-stream wait on unfinished work costs the device some 20 us).
class EvalStreams {
  public:
    static constexpr int kN = 2;
    EvalStreams() {
        for (int i = 0; i < kN; ++i) {
            HIPCHK(hipStreamCreateWithFlags(&st_[i], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&done_[i], hipEventDisableTiming));
        }
        HIPCHK(hipEventCreateWithFlags(&start_, hipEventDisableTiming));
    }
    EvalStreams(const EvalStreams&) = delete;
    EvalStreams& operator=(const EvalStreams&) = delete;
    void fork(hipStream_t s) {
        HIPCHK(hipEventRecord(start_, s));
        for (int i = 0; i < kN; ++i) HIPCHK(hipStreamWaitEvent(st_[i], start_, 0));
    }
    void join(hipStream_t s) {
        for (int i = 0; i < kN; ++i) {
            HIPCHK(hipEventRecord(done_[i], st_[i]));
            HIPCHK(hipStreamWaitEvent(s, done_[i], 0));
        }
    }
    // heavy buckets (large rows) apart from each other and from the hubs
    hipStream_t bucket(int bk) const {
        static const int kMap[kNB - 1] = {0, 0, 1, 1, 1, 0, 1, 0};
        return st_[kMap[bk]];
    }

  private:
    hipStream_t st_[kN];
    hipEvent_t done_[kN];
    hipEvent_t start_;
};

EvalStreams& eval_streams() {
    thread_local EvalStreams e;
    return e;
}

thread_local Counters* t_host_ctr = nullptr;

Counters* host_counters() {
    if (!t_host_ctr) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&t_host_ctr), sizeof(Counters), hipHostMallocDefault));
    return t_host_ctr;
}

// Pinned host copies of the per-round candidate counts (grown as needed,
// kept for the thread's lifetime).
thread_local uint32_t* t_host_rc = nullptr;
thread_local int32_t t_host_rc_cap = 0;

uint32_t* host_round_counts(int32_t rounds) {
    if (rounds > t_host_rc_cap) {
        if (t_host_rc) HIPCHK(hipHostFree(t_host_rc));
        t_host_rc_cap = std::max(rounds, 64);
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&t_host_rc), sizeof(uint32_t) * t_host_rc_cap,
                             hipHostMallocDefault));
    }
    return t_host_rc;
}

// Two events marking the end of consecutive rounds (per thread).
struct RoundEvents {
    hipEvent_t ev[2];
    RoundEvents() {
        for (hipEvent_t& e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
};

RoundEvents& round_events() {
    thread_local RoundEvents r;
    return r;
}

// Records the work enqueued on the capture stream cs (and on streams joined
// to it) while it lives into a graph, when enabled; run() instantiates it,
// launches it on the caller's stream and waits.  The caller's stream may be
// the null stream, which cannot be captured itself.  If an error unwinds
// before run(), the capture is ended and discarded.
class GraphCapture {
  public:
    GraphCapture(hipStream_t cs, hipStream_t exec, bool on) : s_(cs), exec_(exec), on_(on) {
        if (on_) HIPCHK(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    }
    GraphCapture(const GraphCapture&) = delete;
    GraphCapture& operator=(const GraphCapture&) = delete;
    void run() {
        if (!on_) return;
        on_ = false;
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamEndCapture(s_, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
        }
        const hipError_t l = hipGraphLaunch(exec, exec_);
        const hipError_t w = l == hipSuccess ? hipStreamSynchronize(exec_) : l;
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        HIPCHK(w);
    }
    ~GraphCapture() {
        if (!on_) return;
        hipGraph_t graph = nullptr;
        if (hipStreamEndCapture(s_, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
    }

  private:
    hipStream_t s_;
    hipStream_t exec_;
    bool on_;
};

// The stream rounds are captured on (per thread, default priority).
hipStream_t capture_stream() {
    struct Holder {
        hipStream_t st;
        Holder() { HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking)); }
    };
    thread_local Holder h;
    return h.st;
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
            label_weights_kernel<false><<<static_cast<unsigned>(std::min<int64_t>((g.n + kLWChunk - 1) / kLWChunk,
                                                                                  kMaxBlocks)),
                                          256, 0, s>>>(g.n, label, g.vw, w, nw);
        LAUNCHCHK();
    }
}

LPResult run_lp(const DevGraph& g, int32_t phase, int32_t level, uint64_t seed, int32_t nsub, int32_t rounds,
                int64_t bound, int32_t* label, int32_t* w, int32_t nw, const int32_t* color_override,
                const LPTuning& tune, hipStream_t s, const MultiGraph* mg) {
    LPResult res;
    const int32_t n = g.n;
    if (n == 0 || rounds <= 0) return res;
    if (nsub < 1 || nsub > 16) fail(-1, "subrounds must be in 1..16");
    const bool small = nw <= kSmallLabels;
    static const bool trace = std::getenv("SCLAP_TRACE") != nullptr;  // per sub-round counts on stderr

    // --- schedule: nodes grouped by (colour, degree bucket), ascending ids
    const int32_t ncat = nsub * kNB;
    Thresholds th;
    {
        const int32_t lane = std::max(1, std::min(tune.lane_max, kLaneMax));
        const int32_t wave = std::max(lane, std::min(tune.wave_max, kWaveMaxDeg));
        const int32_t block = std::max(wave, std::min(tune.block_max, kBlockMaxDeg));
        th.t[0] = std::min(kLaneSmall, lane);
        th.t[1] = lane;
        th.t[2] = std::max(lane, std::min(kG16Max, wave));
        th.t[3] = std::max(th.t[2], std::min(kG32Max, wave));
        th.t[4] = wave;
        th.t[5] = std::min(block, std::max(wave, kBlock1Max));
        th.t[6] = std::min(block, std::max(th.t[5], kBlock2Max));
        th.t[7] = block;
    }
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
    const uint64_t lvl64 = static_cast<uint64_t>(static_cast<uint32_t>(level));
    const uint64_t ph64 = static_cast<uint64_t>(static_cast<uint32_t>(phase));
    DBuf<uint64_t> g_hc, g_tp;
    if (mg) {
        g_hc.alloc(std::max(mg->G, 1), s);
        g_tp.alloc(std::max(mg->G, 1), s);
        graph_prefix_kernel<<<grid_for(mg->G, 256), 256, 0, s>>>(mg->G, mg->seed, 1, lvl64, ph64, -1, g_hc.get());
        LAUNCHCHK();
    }
    {
        ProfScope ps("lp_schedule", 0, s);
        classify_kernel<<<capped_grid(n), 256, 0, s>>>(n, g.xadj, color_override, hc, mg ? mg->gid : nullptr,
                                                         g_hc.get(), mg ? mg->nbase : nullptr,
                                                         mg ? mg->active : nullptr, nsub, th,
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
    // refinement labels fit dense arrays when there are few enough blocks
    // (the same test sets EvalArgs::dense_k below); hub chunks are then longer
    const int32_t dense_labels = phase != kCluster ? (mg ? mg->max_labels : nw) : 0;
    const int64_t hub_chunk = dense_labels > 0 && dense_labels <= kDenseMax ? kHubDenseChunk : kHubChunk;
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
            // at most 1024 entries per label partition on average (half the
            // LDS table's limit), at most 2048 partitions
            int32_t lg = 0;
            while (lg < kMaxPartLog && (static_cast<int64_t>(1024) << lg) < hd[h]) ++lg;
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
            for (int64_t sl = 0; sl < hd[h]; sl += hub_chunk) {
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
    DBuf<int32_t> ct(cap, s), cg(cap, s), tsum(nw, s), tcnt(nw, s), seg_off(nw, s), seg_fill(nw, s);
    DBuf<int32_t> seg_list(std::min<int64_t>(cap, nw), s), swt(cap, s);
    DBuf<uint8_t> ok(cap, s);
    DBuf<uint32_t> slow_idx(cap, s);
    DBuf<uint64_t> skey(cap, s);
    // multi-workgroup selection state: at most cap / kSmallSeg large segments
    const int32_t small_max = std::max(1, std::min(tune.select_small_max, kSmallSeg));
    const int64_t max_large = cap / small_max + 1;
    const int64_t max_lchunks = cap / kSegChunk + max_large;
    DBuf<int32_t> ltarget(max_large, s), lbase(max_large, s), llen(max_large, s), lchunk0(max_large, s);
    DBuf<int32_t> lowner(max_lchunks, s);
    DBuf<uint32_t> lhist(max_large * kLBins, s);
    DBuf<uint64_t> lprefix(max_large, s);
    DBuf<int64_t> lroom(max_large, s);
    DBuf<uint32_t> ldone(max_large, s);
    fill_u32(lhist.get(), 0, max_large * kLBins, s);
    fill_u32(ldone.get(), 0, max_large, s);
    LargeSel LS{ltarget.get(), lbase.get(), llen.get(), lchunk0.get(), lowner.get(), lhist.get(), lprefix.get(),
                lroom.get(),
                ldone.get()};
    // digits of the selection key: node id bits plus at most 32 bits of gain range
    // launches of the multi-workgroup selection: enough digits for node ids
    // plus a 12-bit gain range; wider keys finish in the last launch
    const int max_launches = (bits_for(static_cast<uint64_t>(n - 1)) + 32 + kLDigit - 1) / kLDigit;
    const int sel_launches =
        tune.select_launches > 0
            ? std::min(tune.select_launches, max_launches)
            : std::min(max_launches, (bits_for(static_cast<uint64_t>(n - 1)) + 12 + kLDigit - 1) / kLDigit);
    // boundary key of every target that cannot take all its candidates
    DBuf<uint64_t> bnd(nw, s);
    fill_i32(tsum.get(), 0, nw, s);
    fill_i32(tcnt.get(), 0, nw, s);
    fill_i32(seg_off.get(), -1, nw, s);
    fill_i32(seg_fill.get(), 0, nw, s);

    EvalArgs A;
    A.xadj = g.xadj;
    A.adj = g.adj;
    A.S = g.S;
    A.ew = g.ew;
    A.vw = g.vw;
    A.label = label;
    A.w = w;
    A.bound = bound;
    A.refine = phase != kCluster ? 1 : 0;  // the initial phase follows the refinement rules
    A.gid = mg ? mg->gid : nullptr;
    A.g_tp = g_tp.get();
    A.g_bound = mg ? mg->bound : nullptr;
    A.g_lbase = mg ? mg->lbase : nullptr;
    const Bounds BB{bound, mg ? mg->lgid : nullptr, mg ? mg->bound : nullptr};
    // refinement labels are blocks: dense connection arrays when few enough
    const int32_t dense_k = dense_labels;
    A.dense_k = dense_k > 0 && dense_k <= kDenseMax ? dense_k : 0;
    const bool dense = A.dense_k > 0;
    DBuf<int32_t> hub_sum;
    if (dense) {
        int64_t max_hubs = 1;
        for (const HubPlan& P : plans) max_hubs = std::max<int64_t>(max_hubs, P.count);
        hub_sum.alloc(max_hubs * A.dense_k, s);
        fill_i32(hub_sum.get(), 0, max_hubs * A.dense_k, s);
    }
    DBuf<uint8_t> lab8;
    DBuf<uint16_t> lab16;
    if (nw <= 256) {
        lab8.alloc(n, s);
        narrow_kernel<uint8_t><<<grid_for(n, 256), 256, 0, s>>>(label, n, lab8.get());
        LAUNCHCHK();
    } else if (nw <= 65536) {
        lab16.alloc(n, s);
        narrow_kernel<uint16_t><<<grid_for(n, 256), 256, 0, s>>>(label, n, lab16.get());
        LAUNCHCHK();
    }
    A.label8 = lab8.get();
    A.label16 = lab16.get();
    // quiet-node tracking starts once a round has few candidates (marking the
    // neighbours of every mover is then cheap) and skipping one round later;
    // the kernels derive the start from the per-round counts (quiet_mode)
    DBuf<uint8_t> quiet;
    // the default (0) leaves it off here; the batch driver turns it on
    const bool track_quiet = tune.skip_quiet > 0;
    if (track_quiet) {
        quiet.alloc(n, s);
        fill_u8(quiet.get(), 0, n, s);
    }
    A.quiet = quiet.get();
    A.quiet_n = n;

    // Algorithmic bytes of one evaluation launch, the figure of one round's
    // minimal traffic per unit: per evaluated node 24 (its row offsets, own
    // label, node weight and the weight of one label), per slot 12 (the
    // neighbour id, the edge weight and the neighbour's label), whether or
    // not the kernel reads weights that hold only ones or narrow labels.
    const double node_bytes = 24.0;
    const double slot_bytes = 12.0;
    auto eval_bytes = [&](int64_t nodes_in, unsigned long long slots_in) {
        return node_bytes * static_cast<double>(nodes_in) + slot_bytes * static_cast<double>(slots_in);
    };
    reset_counters_kernel<<<1, 1, 0, s>>>(ctr.get());
    LAUNCHCHK();
    const int bits_v = bits_for(static_cast<uint64_t>(n - 1));
    EvalStreams& evs = eval_streams();

    // candidates per round, read back one round late (see stopped())
    DBuf<uint32_t> rcnt(std::max(rounds, 1), s);
    fill_u32(rcnt.get(), 0, std::max(rounds, 1), s);
    A.rcnt = rcnt.get();
    uint32_t* hrc = host_round_counts(rounds);
    RoundEvents& rev = round_events();
    bool halted = false;
    // bookkeeping of a finished round q (read back from the device)
    auto finish_round = [&](int32_t q) {
        HIPCHK(hipEventSynchronize(rev.ev[q & 1]));
        const uint32_t round_cands = hrc[q];
        res.rounds_run = q + 1;
        res.moves += round_cands;
        if (round_cands == 0) halted = true;
    };
    // Captured execution (tuning option): all rounds of this call are
    // recorded into one HIP graph and launched at once, so the host neither
    // launches kernel by kernel nor waits between rounds; rounds after one
    // without candidates run as gated no-ops (the result is the same, see
    // stopped()).  Not the default: on this GPU the graph runs the same
    // kernels about 1.5 times slower than the host's pipelined launches.  Not
    // while per-launch timing events or the trace are on (events recorded in
    // a graph cannot be timed).
    const bool capture = !trace && !profiler().on && tune.capture > 0;
    // the rounds are enqueued on the capture stream and the graph runs on the
    // caller's stream; buffers above were allocated on the caller's stream
    const hipStream_t caller = s;
    if (capture) s = capture_stream();
    GraphCapture rounds_graph(s, caller, capture);

    for (int32_t r = 0; r < rounds && !halted; ++r) {
        const uint32_t* gate = r > 0 ? rcnt.get() + (r - 1) : nullptr;
        if (mg) {
            graph_prefix_kernel<<<grid_for(mg->G, 256), 256, 0, s>>>(mg->G, mg->seed, 2, lvl64, ph64, r, g_tp.get());
            LAUNCHCHK();
        }
        A.round = r;
        A.gate = gate;
        A.tp = hash_prefix({seed, 2, static_cast<uint64_t>(static_cast<uint32_t>(level)),
                            static_cast<uint64_t>(static_cast<uint32_t>(phase)),
                            static_cast<uint64_t>(static_cast<uint32_t>(r))});
        for (int32_t sc = 0; sc < nsub; ++sc) {
            const int32_t c0 = sc * kNB;
            const int64_t ccount = off[c0 + kNB] - off[c0];
            if (ccount == 0) continue;
            const int32_t* cnodes = nodes + off[c0];
            // evaluation: one result per schedule entry of this colour; the
            // buckets are independent and run side by side on the evaluation
            // streams (hubs on the caller's stream), joined before admission
            unsigned long long colour_slots = 0;
            for (int32_t bk = 0; bk < kNB; ++bk) colour_slots += cslots[c0 + bk];
            const bool side = colour_slots >= (1ULL << 22);  // small colours stay on one stream
            if (side) evs.fork(s);
            // hubs first: their chain (chunks, partitions, decision) is the
            // longest, so its workgroups should be dispatched before the
            // other buckets fill the device
            const HubPlan& P = plans[sc];
            const hipStream_t hs = s;
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
                fill_i32(H.rcount, 0, static_cast<int64_t>(P.nparts) + 3 * Hn, hs);
                A.nodes = H.hub_nodes;
                A.count = Hn;
                A.ct = ct.get() + (off[c0 + kHubBucket] - off[c0]);
                A.cg = cg.get() + (off[c0 + kHubBucket] - off[c0]);
                if (dense) {
                    ProfScope ps("lp_refine_hub_dense", eval_bytes(Hn, cslots[c0 + kHubBucket]), hs);
                    hub_dense_chunk_kernel<<<P.nchunks, kHubThreads, 0, hs>>>(A, H, hub_sum.get());
                    LAUNCHCHK();
                    hub_dense_finish_kernel<<<Hn, 256, 0, hs>>>(A, H, hub_sum.get());
                    LAUNCHCHK();
                } else {
                {
                    ProfScope ps(A.refine ? "lp_refine_hub_chunk" : "lp_eval_hub_chunk", eval_bytes(Hn, cslots[c0 + kHubBucket]), hs);
                    hub_chunk_kernel<<<P.nchunks, kHubThreads, 0, hs>>>(A, H);
                    LAUNCHCHK();
                }
                {
                    ProfScope ps(A.refine ? "lp_refine_hub_part" : "lp_eval_hub_part", 0, hs);
                    hub_part_kernel<<<P.nparts, kPartThreads, 0, hs>>>(A, H);
                    LAUNCHCHK();
                    hub_finish_kernel<<<Hn, 64, 0, hs>>>(A, H);
                    LAUNCHCHK();
                }
                {
                    ProfScope ps(A.refine ? "lp_refine_hub_table" : "lp_eval_hub_table", 0, hs);
                    hub_clear_kernel<<<P.ntchunks, 256, 0, hs>>>(H);
                    LAUNCHCHK();
                    hub_table_insert_kernel<<<P.nparts, 256, 0, hs>>>(H);
                    LAUNCHCHK();
                    hub_scan_kernel<<<P.ntchunks, 256, 0, hs>>>(A, H, P.nparts);
                    LAUNCHCHK();
                    hub_big_finish_kernel<<<Hn, 64, 0, hs>>>(A, H, tfirst_shifted);
                    LAUNCHCHK();
                }
                }
            }
            int32_t bk_from = 0;
            if (!side && tune.fuse >= 0) {  // buckets 0..5 of a small colour in one launch
                FusedBuckets F;
                static const int32_t kPerBlock[kFusedBuckets] = {256, 256, 16, 8, 4, 1};  // nodes per workgroup
                int32_t blocks = 0, fnodes = 0;
                unsigned long long fslots = 0;
                for (int32_t bk = 0; bk < kFusedBuckets; ++bk) {
                    const int64_t count = off[c0 + bk + 1] - off[c0 + bk];
                    F.nodes[bk] = nodes + off[c0 + bk];
                    F.ct[bk] = ct.get() + (off[c0 + bk] - off[c0]);
                    F.cg[bk] = cg.get() + (off[c0 + bk] - off[c0]);
                    F.count[bk] = static_cast<int32_t>(count);
                    F.first[bk] = blocks;
                    blocks += static_cast<int32_t>((count + kPerBlock[bk] - 1) / kPerBlock[bk]);
                    fnodes += static_cast<int32_t>(count);
                    fslots += cslots[c0 + bk];
                }
                F.first[kFusedBuckets] = blocks;
                if (blocks > 0) {
                    ProfScope ps(A.refine ? "lp_refine_fused" : "lp_eval_fused", eval_bytes(fnodes, fslots), s);
                    if (dense) eval_fused_kernel<true><<<blocks, 256, 0, s>>>(A, F);
                    else eval_fused_kernel<false><<<blocks, 256, 0, s>>>(A, F);
                    LAUNCHCHK();
                }
                bk_from = kFusedBuckets;
            }
            for (int32_t bk = bk_from; bk < kHubBucket; ++bk) {
                const hipStream_t bs = side ? evs.bucket(bk) : s;
                const int64_t count = off[c0 + bk + 1] - off[c0 + bk];
                if (count == 0) continue;
                A.nodes = nodes + off[c0 + bk];
                A.count = static_cast<int32_t>(count);
                A.ct = ct.get() + (off[c0 + bk] - off[c0]);
                A.cg = cg.get() + (off[c0 + bk] - off[c0]);
                static const char* const kNames[2][kHubBucket] = {
                    {"lp_eval_lane4", "lp_eval_lane16", "lp_eval_group16", "lp_eval_group32", "lp_eval_wave",
                     "lp_eval_block1k", "lp_eval_block4k", "lp_eval_block8k"},
                    {"lp_refine_lane4", "lp_refine_lane16", "lp_refine_group16", "lp_refine_group32",
                     "lp_refine_wave", "lp_refine_block1k", "lp_refine_block4k", "lp_refine_block8k"}};
                ProfScope ps(kNames[A.refine][bk], eval_bytes(count, cslots[c0 + bk]), bs);
                const unsigned nb = static_cast<unsigned>(count);
                if (bk == 0) {
                    eval_lane_kernel<kLaneSmall><<<grid_for(count, 256), 256, 0, bs>>>(A);
                } else if (bk == 1) {
                    eval_lane_kernel<kLaneMax><<<grid_for(count, 256), 256, 0, bs>>>(A);
                } else if (dense) {  // refinement blocks: dense connection arrays
                    if (bk == 2) eval_dense_group_kernel<16><<<grid_for(count, 16), 256, 0, bs>>>(A);
                    else if (bk == 3) eval_dense_group_kernel<32><<<grid_for(count, 8), 256, 0, bs>>>(A);
                    else if (bk == 4) eval_dense_group_kernel<64><<<grid_for(count, 4), 256, 0, bs>>>(A);
                    else if (bk == 5) eval_dense_block_kernel<256><<<nb, 256, 0, bs>>>(A);
                    else if (bk == 6) eval_dense_block_kernel<512><<<nb, 512, 0, bs>>>(A);
                    else eval_dense_block_kernel<1024><<<nb, 1024, 0, bs>>>(A);
                } else if (bk == 2) {
                    eval_group_kernel<16, 2 * kG16Max><<<grid_for(count, 16), 256, 0, bs>>>(A);
                } else if (bk == 3) {
                    eval_group_kernel<32, 2 * kG32Max><<<grid_for(count, 8), 256, 0, bs>>>(A);
                } else if (bk == 4) {
                    eval_group_kernel<64, kWaveTable><<<grid_for(count, 4), 256, 0, bs>>>(A);
                } else if (bk == 5) {
                    eval_block_kernel<256, 2 * kBlock1Max><<<nb, 256, 0, bs>>>(A);
                } else if (bk == 6) {
                    eval_block_kernel<1024, 2 * kBlock2Max><<<nb, 1024, 0, bs>>>(A);
                } else {
                    if (tune.block_table == kBlockTablePow2)
                        eval_block_kernel<1024, kBlockTablePow2><<<nb, 1024, 0, bs>>>(A);
                    else
                        eval_block_kernel<1024, kBlockTable><<<nb, 1024, 0, bs>>>(A);
                }
                LAUNCHCHK();
            }
            if (side) evs.join(s);

            // colours below 2^16 entries: one entry per thread and pass, so
            // that every workgroup of the grid has work; larger ones keep
            // several loads in flight per thread
            const bool fine = ccount < (1 << 16);
            // per-target candidate weight and count, then admission: targets
            // that can take all their candidates admit them; the others
            // select the admitted prefix on the device
            {
                ProfScope ps(A.refine ? "lp_refine_admit" : "lp_admit", 0, s);
                const unsigned gc = capped_grid(ccount);
                auto accum = small ? (fine ? cand_accum_kernel<true, 1> : cand_accum_kernel<true, kAggChunk / 256>)
                                   : (fine ? cand_accum_kernel<false, 1> : cand_accum_kernel<false, kAggChunk / 256>);
                accum<<<gc, 256, 0, s>>>(ct.get(), cnodes, ccount, g.vw, tsum.get(), tcnt.get(), nw, ctr.get(), gate,
                                         rcnt.get() + r);
                LAUNCHCHK();
                auto admit = small ? (fine ? admit_kernel<true, 1> : admit_kernel<true, 16>)
                                   : (fine ? admit_kernel<false, 1> : admit_kernel<false, 16>);
                admit<<<gc, 256, 0, s>>>(ct.get(), cg.get(), ccount, w, tsum.get(), tcnt.get(), BB, ok.get(),
                                         slow_idx.get(), seg_off.get(), seg_list.get(), LS, small_max, nw, ctr.get(),
                                         gate);
                LAUNCHCHK();
            }
            {
                ProfScope ps(A.refine ? "lp_refine_admit_select" : "lp_admit_select", 0, s);
                const unsigned gc = capped_grid(ccount);
                auto scatter = small ? (fine ? scatter_kernel<true, 1> : scatter_kernel<true, kAggChunk / 256>)
                                     : (fine ? scatter_kernel<false, 1> : scatter_kernel<false, kAggChunk / 256>);
                scatter<<<gc, 256, 0, s>>>(slow_idx.get(), cnodes, ct.get(), cg.get(), g.vw, bits_v, nw, seg_off.get(),
                                           seg_fill.get(), skey.get(), swt.get(), ctr.get());
                LAUNCHCHK();
                select_kernel<<<kMaxBlocks, 256, 0, s>>>(seg_list.get(), seg_off.get(), seg_fill.get(), tcnt.get(), w,
                                                         BB, bits_v, skey.get(), swt.get(), bnd.get(), small_max,
                                                         ctr.get());
                LAUNCHCHK();
                // a target has at most ccount candidates: no large segment
                // unless the colour has more than the single-workgroup limit
                if (ccount > small_max) {
                    for (int launch = 0; launch < sel_launches; ++launch) {
                        large_pass_kernel<<<kLargeBlocks, kLargeThreads, 0, s>>>(
                            LS, launch, sel_launches, bits_v, skey.get(), swt.get(), bnd.get(), ctr.get());
                        LAUNCHCHK();
                    }
                }
            }
            if (trace) {
                HIPCHK(hipMemcpyAsync(hctr, ctr.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                fprintf(stderr, "[sclap] %s L%d r%d s%d n=%lld cand=%u slow=%u targets=%u gain=[%d,%d] hubs=%d\n",
                        phase != kCluster ? "refine" : "cluster", level, r, sc, static_cast<long long>(ccount),
                        hctr->ncand, hctr->nslow, hctr->nseg, hctr->nslow ? hctr->gmin : 0,
                        hctr->nslow ? hctr->gmax : 0, plans[sc].count);
            }
            {
                ProfScope ps("lp_apply", 0, s);
                if (small) {
                    apply_kernel<true><<<capped_grid(ccount), 256, 0, s>>>(ct.get(), ok.get(), cnodes, ccount,
                                                                           cg.get(), bits_v, bnd.get(), g.vw, label,
                                                                           lab8.get(), lab16.get(), w, tsum.get(),
                                                                           tcnt.get(), nw, ctr.get(), gate);
                    LAUNCHCHK();
                } else {
                    apply_kernel<false><<<grid_for(ccount, 256), 256, 0, s>>>(ct.get(), ok.get(), cnodes, ccount,
                                                                              cg.get(), bits_v, bnd.get(), g.vw, label,
                                                                              lab8.get(), lab16.get(), w, tsum.get(),
                                                                              tcnt.get(), nw, ctr.get(), gate);
                    LAUNCHCHK();
                }
            }
            if (A.quiet) {
                ProfScope ps("lp_unquiet", 0, s);
                unquiet_kernel<<<grid_for(ccount, 256), 256, 0, s>>>(ct.get(), ok.get(), cnodes,
                                                                      static_cast<int32_t>(ccount), g.xadj, g.adj,
                                                                      A.quiet, gate, rcnt.get(), r, n);
                LAUNCHCHK();
            }
        }
        // a round without candidates moved nothing (the first candidate of
        // every target is always admitted) and ends the run; its count is
        // read while the next round runs
        HIPCHK(hipMemcpyAsync(hrc + r, rcnt.get() + r, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (!capture) {
            HIPCHK(hipEventRecord(rev.ev[r & 1], s));
            if (r > 0) finish_round(r - 1);
        }
    }
    s = caller;
    if (capture) {
        rounds_graph.run();  // launches the graph on the caller's stream and waits for it
        for (int32_t q = 0; q < rounds && !halted; ++q) {
            res.rounds_run = q + 1;
            res.moves += hrc[q];
            if (hrc[q] == 0) halted = true;
        }
    } else if (!halted && rounds > 0) {
        finish_round(rounds - 1);
    }
    res.visits = static_cast<int64_t>(res.rounds_run) * g.S;
    HIPCHK(hipStreamSynchronize(s));
    if (profiler().on) profiler().collect();
    return res;
}

}  // namespace sclap
