// Graph-wide operations on gfx950: contraction, projection, cut and block
// weights, validation, range checks.
#pragma once

#include <vector>

#include "lp.hpp"

namespace sclap {

// A graph in device memory owned by the library.
struct OwnedDevGraph {
    int32_t n = 0;
    int64_t S = 0;
    DBuf<int64_t> xadj;
    DBuf<int32_t> adj;
    DBuf<int32_t> ew;
    DBuf<int32_t> vw;
    DevGraph view() const {
        DevGraph g;
        g.n = n;
        g.S = S;
        g.xadj = xadj.get();
        g.adj = adj.get();
        g.ew = ew.get();
        g.vw = vw.get();
        return g;
    }
};

// Contraction (Section 3.1; Section 4.3): labels in [0, n) -> C[n] and the
// coarse graph with sorted rows.  Always materialises coarse edge and node
// weights.
// probe (device, nprobe entries in [0, n]) optionally reports the coarse id
// base of label positions: probe_out[i] = number of used labels < probe[i].
// sorted = false leaves each coarse row's distinct neighbours in an unspecified
// order (label propagation and contraction do not depend on row order).
// bucket_mean (tuning, 0 = default): merged entries per bucket when long rows
// are merged unsorted.
void contract(const DevGraph& g, const int32_t* labels, int32_t* C, OwnedDevGraph& coarse, hipStream_t s,
              const int32_t* probe = nullptr, int32_t nprobe = 0, int32_t* probe_out = nullptr, bool sorted = true,
              int32_t bucket_mean = 0);

// Orders every row of g by neighbour id (rows hold distinct neighbours).
void sort_rows(OwnedDevGraph& g, hipStream_t s);

// part[v] = coarse_part[C[v]]
void project(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part, hipStream_t s);

// cut (host out) and block weights bw[k] (host out).
void cut_and_weights(const DevGraph& g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw, hipStream_t s);
// The same without allocating device memory: a fixed per-device workspace in
// the library image (k <= 65536, at most 3,932,159 slot tiles of 2048); checks
// part values itself.  Overlapping calls on one device race.
void cut_and_weights_noalloc(const DevGraph& g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw,
                             hipStream_t s);

// Checks CSR structure, ranges, weights, totals and symmetry (hash test).
// Returns 0 or a negative status.  Also reports c(V) and max c(v).
int validate_graph(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s);

// c(V) and max_v c(v) without validation.
void node_weight_stats(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s);

// True iff every value of a[0..count) lies in [lo, hi).
bool all_in_range(const int32_t* a, int64_t count, int32_t lo, int32_t hi, hipStream_t s);
// Average time (ms) of a pass that gathers one 1- or 4-byte label per slot
// of g (label[adj[e]]), over reps passes after one warm-up.
float gather_probe(const DevGraph& g, int32_t label_bytes, int32_t reps, hipStream_t s);

// Several disjoint graphs in one CSR.  Member m owns nodes [nb[m], nb[m+1])
// and slots [sb[m], sb[m+1]); ids[m] is its index in the caller's batch.

// gid[v] = ids[m] for the member m holding v.
void member_ids(int32_t n, const std::vector<int32_t>& nb, const std::vector<int32_t>& ids, int32_t* gid,
                hipStream_t s);
// sb[m] = xadj[nb[m]] for every entry of nb (host result).
std::vector<int64_t> member_slot_bases(const int64_t* xadj, const std::vector<int32_t>& nb, hipStream_t s);
// True iff every slot's neighbour lies in the slot owner's member.
bool members_closed(const DevGraph& g, const std::vector<int32_t>& nb, const std::vector<int64_t>& sb,
                    hipStream_t s);
// Per graph c(V_g) and max c(v) over its nodes (host arrays of G entries).
void graph_node_stats(int32_t n, const int32_t* gid, const int32_t* vw, int32_t G, int64_t* cV, int64_t* cmax,
                      hipStream_t s);
// Per graph cut of part (host array of G entries).
void graph_cuts(const DevGraph& g, const int32_t* part, const int32_t* gid, int32_t G, int64_t* cut, hipStream_t s);
// dst = the members of src with old bases (onb, osb), placed at (nnb, nsb);
// neighbour ids move with their member.  src must carry node and edge weights.
void compact_members(const DevGraph& src, const std::vector<int32_t>& onb, const std::vector<int64_t>& osb,
                     const std::vector<int32_t>& nnb, const std::vector<int64_t>& nsb, OwnedDevGraph& dst,
                     hipStream_t s);
// The members of src with old bases (onb, osb) packed for a host copy:
// member m's nnb[m+1] - nnb[m] nodes at [nnb[m], ...) of vw (if src.vw),
// its row offsets (starting at 0) at [nnb[m] + m, ... + nm] of x, and its
// slots at [nsb[m], nsb[m+1]) of adj, each neighbour given as its rank among
// the member's nodes of positive degree (-1 for a neighbour without
// neighbours, which only an asymmetric graph has).  x holds n_new + Mk
// entries.  Synchronises.
void pack_members_for_host(const DevGraph& src, const std::vector<int32_t>& onb, const std::vector<int64_t>& osb,
                           const std::vector<int32_t>& nnb, const std::vector<int64_t>& nsb, int64_t* x,
                           int32_t* adj, int32_t* vw, hipStream_t s);
// dst[onb[m] + i - nnb[m]] = src[i] for every packed node i (device arrays;
// dnb holds nnb[0..Mk] then onb[0..Mk-1]).
void unpack_members(const int32_t* src, int32_t n_new, int32_t Mk, const int32_t* dnb, int32_t* dst, hipStream_t s);
// C[v] += delta[gid[v]], or -1 where delta is INT_MIN (graph dropped).
void remap_members(int32_t n, const int32_t* gid, const std::vector<int32_t>& delta, int32_t* C, hipStream_t s);
// part[v] = coarse_part[C[v]] where C[v] >= 0.
// The subgraph of the slots u->v with blk[u] == blk[v], slot order kept
// (clustering inside the blocks of a partition, Section 4.4, Iterated Multilevel Schemes).  out.vw is left
// empty: the caller pairs out's view with g.vw.
void within_blocks(const DevGraph& g, const int32_t* blk, OwnedDevGraph& out, hipStream_t s);

// cblk[C[v]] = blk[v] for every v with C[v] >= 0 (a coarse node lies in the
// block of its members).
void inherit_blocks(int32_t n, const int32_t* C, const int32_t* blk, int32_t* cblk, hipStream_t s);

// Sub-round of every node for degree-ordered clustering (Section 3.1;
// Section 4.1): per graph, nodes with neighbours ranked by (degree, id) and
// cut into nsub equal groups; degree-0 nodes get 0.  Single graph: gid,
// gbase and gcount null.  Batch: gid[n] is the graph of each node, and graph
// gr's nodes are [gbase[gr], gbase[gr] + gcount[gr]) (device arrays of G
// entries; graph ranges in ascending graph order).
void degree_colors(const DevGraph& g, int32_t G, const int32_t* gid, const int32_t* gbase, const int32_t* gcount,
                   int32_t nsub, int32_t* color, hipStream_t s);

// out[e] = rank of adj[e] among the nodes of positive degree (ascending ids),
// -1 if adj[e] has no neighbours (not symmetric): the adjacency of the
// positive-degree core, renumbered (S entries).
void core_ranks(const DevGraph& g, int32_t* out, hipStream_t s);

// Initial partition by label propagation from hashed seeds with a pool label
// k (never eligible, always overloaded): seeds are the min(k, #nodes with
// neighbours) such nodes of smallest (H(seed, 5, level, v), v); `rounds`
// rounds under Lmax with k + 1 labels (phase kInitial); the nodes left in the
// pool fill the blocks' remaining room max(0, T - w(b)) in id and block order.
// Writes part[n] in [0, k); returns the label-propagation statistics.
LPResult device_initial_partition(const DevGraph& g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed, int32_t level,
                                  int32_t nsub, int32_t rounds, const LPTuning& tune, int32_t* part, hipStream_t s);

void project_kept(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part, hipStream_t s);
// part[v] += sign * add[gid[v]] (add: device array indexed by graph).
void shift_by_graph(int32_t n, const int32_t* gid, const int32_t* add, int32_t sign, int32_t* part, hipStream_t s);

}  // namespace sclap
