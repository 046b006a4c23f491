// Graph-wide operations on gfx950: contraction, projection, cut and block
// weights, validation, range checks.
#pragma once

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
void contract(const DevGraph& g, const int32_t* labels, int32_t* C, OwnedDevGraph& coarse, hipStream_t s);

// part[v] = coarse_part[C[v]]
void project(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part, hipStream_t s);

// cut (host out) and block weights bw[k] (host out).
void cut_and_weights(const DevGraph& g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw, hipStream_t s);

// Checks CSR structure, ranges, weights, totals and symmetry (hash test).
// Returns 0 or a negative status.  Also reports c(V) and max c(v).
int validate_graph(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s);

// c(V) and max_v c(v) without validation.
void node_weight_stats(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s);

// True iff every value of a[0..count) lies in [lo, hi).
bool all_in_range(const int32_t* a, int64_t count, int32_t lo, int32_t hi, hipStream_t s);

}  // namespace sclap
