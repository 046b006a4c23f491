// Multilevel drivers and the host initial partitioner (Section 4.5), shared by
// the C ABI and the serving loop.
#pragma once

#include <chrono>

#include "graph_ops.hpp"
#include "sclap.h"

namespace sclap {

// Resolved sclap_options.
struct Opts {
    int32_t coarsen_rounds = 10;
    int32_t refine_rounds = 10;
    int32_t nsub = 4;
    int32_t divisor = 18;
    int32_t coarsest = 10000;
    int32_t max_levels = SCLAP_MAX_LEVELS;
    int32_t validate = 1;
    const int32_t* color_override = nullptr;
    int32_t vcycles = 1;
    int32_t degree_order = 0;
    int32_t bucket_mean = 0;  // contraction tuning
    int32_t initial = 0;      // 0: host greedy growing; 1: device label propagation from seeds
    LPTuning tune;
};

// Seed of multilevel cycle c (Section 4.4, Miscellanea: iterated V-cycles): the caller's
// seed for the first, H(seed, 4, c) for later ones.
uint64_t cycle_seed(uint64_t seed, int32_t cycle);

// Defaults for NULL; checks ranges (throws Error).
Opts resolve(const sclap_options* o);

// Device view of a caller graph with device pointers; reads S = xadj[n].
DevGraph dev_view(const sclap_graph* g, hipStream_t s);

// Validates (or only measures) a device graph: c(V) and max c(v).
void check_graph(const DevGraph& g, bool validate, int64_t* cV, int64_t* cmax, hipStream_t s);

// Lmax = T + floor(T * round(eps * 10^6) / 10^6), T = ceil(cV / k).
int64_t lmax_of(int64_t cV, int32_t k, double eps);
void check_k_eps(int32_t k, double eps);

// Greedy BFS growing of blocks 0..k-2 up to T, the rest in id order to the
// lightest block (host memory).  rows_sorted: rows ascend (skips a sort).
// adj_ranked: adj holds each neighbour's rank among the positive-degree nodes
// (core_ranks) instead of its id.  threads: host threads it may use (0: up
// to 16; callers that already run one graph per thread pass 1).
void host_initial_partition(int32_t n, const int64_t* xadj, const int32_t* adj, const int32_t* vw, int32_t k,
                            int64_t T, int32_t* part, bool rows_sorted = false, bool adj_ranked = false,
                            int32_t threads = 0);

// One graph: outputs part (device, n), cut and bw[k] (host); o.vcycles
// multilevel cycles.
int partition_impl(const DevGraph& g0, int32_t k, double eps, uint64_t seed, const Opts& o, int32_t* part_out,
                   int64_t* cut, int64_t* bw, sclap_stats* stats, hipStream_t s);

// A batch of graphs in one CSR (see sclap_partition_batch).
int partition_batch_impl(const DevGraph& g0, int32_t G, const int32_t* node_base, const int32_t* k,
                         const double* eps, const uint64_t* seed, const Opts& o, int32_t* part_out, int64_t* cut,
                         int64_t* bw, sclap_batch_stats* stats, hipStream_t s);

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t);

// Fastest candidate degree-bucket thresholds for one clustering round of g.
LPTuning autotune(const DevGraph& g, int32_t k, const Opts& o, hipStream_t s);

// Serving loop (server.hip); errors throw Error.
sclap_server* server_create(int32_t device, int64_t hbm_budget, int32_t slots, int32_t max_batch,
                            const sclap_options* opt);
uint64_t server_submit(sclap_server* sv, const sclap_graph* g, int32_t k, double eps, uint64_t seed);
int server_poll(sclap_server* sv, uint64_t id, int32_t timeout_ms, int32_t* done, int32_t* part, int64_t* cut,
                int64_t* block_w, sclap_request_info* info);
void server_destroy(sclap_server* sv);
// The server's batch-packing rule (see server.hip): how many of `count`
// queued requests one batch takes.
int32_t plan_batch(const int64_t* nodes, const int64_t* slots, const int64_t* footprint, int32_t count,
                   int64_t free_budget, int32_t max_batch, bool idle);

}  // namespace sclap
