/*
 * sclap.h: C ABI of the MI355X (gfx950) library for size-constrained label
 * propagation (SCLaP), cluster contraction and multilevel graph
 * partitioning, after Meyerhenke, Sanders and Schulz, "Parallel Graph
 * Partitioning for Complex Networks" (2014).
 *
 * Problem (Section 2.1, Basic concepts): an undirected graph
 * G = (V = {0..n-1}, E, c, w) with node weights c >= 0 and edge weights w >= 1
 * is split into k blocks V_0..V_{k-1} with c(V_b) <= Lmax, where
 * Lmax = (1+eps) * ceil(c(V)/k), minimising the cut, the total weight of the
 * edges whose ends lie in different blocks.
 *
 * Graph layout (all entry points): symmetric CSR.
 *   xadj   int64[n+1]  row offsets, xadj[0] = 0, non-decreasing
 *   adjncy int32[S]    neighbour ids (S = xadj[n]); no self-loops; each
 *                      undirected edge appears in both rows with equal weight
 *   vwgt   int32[n]    node weights c(v) >= 0, or NULL for all 1
 *   adjwgt int32[S]    edge weights w >= 1, or NULL for all 1
 * c(V) and the undirected edge-weight total must each be <= 2^31-1.
 *
 * Memory: entry points without a suffix take host pointers and copy to and
 * from the current HIP device.  Entry points ending in _dev take device
 * pointers for the graph and every per-node array, plus the hipStream_t
 * (passed as void*, NULL = the default stream) on which all work is
 * enqueued; scalar outputs and the k block weights are host pointers.  The
 * caller owns every buffer it passes and must size outputs to n (per-node)
 * and k (per-block).  The library keeps no pointer after a call returns,
 * except for graphs returned in sclap_graph_owned (free them with
 * sclap_graph_free).  A _dev call returns after its results are complete.
 *
 * Determinism: every output is a pure function of (graph, k, eps, seed and
 * the semantic options).  The tuning knobs in sclap_options (degree-bucket
 * thresholds, table sizes) never change a result.
 *
 * Status codes: SCLAP_OK (0); SCLAP_WARN_IMBALANCED (1): result returned but
 * some block exceeds Lmax; negative values are errors, after which outputs are
 * unspecified; sclap_last_error() then describes the error.
 */
#ifndef SCLAP_H
#define SCLAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCLAP_OK 0
#define SCLAP_WARN_IMBALANCED 1
#define SCLAP_ERR_INVALID (-1)       /* bad argument or malformed graph */
#define SCLAP_ERR_NOT_SYMMETRIC (-2) /* some edge (u,v,w) lacks its twin (v,u,w) */
#define SCLAP_ERR_OVERFLOW (-3)      /* c(V) or the edge-weight total exceeds 2^31-1 */
#define SCLAP_ERR_NO_MEMORY (-4)     /* device allocation failed */
#define SCLAP_ERR_HIP (-5)           /* a HIP runtime call failed */
#define SCLAP_ERR_BUSY (-6)          /* server queue full */

typedef struct {
    int32_t n;
    const int64_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;   /* NULL => all 1 */
    const int32_t* adjwgt; /* NULL => all 1 */
} sclap_graph;

/* A graph allocated by the library (host memory, or device memory when
 * on_device is 1); release with sclap_graph_free. */
typedef struct {
    int32_t n;
    int64_t S;
    int64_t* xadj;
    int32_t* adjncy;
    int32_t* vwgt;
    int32_t* adjwgt;
    int32_t on_device;
} sclap_graph_owned;

typedef struct {
    /* semantic options (change results) */
    int32_t coarsen_rounds;  /* label propagation rounds per clustering (default 10) */
    int32_t refine_rounds;   /* label propagation rounds per refinement (default 10) */
    int32_t subrounds;       /* hash-coloured sub-rounds per round, 1..16 (default 4) */
    int32_t cluster_divisor; /* W = floor(c(V) / (cluster_divisor * k)) (default 18) */
    int32_t coarsest_nodes;  /* stop coarsening at <= this many nodes (default 10000) */
    int32_t max_levels;      /* at most this many contractions, 0..64 (default 64) */
    int32_t validate;        /* 1: check the input graph first (default 1) */
    /* Replaces the hash colour of every node (values in [0, subrounds)) in
     * sclap_cluster, sclap_refine and their _dev variants only; host or device
     * memory to match the entry point; NULL = hash colours. */
    const int32_t* color_override;
    /* tuning knobs (never change results; 0 = library default) */
    int32_t lane_max_degree;  /* rows up to this degree: one lane per node */
    int32_t wave_max_degree;  /* up to this: one wave64 per node, LDS table */
    int32_t block_max_degree; /* up to this: one workgroup per node, LDS table; above: hub path */
    int32_t hub_part_limit;   /* hub label partitions summed in LDS up to this many entries */
    int32_t hub_region_cap;   /* entries a hub partition keeps before spilling to its overflow list */
    int32_t select_small_max; /* overflowing targets with more candidates: multi-workgroup selection */
    int32_t skip_quiet;       /* 1: once few nodes move, skip nodes that emitted nothing, had no
                                 neighbouring label stronger than their own and saw no neighbour move
                                 since (their decision is unchanged); -1: evaluate every node;
                                 0: on for batches, off for single graphs */
    int32_t vcycles;          /* multilevel cycles (Section 4.4, iterated V-cycles; 0 counts as 1,
                                 at most 64): every cycle after the first clusters only inside the
                                 blocks of the previous result, so no cut edge is contracted, and
                                 starts refinement from that result on its coarsest graph; cycle c
                                 uses the seed H(seed, 4, c) for c >= 1.  The last result is
                                 returned.  Default 1. */
    int32_t degree_order;     /* 1: clustering visits nodes by increasing degree (Section 3.1;
                                 Section 4.1, coarsening only): the nodes with neighbours are ranked
                                 by (degree, id) and cut into `subrounds` equal consecutive groups,
                                 group s forming sub-round s (degree-0 nodes: sub-round 0); the
                                 degree counts the neighbours looked at.  Used by sclap_cluster*
                                 when color_override is NULL, and by every multilevel entry point.
                                 0 (default): hash colours. */
    int32_t contract_bucket_mean; /* tuning (never changes results; 0 = 1024): merged entries per
                                     bucket when contraction merges very long coarse rows by buckets */
    int32_t initial_partitioner;  /* 0 (default): host greedy growing (sclap_initial_partition);
                                     1: on the device, label propagation from seeds: the
                                     min(k, #nodes with neighbours) nodes with neighbours of smallest
                                     (H(seed, 5, level, v), v) start blocks 0.., all others start in a
                                     pool label k that is never eligible and always overloaded; then
                                     refine_rounds rounds under Lmax with k + 1 labels and hash
                                     phase 2; nodes left in the pool fill the blocks' remaining room
                                     max(0, T - w(b)) in id and block order.  Needs Lmax and c(V)
                                     below 2^30; single-graph entry points only. */
    int32_t select_launches;      /* tuning (never changes results; 0 = library default): launches of
                                     the multi-workgroup selection per sub-round, one key digit each;
                                     keys with more digits finish in the last launch */
    int32_t graph_capture;        /* tuning (never changes results): 1: every label-propagation call
                                     records all its rounds into one HIP graph and launches it once,
                                     with no host work between rounds; 0 (default) or -1: kernels are
                                     launched one by one, the host one round ahead of the device */
    int32_t fused_eval;           /* tuning (never changes results): 0 (default) or 1: a colour with
                                     fewer than 2^22 adjacency slots evaluates its buckets of up to
                                     1 024 slots per node in one launch; -1: one launch per bucket */
    int32_t block_table;          /* tuning (never changes results): entries of the LDS table of the
                                     workgroup-per-node bucket with the longest rows, 10240 (80 KB,
                                     probed modulo its size; 0 = 10240) or 16384 (128 KB) */
} sclap_options;

#define SCLAP_MAX_LEVELS 64

/* Per-call statistics (optional output). */
typedef struct {
    int32_t levels;                          /* contractions kept (L) */
    int64_t visits;                          /* adjacency slots scanned by node evaluation */
    int32_t level_n[SCLAP_MAX_LEVELS + 1];   /* nodes per level */
    int64_t level_S[SCLAP_MAX_LEVELS + 1];   /* adjacency slots per level */
    int32_t cluster_rounds[SCLAP_MAX_LEVELS + 1]; /* rounds executed per clustering */
    int32_t refine_rounds[SCLAP_MAX_LEVELS + 1];  /* rounds executed per refinement */
    double ms_coarsen;   /* wall time of clustering + contraction */
    double ms_initial;   /* coarsest-graph transfer + initial partition */
    double ms_refine;    /* projection + refinement */
    double ms_lp;        /* label propagation rounds only (cluster + refine) */
} sclap_stats;

/* Fills *opt with the defaults above.  Returns 0. */
int sclap_default_options(sclap_options* opt);

/* Message for the last non-zero status on this thread ("" if none). */
const char* sclap_last_error(void);

/*
 * Device memory: the library keeps blocks it freed on a stream for reuse by
 * later calls on that stream (at most a quarter of the device's memory).
 * sclap_trim_memory returns every cached block of the current device to the
 * device's memory pool; call it when the memory is needed elsewhere or before
 * destroying a stream that was passed to _dev calls.  Returns 0.
 */
int sclap_trim_memory(void);

/*
 * Input staging and validation (Section 2.1 problem statement): offsets
 * non-decreasing from 0, ids in range, no self-loops, w >= 1, c >= 0, both
 * totals <= 2^31-1, symmetric with equal weights.  The device variant tests
 * symmetry with an order-independent 64-bit hash of (u, v, w) over all slots
 * (a false pass has probability about 2^-64); the host variant checks it
 * exactly.  Returns 0, SCLAP_ERR_INVALID, SCLAP_ERR_NOT_SYMMETRIC or
 * SCLAP_ERR_OVERFLOW.
 */
int sclap_validate(const sclap_graph* g);
int sclap_validate_dev(const sclap_graph* g, void* stream);

/*
 * Size-constrained label propagation clustering (Section 3.1, Label
 * Propagation with Size Constraints): every node starts in its own cluster;
 * `rounds` rounds of hash-coloured sub-rounds move each node to the eligible
 * neighbouring cluster of strongest connection, where eligible means the
 * cluster stays within U; a round without moves ends the run early (the
 * result is the same as running all rounds).  `level` and `seed` key the
 * colour and tie-break hashes.  Outputs labels[n] (cluster ids in [0, n)) and
 * *rounds_run (may be NULL).
 */
int sclap_cluster(const sclap_graph* g, int64_t U, int32_t rounds, uint64_t seed, int32_t level,
                  const sclap_options* opt, int32_t* labels, int32_t* rounds_run);
int sclap_cluster_dev(const sclap_graph* g, int64_t U, int32_t rounds, uint64_t seed, int32_t level,
                      const sclap_options* opt, int32_t* labels, int32_t* rounds_run, void* stream);

/*
 * Clustering inside the blocks of a partition (Section 4.4, Iterated
 * Multilevel Schemes): as sclap_cluster, but a node only looks at the
 * neighbours u with block[u] == block[v], so it only joins clusters of its own
 * block and every cluster lies inside one block (contracting it keeps every
 * cut edge of the partition).  block[n]: any int32 values, same memory as the
 * other arrays of the call (host / device), read only.
 */
int sclap_cluster_within(const sclap_graph* g, const int32_t* block, int64_t U, int32_t rounds, uint64_t seed,
                         int32_t level, const sclap_options* opt, int32_t* labels, int32_t* rounds_run);
int sclap_cluster_within_dev(const sclap_graph* g, const int32_t* block, int64_t U, int32_t rounds,
                             uint64_t seed, int32_t level, const sclap_options* opt, int32_t* labels,
                             int32_t* rounds_run, void* stream);

/*
 * Cluster contraction (Section 3.1 contraction definition; Section 4.3
 * relabelling): labels[n] in [0, n) -> C[n] with C(v) = rank of label(v)
 * among the used labels, and the coarse graph (node weight = sum of members,
 * edge weight = total weight between two clusters, rows sorted by neighbour
 * id).  The coarse graph is allocated by the library: host memory for
 * sclap_contract, device memory for sclap_contract_dev.
 */
int sclap_contract(const sclap_graph* g, const int32_t* labels, int32_t* C, sclap_graph_owned* coarse);
int sclap_contract_dev(const sclap_graph* g, const int32_t* labels, int32_t* C, sclap_graph_owned* coarse,
                       void* stream);
void sclap_graph_free(sclap_graph_owned* g);

/* Uncoarsening (Section 3.1; Section 4.3): part[v] = coarse_part[C[v]] for
 * v < n; C values must lie in [0, n_coarse) (checked). */
int sclap_project(int32_t n, int32_t n_coarse, const int32_t* C, const int32_t* coarse_part, int32_t* part);
int sclap_project_dev(int32_t n, int32_t n_coarse, const int32_t* C, const int32_t* coarse_part, int32_t* part,
                      void* stream);

/*
 * SCLaP as local search (Section 3.1, last paragraph; Section 4.5): improves
 * part[n] (in/out, blocks in [0, k)) for `rounds` rounds with block bound
 * Lmax; a node of an overloaded block moves to the best eligible
 * neighbouring block even at a loss.
 */
int sclap_refine(const sclap_graph* g, int32_t k, int64_t Lmax, int32_t rounds, uint64_t seed, int32_t level,
                 const sclap_options* opt, int32_t* part, int32_t* rounds_run);
int sclap_refine_dev(const sclap_graph* g, int32_t k, int64_t Lmax, int32_t rounds, uint64_t seed,
                     int32_t level, const sclap_options* opt, int32_t* part, int32_t* rounds_run, void* stream);

/* Objective and balance (Section 2.1): *cut = total weight of edges between
 * blocks, block_w[k] = c(V_b). */
int sclap_cut(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w);
int sclap_cut_dev(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w,
                  void* stream);

/*
 * sclap_cut_dev without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): same arguments, results and errors as
 * sclap_cut_dev, but every temporary lives in a fixed 16 MiB workspace that
 * the library image holds on each device it runs on (until the process
 * ends).  Limits: k <= 65536 and at most 3,932,159 tiles of 2048 adjacency
 * slots (about 8 * 10^9 slots); larger inputs return SCLAP_ERR_INVALID
 * before any work.  The call allocates nothing; calls that overlap on one
 * device share the workspace and race (serialise them, e.g. on one stream).
 */
int sclap_cut_dev_noalloc(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w,
                          void* stream);

/*
 * Host initial partition of a (coarsest) graph, the plain routine used in
 * place of the paper's evolutionary algorithm (Section 4.5): greedy
 * breadth-first growing of blocks 0..k-2 up to T = ceil(c(V)/k) each, then
 * the remaining nodes in id order to the lightest block.  Host memory.
 * Returns SCLAP_ERR_NOT_SYMMETRIC if a neighbour id is out of range or
 * belongs to a node without neighbours.
 */
int sclap_initial_partition(const sclap_graph* g, int32_t k, int32_t* part);

/*
 * The device initial partitioner (see sclap_options.initial_partitioner): label
 * propagation from the hashed seeds of `level` and `seed` with a pool label,
 * `rounds` rounds under Lmax (options: subrounds and tuning knobs), then the
 * pool fills the remaining room up to T.  Device memory; part[n] receives
 * blocks in [0, k); *visits (may be NULL) the adjacency slots evaluated.
 */
int sclap_initial_partition_lp_dev(const sclap_graph* g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed,
                                   int32_t level, int32_t rounds, const sclap_options* opt, int32_t* part,
                                   int64_t* visits, void* stream);

/* Lmax = T + floor(T * round(eps * 10^6) / 10^6), T = ceil(cV / k). */
int64_t sclap_lmax(int64_t cV, int32_t k, double eps);

/*
 * Multilevel partitioning (Section 4.5): cluster + contract while the graph
 * has more than coarsest_nodes nodes (a level is kept only if it shrinks;
 * coarsening continues only after a shrink of at least 5%), initial partition
 * of the coarsest graph, then projection and refinement on every level.
 * Outputs part[n], *cut, block_w[k]; stats may be NULL.  Returns 0 or
 * SCLAP_WARN_IMBALANCED or an error.
 */
int sclap_partition(const sclap_graph* g, int32_t k, double eps, uint64_t seed, const sclap_options* opt,
                    int32_t* part, int64_t* cut, int64_t* block_w, sclap_stats* stats);
int sclap_partition_dev(const sclap_graph* g, int32_t k, double eps, uint64_t seed, const sclap_options* opt,
                        int32_t* part, int64_t* cut, int64_t* block_w, sclap_stats* stats, void* stream);

/*
 * Batched multilevel partitioning (the Section 4.5 algorithm applied to many
 * independent graphs at once).  The batch is one CSR holding `count` graphs:
 * graph i owns nodes [node_base[i], node_base[i+1]) (node_base: host array
 * of count+1 entries, node_base[0] = 0, node_base[count] = n) and every edge
 * joins two nodes of the same graph (checked when validating).  Graph i is
 * partitioned into k[i] blocks with eps[i] and seed[i]; its result is exactly
 * what sclap_partition returns for that graph alone with the same options:
 * every hash and order uses graph-local ids.  Each level runs every kernel
 * once for all graphs still coarsening.
 *   part[n]          graph-local block ids, per node of the batch
 *   cut[count]       host; cut of each graph
 *   block_w[sum k]   host; graph i's block weights start at k[0]+..+k[i-1]
 * Each graph's c(V) must be <= 2^31-1; when validating, so must the totals of
 * the whole batch.  Returns 0, SCLAP_WARN_IMBALANCED (some graph has a block
 * above its Lmax) or an error.
 */
typedef struct {
    int32_t levels;        /* most contractions kept by any graph */
    int64_t visits;        /* adjacency slots scanned by node evaluation, whole batch */
    double ms_coarsen;     /* clustering + contraction of all levels */
    double ms_initial;     /* coarsest-graph transfers + host initial partitions */
    double ms_refine;      /* projection + refinement */
    double ms_lp;          /* label propagation rounds only */
    int32_t* graph_levels; /* optional caller array [count]: contractions kept per graph, or NULL */
} sclap_batch_stats;

int sclap_partition_batch(const sclap_graph* g, int32_t count, const int32_t* node_base, const int32_t* k,
                          const double* eps, const uint64_t* seed, const sclap_options* opt, int32_t* part,
                          int64_t* cut, int64_t* block_w, sclap_batch_stats* stats);
int sclap_partition_batch_dev(const sclap_graph* g, int32_t count, const int32_t* node_base, const int32_t* k,
                              const double* eps, const uint64_t* seed, const sclap_options* opt, int32_t* part,
                              int64_t* cut, int64_t* block_w, sclap_batch_stats* stats, void* stream);

/*
 * Serving: continuous batching of partition requests on one GPU (the batched
 * partitioner above behind a request queue).  sclap_server_submit copies the
 * request's host graph into the server and queues it; `slots` worker threads,
 * each with its own HIP stream, repeatedly take the longest queue prefix
 * (at most max_batch graphs) whose device-memory footprint fits the free part
 * of hbm_budget and partition it as one batch, so requests that arrive while
 * others run are admitted as soon as a slot and memory are free, and their
 * work overlaps on the device.  Footprint of a request: 64 B per node plus
 * 64 B per adjacency slot plus 4 MiB; a request larger than the budget is
 * refused (SCLAP_ERR_NO_MEMORY), a full queue returns SCLAP_ERR_BUSY.  Each
 * result equals sclap_partition of that graph alone with the server's options.
 *
 * sclap_server_create: device index, hbm_budget in bytes (<= 0: 80% of the
 * device memory free at creation), slots in 1..16, max_batch >= 1; returns
 * NULL on error (see sclap_last_error).
 * sclap_server_poll: waits up to timeout_ms (0: no wait, < 0: until done);
 * *done = 0 while the request runs (nothing written), else writes part[n],
 * *cut, block_w[k] (host; any may be NULL) and info (may be NULL), releases
 * the request and returns its status (a request's errors are reported here).
 * sclap_server_destroy waits for running batches and drops queued requests;
 * no other call on the server may run concurrently with it.  The other calls
 * are thread-safe.
 */
typedef struct sclap_server sclap_server;

typedef struct {
    double submit_ms;   /* times since the server's creation */
    double start_ms;    /* batch taken up by a worker */
    double done_ms;     /* results stored */
    int32_t batch_size; /* graphs in the request's batch */
    int32_t reserved;
} sclap_request_info;

sclap_server* sclap_server_create(int32_t device, int64_t hbm_budget, int32_t slots, int32_t max_batch,
                                  const sclap_options* opt);
int sclap_server_submit(sclap_server* sv, const sclap_graph* g, int32_t k, double eps, uint64_t seed,
                        uint64_t* req);
int sclap_server_poll(sclap_server* sv, uint64_t req, int32_t timeout_ms, int32_t* done, int32_t* part,
                      int64_t* cut, int64_t* block_w, sclap_request_info* info);
void sclap_server_destroy(sclap_server* sv);

/*
 * The server's batch-packing rule, for callers that form their own batches
 * (and for tests): of `count` queued requests with the given node counts,
 * adjacency slot counts and footprints (host arrays, in queue order), one
 * batch takes the longest prefix, at most max_batch, whose summed footprint
 * fits free_budget (idle != 0: nothing else runs, so the first request is
 * taken whatever its footprint) and whose summed node count stays within
 * 2^31-1 (the batch's node ids are int32).  slots is read by no rule yet.
 * Returns the number taken, or SCLAP_ERR_INVALID.
 */
int32_t sclap_server_plan_batch(const int64_t* nodes, const int64_t* slots, const int64_t* footprint, int32_t count,
                                int64_t free_budget, int32_t max_batch, int32_t idle);

/*
 * Tuning (result-free): searches the tuning options for the device graph g
 * (normally a batch union, with k a representative block count) and writes
 * the choice into opt's tuning fields (lane_max_degree, wave_max_degree,
 * block_max_degree, graph_capture, block_table).  The objective is the measured time of one
 * clustering round from singletons (cluster bound from k as in
 * sclap_partition) plus one refinement round of a k-way partition, the faster
 * of two timings.  The degree thresholds decide which kernel and LDS table a
 * row gets (registers of one lane; 64-, 128- or 512-entry tables for 16, 32
 * or 64 lanes; 2048-, 8192- or 10240-entry tables for a workgroup; hub chunks
 * above), so the search sizes the tables by degree range; it also tries the
 * other table size of the longest-row workgroup bucket (block_table).
 * Coordinate search from the library defaults: capture, then block, wave and
 * lane thresholds, then the table size; a value is kept only if it is at
 * least 3 % faster.  Semantic fields of opt
 * are read, not changed; results of later calls do not depend on the choice.
 */
int sclap_autotune_dev(const sclap_graph* g, int32_t k, sclap_options* opt, void* stream);

/*
 * Instrumentation.  sclap_profile_begin() starts timing every kernel launch
 * that later calls on this thread issue, with HIP events recorded on the
 * launching stream around each launch; sclap_profile_end() stops, writes up to
 * `capacity` per-kernel totals to out (launch count, summed event time, and
 * the algorithmic bytes the launches must move: for node evaluation 24 per
 * evaluated node (row offsets, label, node weight, one label weight) and 12
 * per adjacency slot (neighbour id, edge weight, neighbour label)), sets
 * *count and clears the totals.  Timing adds event records (each one costs
 * device time between launches) but does not change any result.
 */
typedef struct {
    char name[48];
    int64_t launches;
    double ms;
    double bytes;
} sclap_kernel_stat;

int sclap_profile_begin(void);
int sclap_profile_end(sclap_kernel_stat* out, int32_t capacity, int32_t* count);

/*
 * Measurement helper: the rate at which the neighbour labels of the device
 * graph g can be gathered, the access that bounds node evaluation (Section
 * 3.1: a node scans the labels of all its neighbours).  Runs reps passes of a
 * kernel that sums label[adj[e]] over every slot (label_bytes 4: int32 labels,
 * as in clustering; 1: byte labels, as in refinement with at most 256 blocks)
 * with several loads in flight per thread, after one warm-up pass, and writes
 * the average pass time in milliseconds to *ms.  Allocates n label entries.
 */
int sclap_gather_probe_dev(const sclap_graph* g, int32_t label_bytes, int32_t reps, double* ms, void* stream);

/*
 * Same as sclap_profile_begin, but only launches of the kernel named `name`
 * (a name that sclap_profile_end reports, copied) get events; every other
 * launch runs as with profiling off.  NULL or "" times every kernel.  For
 * timing one kernel inside a measured run without the cost of events around
 * all the others.
 */
int sclap_profile_begin_only(const char* name);

#ifdef __cplusplus
}
#endif
#endif /* SCLAP_H */
