/*
 * CPU oracle for size-constrained label propagation (SCLaP), cluster
 * contraction and the multilevel partitioner of Meyerhenke, Sanders and
 * Schulz, "Parallel Graph Partitioning for Complex Networks" (2014).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Semantics (all integer; see each function for the passage it follows):
 *   - graph G = (V = {0..n-1}, E, c, w), symmetric CSR, no self-loops,
 *     c(v) >= 0, w(e) >= 1, c(V) and the undirected edge-weight total each
 *     fit in a signed 32-bit integer (Section 2.1, Basic concepts);
 *   - a round visits the nodes in sub-rounds s = 0..nsub-1; sub-round s
 *     evaluates every node of colour s against the state at the start of the
 *     sub-round, then admits moves per target in (gain desc, node asc) order
 *     while the target stays within the bound, then applies them;
 *   - colours and tie-break priorities come from a SplitMix64-based hash.
 *
 * Status codes: 0 ok, 1 result returned but some block exceeds Lmax,
 * -1 invalid argument, -2 graph not symmetric, -3 weight overflow.
 */
#ifndef SCLAP_ORACLE_H
#define SCLAP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;
    const int64_t* xadj;   /* [n+1] */
    const int32_t* adjncy; /* [xadj[n]] */
    const int32_t* vwgt;   /* [n] or NULL (all 1) */
    const int32_t* adjwgt; /* [xadj[n]] or NULL (all 1) */
} orc_graph;

enum { ORC_CLUSTER = 0, ORC_REFINE = 1, ORC_INITIAL = 2 };

/* Hash: SplitMix64 output function of z + 0x9E3779B97F4A7C15, chained. */
uint64_t orc_mix(uint64_t z);
uint64_t orc_hash(const uint64_t* words, int32_t nwords);
int32_t orc_color(uint64_t seed, int32_t level, int32_t phase, int32_t v, int32_t nsub);
uint64_t orc_tie(uint64_t seed, int32_t level, int32_t phase, int32_t round, int32_t x);

/* Bounds (Section 2.1 balance constraint; Section 3.1 cluster bound). */
int64_t orc_lmax(int64_t cV, int32_t k, double eps);
int64_t orc_cluster_bound(const orc_graph* g, int32_t k, int32_t divisor);

int32_t orc_validate(const orc_graph* g);

/* Evaluation of one node against a frozen state (Section 3.1). */
typedef struct {
    int32_t emit;        /* 1 if v proposes a move */
    int32_t target;      /* best eligible neighbouring label, -1 if none */
    int64_t gain;        /* conn(target) - conn(own label) */
    int64_t conn_target;
    int64_t conn_own;
    int32_t over;        /* own block overloaded (refinement only) */
} orc_eval;

int32_t orc_eval_node(const orc_graph* g, int32_t phase, int32_t level, int32_t round, uint64_t seed,
                      int64_t bound, const int32_t* label, const int64_t* w, int32_t v, orc_eval* out);
/* The same with block[n] != NULL: only neighbours u with block[u] == block[v]
 * count (clustering inside the blocks of a partition, Section 4.4). */
int32_t orc_eval_node_within(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level,
                             int32_t round, uint64_t seed, int64_t bound, const int32_t* label, const int64_t* w,
                             int32_t v, orc_eval* out);

/* One sub-round: evaluate colour `sub`, admit, apply.  Returns #moves.
 * Optional outputs: visits (+= degrees of evaluated nodes), ncand (+= #candidates). */
int64_t orc_subround(const orc_graph* g, int32_t phase, int32_t level, int32_t round, int32_t sub,
                     int32_t nsub, uint64_t seed, int64_t bound, const int32_t* color_override,
                     int32_t* label, int64_t* w, int64_t* visits, int64_t* ncand);
int64_t orc_subround_within(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level,
                            int32_t round, int32_t sub, int32_t nsub, uint64_t seed, int64_t bound,
                            const int32_t* color_override, int32_t* label, int64_t* w, int64_t* visits,
                            int64_t* ncand);
/* orc_subround (hash colours, no block array) with the node evaluation on
 * `threads` OpenMP threads; admission and apply stay sequential, so the result
 * is identical.  For the CPU baseline on all cores. */
int64_t orc_subround_par(const orc_graph* g, int32_t phase, int32_t level, int32_t round, int32_t sub, int32_t nsub,
                         uint64_t seed, int64_t bound, int32_t* label, int64_t* w, int64_t* visits, int32_t threads);
/* Threads OpenMP would use by default (1 without OpenMP). */
int32_t orc_max_threads(void);

int32_t orc_cluster(const orc_graph* g, int64_t U, int32_t rounds, int32_t nsub, uint64_t seed,
                    int32_t level, const int32_t* color_override, int32_t* labels, int32_t* rounds_run,
                    int64_t* visits);

/* Clustering inside the blocks of block[n] (Section 4.4, Iterated Multilevel
 * Schemes); visits counts only the same-block slots looked at. */
int32_t orc_cluster_within(const orc_graph* g, const int32_t* block, int64_t U, int32_t rounds, int32_t nsub,
                           uint64_t seed, int32_t level, const int32_t* color_override, int32_t* labels,
                           int32_t* rounds_run, int64_t* visits);

int32_t orc_refine(const orc_graph* g, int32_t k, int64_t Lmax, int32_t rounds, int32_t nsub, uint64_t seed,
                   int32_t level, const int32_t* color_override, int32_t* part, int32_t* rounds_run,
                   int64_t* visits);

/* Contraction (Section 3.1, Section 4.3).  Output buffers: C[n], cxadj[n+1],
 * cadj[S], cadjw[S], cvw[n] (the coarse graph never needs more). */
int32_t orc_contract(const orc_graph* g, const int32_t* labels, int32_t* C, int32_t* n_coarse,
                     int64_t* cxadj, int32_t* cadj, int32_t* cadjw, int32_t* cvw, int64_t* S_coarse);

void orc_project(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part);

int32_t orc_cut(const orc_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw);

int32_t orc_initial_partition(const orc_graph* g, int32_t k, int64_t T, int32_t* part);

typedef struct {
    int32_t coarsen_rounds;  /* 10 */
    int32_t refine_rounds;   /* 10 */
    int32_t subrounds;       /* 4 */
    int32_t cluster_divisor; /* 18 */
    int32_t coarsest_nodes;  /* 10000 */
    int32_t max_levels;      /* 64 */
    int32_t vcycles;         /* 1: multilevel cycles, each after the first inside the previous blocks */
    int32_t degree_order;    /* 0; 1: clustering sub-rounds by increasing degree (orc_degree_colors) */
    int32_t initial;         /* 0: orc_initial_partition; 1: orc_initial_partition_lp */
} orc_options;

/* Initial partition by label propagation from hashed seeds with a pool label
 * (see the definition in the source); phase 2 hashes.  Returns -1 unless
 * Lmax < 2^30 and c(V) < 2^30. */
int32_t orc_initial_partition_lp(const orc_graph* g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed,
                                 int32_t level, int32_t rounds, int32_t nsub, int32_t* part, int32_t* rounds_run,
                                 int64_t* visits);

/* Sub-round of every node for degree-ordered clustering (Section 3.1,
 * Section 4.1); block may be NULL. */
void orc_degree_colors(const orc_graph* g, const int32_t* block, int32_t nsub, int32_t* color);

uint64_t orc_cycle_seed(uint64_t seed, int32_t cycle);

#define ORC_MAX_LEVELS 64
typedef struct {
    int32_t levels;                         /* L: number of contractions kept */
    int64_t visits;                         /* adjacency slots scanned in evaluation */
    int32_t level_n[ORC_MAX_LEVELS + 1];
    int64_t level_S[ORC_MAX_LEVELS + 1];
    int32_t cluster_rounds[ORC_MAX_LEVELS + 1];
    int32_t refine_rounds[ORC_MAX_LEVELS + 1];
} orc_stats;

void orc_default_options(orc_options* o);

int32_t orc_partition(const orc_graph* g, int32_t k, double eps, uint64_t seed, const orc_options* opt,
                      int32_t* part, int64_t* cut, int64_t* bw, orc_stats* stats);

#ifdef __cplusplus
}
#endif
#endif
