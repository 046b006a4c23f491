/*
 * CPU oracle for SCLaP, cluster contraction and the multilevel partitioner
 * (Meyerhenke, Sanders, Schulz 2014).  TEST INFRASTRUCTURE ONLY: the plain,
 * single-threaded reference the GPU library is checked against.  It is written
 * for clarity, not speed, and shares no code with the GPU library.
 *
 * Readings of the paper adopted here (where it is silent, soft or
 * asynchronous) are those of the deterministic round semantics:
 *   - visit order: hash-coloured sub-rounds, Jacobi inside a sub-round;
 *   - random tie-break: a hash priority per label, then the label id;
 *   - staying is preferred unless a move strictly gains (or the own block
 *     is overloaded during refinement);
 *   - soft / approximate size bounds: strict admission per target in
 *     (gain desc, node asc) order against the start-of-sub-round weight;
 *   - eps is taken in parts per million, Lmax = T + floor(T * ppm / 10^6);
 *   - coarse node ids are the ranks of the used cluster labels, coarse rows
 *     are sorted by neighbour id.
 */
#include "sclap_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define I32MAX 2147483647LL

/* ------------------------------------------------------------------ hash */

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014) applied to
 * z + golden gamma. */
uint64_t orc_mix(uint64_t z) {
    z += GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* H(w0, ..., wj): h = mix(w0), then h = mix(h ^ wi). */
uint64_t orc_hash(const uint64_t* words, int32_t nwords) {
    uint64_t h = orc_mix(words[0]);
    for (int32_t i = 1; i < nwords; ++i) h = orc_mix(h ^ words[i]);
    return h;
}

/* Sub-round colour of node v: H(seed, 1, level, phase, v) mod nsub.  Fixed
 * per (level, phase).  Deterministic stand-in for the paper's random or
 * degree-ordered visiting order (Section 3.1, Section 4.1). */
int32_t orc_color(uint64_t seed, int32_t level, int32_t phase, int32_t v, int32_t nsub) {
    uint64_t w[5] = {seed, 1, (uint64_t)(uint32_t)level, (uint64_t)(uint32_t)phase, (uint64_t)(uint32_t)v};
    return (int32_t)(orc_hash(w, 5) % (uint64_t)nsub);
}

/* Tie-break priority of label x in round r: H(seed, 2, level, phase, r, x).
 * Replaces "ties are broken randomly" (Section 3.1). */
uint64_t orc_tie(uint64_t seed, int32_t level, int32_t phase, int32_t round, int32_t x) {
    uint64_t w[6] = {seed, 2, (uint64_t)(uint32_t)level, (uint64_t)(uint32_t)phase, (uint64_t)(uint32_t)round,
                     (uint64_t)(uint32_t)x};
    return orc_hash(w, 6);
}

/* --------------------------------------------------------------- helpers */

static int64_t node_w(const orc_graph* g, int32_t v) { return g->vwgt ? g->vwgt[v] : 1; }
static int64_t edge_w(const orc_graph* g, int64_t i) { return g->adjwgt ? g->adjwgt[i] : 1; }

static int64_t total_node_weight(const orc_graph* g) {
    int64_t s = 0;
    for (int32_t v = 0; v < g->n; ++v) s += node_w(g, v);
    return s;
}

/* Balance constraint (Section 2.1): Lmax = (1+eps) * ceil(c(V)/k), with eps
 * read in parts per million and the product floored. */
int64_t orc_lmax(int64_t cV, int32_t k, double eps) {
    int64_t T = (cV + k - 1) / k;
    int64_t ppm = llround(eps * 1e6);
    return T + (T * ppm) / 1000000;
}

/* Cluster size bound U = max(max_v c(v), W) (Section 3.1) with
 * W = floor(c(V) / (divisor * k)); the paper's W = Lmax / f is the same shape
 * with a different constant. */
int64_t orc_cluster_bound(const orc_graph* g, int32_t k, int32_t divisor) {
    int64_t cmax = 0;
    for (int32_t v = 0; v < g->n; ++v)
        if (node_w(g, v) > cmax) cmax = node_w(g, v);
    int64_t W = total_node_weight(g) / ((int64_t)divisor * k);
    return cmax > W ? cmax : W;
}

typedef struct { int64_t a, b, c; } trip;

static int cmp_trip(const void* x, const void* y) {
    const trip* p = (const trip*)x;
    const trip* q = (const trip*)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->c != q->c) return p->c < q->c ? -1 : 1;
    return 0;
}

/* Input rules (Section 2.1): weights, ranges, no self-loops, symmetric. */
int32_t orc_validate(const orc_graph* g) {
    if (!g || g->n < 0) return -1;
    if (g->n == 0) return 0;
    if (!g->xadj || g->xadj[0] != 0) return -1;
    for (int32_t v = 0; v < g->n; ++v)
        if (g->xadj[v + 1] < g->xadj[v]) return -1;
    int64_t S = g->xadj[g->n];
    if (S > 0 && !g->adjncy) return -1;
    int64_t cV = 0, wsum = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        if (node_w(g, v) < 0) return -1;
        cV += node_w(g, v);
    }
    for (int32_t v = 0; v < g->n; ++v)
        for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i) {
            int32_t u = g->adjncy[i];
            if (u < 0 || u >= g->n || u == v) return -1;
            if (edge_w(g, i) < 1) return -1;
            wsum += edge_w(g, i);
        }
    if (cV > I32MAX || wsum / 2 > I32MAX) return -3;
    /* symmetric as a multiset of (u, v, w) */
    trip* A = (trip*)malloc((size_t)(S > 0 ? S : 1) * sizeof(trip));
    trip* B = (trip*)malloc((size_t)(S > 0 ? S : 1) * sizeof(trip));
    int64_t j = 0;
    for (int32_t v = 0; v < g->n; ++v)
        for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i, ++j) {
            A[j].a = v; A[j].b = g->adjncy[i]; A[j].c = edge_w(g, i);
            B[j].a = g->adjncy[i]; B[j].b = v; B[j].c = edge_w(g, i);
        }
    qsort(A, (size_t)S, sizeof(trip), cmp_trip);
    qsort(B, (size_t)S, sizeof(trip), cmp_trip);
    int32_t st = 0;
    for (int64_t i = 0; i < S; ++i)
        if (cmp_trip(&A[i], &B[i]) != 0) { st = -2; break; }
    free(A);
    free(B);
    return st;
}

/* ------------------------------------------------------------ evaluation */

typedef struct { int32_t label; int64_t w; } lw_pair;

static int cmp_lw(const void* x, const void* y) {
    int32_t a = ((const lw_pair*)x)->label, b = ((const lw_pair*)y)->label;
    return (a > b) - (a < b);
}

/*
 * Evaluate node v (Section 3.1, Label Propagation with Size Constraints):
 *   conn(x) = total weight of edges from v to neighbours labelled x;
 *   a neighbouring label x != own label a is eligible iff w(x) + c(v) <= bound;
 *   the best eligible label maximises conn, ties broken by the hash priority
 *   tie(x) (smaller first) and then by the label id (smaller first);
 *   during refinement a node whose own block is overloaded (w(a) > bound)
 *   moves to the best eligible block regardless of its own block (the
 *   local-search rule); otherwise it moves only for a strictly positive gain.
 */
/*
 * With a block array (clustering inside the blocks of an input partition,
 * Section 4.4, Miscellanea: Iterated Multilevel Schemes), only neighbours in v's own block
 * are looked at: a cluster then never spans two blocks, so these are exactly
 * the clusters of v's block.
 */
static int in_block(const int32_t* block, int32_t v, int32_t u) { return !block || block[u] == block[v]; }

int32_t orc_eval_node_within(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level,
                             int32_t round, uint64_t seed, int64_t bound, const int32_t* label, const int64_t* w,
                             int32_t v, orc_eval* out) {
    memset(out, 0, sizeof(*out));
    out->target = -1;
    int32_t a = label[v];
    int64_t cv = node_w(g, v);
    int64_t b = g->xadj[v], e = g->xadj[v + 1], d = 0;
    out->over = (phase != ORC_CLUSTER && w[a] > bound) ? 1 : 0;
    if (e == b) return 0;
    lw_pair* P = (lw_pair*)malloc((size_t)(e - b) * sizeof(lw_pair));
    for (int64_t i = b; i < e; ++i) {
        if (!in_block(block, v, g->adjncy[i])) continue;
        P[d].label = label[g->adjncy[i]];
        P[d].w = edge_w(g, i);
        ++d;
    }
    qsort(P, (size_t)d, sizeof(lw_pair), cmp_lw);
    int32_t best = -1;
    int64_t best_conn = 0;
    int64_t conn_own = 0;
    for (int64_t i = 0; i < d;) {
        int32_t x = P[i].label;
        int64_t conn = 0;
        while (i < d && P[i].label == x) conn += P[i++].w;
        if (x == a) { conn_own = conn; continue; }
        if (w[x] + cv > bound) continue; /* not eligible */
        int better = 0;
        if (best < 0 || conn > best_conn) better = 1;
        else if (conn == best_conn) {
            uint64_t tx = orc_tie(seed, level, phase, round, x);
            uint64_t tb = orc_tie(seed, level, phase, round, best);
            better = (tx < tb) || (tx == tb && x < best);
        }
        if (better) { best = x; best_conn = conn; }
    }
    free(P);
    out->conn_own = conn_own;
    if (best < 0) return 0;
    out->target = best;
    out->conn_target = best_conn;
    out->gain = best_conn - conn_own;
    out->emit = (out->over || out->gain > 0) ? 1 : 0;
    return 0;
}

int32_t orc_eval_node(const orc_graph* g, int32_t phase, int32_t level, int32_t round, uint64_t seed,
                      int64_t bound, const int32_t* label, const int64_t* w, int32_t v, orc_eval* out) {
    return orc_eval_node_within(g, NULL, phase, level, round, seed, bound, label, w, v, out);
}

/* ------------------------------------------------------------- sub-round */

typedef struct { int32_t t; int64_t gain; int32_t v; int32_t from; int64_t c; } cand;

static int cmp_cand(const void* x, const void* y) {
    const cand* p = (const cand*)x;
    const cand* q = (const cand*)y;
    if (p->t != q->t) return p->t < q->t ? -1 : 1;
    if (p->gain != q->gain) return p->gain > q->gain ? -1 : 1; /* gain descending */
    return (p->v > q->v) - (p->v < q->v);                      /* node ascending */
}

/*
 * One sub-round.  Evaluate all nodes of colour `sub` against the frozen state,
 * then for each target admit the longest prefix of its candidates, in
 * (gain desc, node asc) order, that keeps w(target) <= bound, counting from
 * the target's weight at the start of the sub-round (departures in the same
 * sub-round are not credited).  Every block that started within the bound
 * therefore stays within it, which is the size constraint of Section 3.1.
 */
/* Candidate of node v in this sub-round (Section 3.1 rule, orc_eval_node). */
static int eval_candidate(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level, int32_t round,
                          uint64_t seed, int64_t bound, const int32_t* label, const int64_t* w, int32_t v, cand* out) {
    orc_eval ev;
    orc_eval_node_within(g, block, phase, level, round, seed, bound, label, w, v, &ev);
    if (!ev.emit) return 0;
    out->t = ev.target;
    out->gain = ev.gain;
    out->v = v;
    out->from = label[v];
    out->c = node_w(g, v);
    return 1;
}

/* For each target, admit the longest prefix of its candidates in
 * (gain desc, node asc) order that keeps w(target) <= bound, counted from the
 * target's weight at the start of the sub-round; then apply the moves. */
static int64_t admit_and_apply(cand* C, int64_t nc, int64_t bound, int32_t* label, int64_t* w) {
    qsort(C, (size_t)nc, sizeof(cand), cmp_cand);
    char* admit = (char*)calloc((size_t)(nc > 0 ? nc : 1), 1);
    for (int64_t i = 0; i < nc;) {
        int32_t t = C[i].t;
        int64_t sum = w[t];
        int stopped = 0;
        for (; i < nc && C[i].t == t; ++i) {
            if (!stopped && sum + C[i].c <= bound) {
                sum += C[i].c;
                admit[i] = 1;
            } else {
                stopped = 1;
            }
        }
    }
    int64_t moves = 0;
    for (int64_t i = 0; i < nc; ++i) {
        if (!admit[i]) continue;
        label[C[i].v] = C[i].t;
        w[C[i].t] += C[i].c;
        w[C[i].from] -= C[i].c;
        ++moves;
    }
    free(admit);
    return moves;
}

static int32_t color_of(const int32_t* color_override, uint64_t seed, int32_t level, int32_t phase, int32_t v,
                        int32_t nsub) {
    return color_override ? color_override[v] : orc_color(seed, level, phase, v, nsub);
}

/*
 * One sub-round.  Evaluate all nodes of colour `sub` against the frozen state,
 * then for each target admit the longest prefix of its candidates, in
 * (gain desc, node asc) order, that keeps w(target) <= bound, counting from
 * the target's weight at the start of the sub-round (departures in the same
 * sub-round are not credited).  Every block that started within the bound
 * therefore stays within it, which is the size constraint of Section 3.1.
 */
int64_t orc_subround_within(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level,
                            int32_t round, int32_t sub, int32_t nsub, uint64_t seed, int64_t bound,
                            const int32_t* color_override, int32_t* label, int64_t* w, int64_t* visits,
                            int64_t* ncand) {
    int32_t n = g->n;
    cand* C = (cand*)malloc((size_t)(n > 0 ? n : 1) * sizeof(cand));
    int64_t nc = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (color_of(color_override, seed, level, phase, v, nsub) != sub) continue;
        if (visits)
            for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i) *visits += in_block(block, v, g->adjncy[i]);
        nc += eval_candidate(g, block, phase, level, round, seed, bound, label, w, v, &C[nc]);
    }
    if (ncand) *ncand += nc;
    int64_t moves = admit_and_apply(C, nc, bound, label, w);
    free(C);
    return moves;
}

/*
 * The same sub-round with the evaluation spread over `threads` OpenMP
 * threads (the CPU baseline on all host cores).  Evaluation reads only the
 * frozen state, so the candidates are those of the sequential loop; they are
 * kept per node and gathered in node order, and admission and apply run
 * sequentially as above: the result is identical.
 */
int64_t orc_subround_par(const orc_graph* g, int32_t phase, int32_t level, int32_t round, int32_t sub, int32_t nsub,
                         uint64_t seed, int64_t bound, int32_t* label, int64_t* w, int64_t* visits, int32_t threads) {
    int32_t n = g->n;
    cand* P = (cand*)malloc((size_t)(n > 0 ? n : 1) * sizeof(cand));
    char* has = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t vis = 0;
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads) reduction(+ : vis)
    for (int32_t v = 0; v < n; ++v) {
        if (orc_color(seed, level, phase, v, nsub) != sub) continue;
        vis += g->xadj[v + 1] - g->xadj[v];
        has[v] = (char)eval_candidate(g, NULL, phase, level, round, seed, bound, label, w, v, &P[v]);
    }
    if (visits) *visits += vis;
    int64_t nc = 0;
    for (int32_t v = 0; v < n; ++v)
        if (has[v]) P[nc++] = P[v];
    int64_t moves = admit_and_apply(P, nc, bound, label, w);
    free(has);
    free(P);
    return moves;
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t orc_subround(const orc_graph* g, int32_t phase, int32_t level, int32_t round, int32_t sub,
                     int32_t nsub, uint64_t seed, int64_t bound, const int32_t* color_override,
                     int32_t* label, int64_t* w, int64_t* visits, int64_t* ncand) {
    return orc_subround_within(g, NULL, phase, level, round, sub, nsub, seed, bound, color_override, label, w,
                               visits, ncand);
}

/* Runs rounds of sub-rounds until `rounds` are done or a round moves nothing
 * (Section 3.1: at most l iterations, or until converged). */
static int32_t run_rounds(const orc_graph* g, const int32_t* block, int32_t phase, int32_t level, int32_t rounds,
                          int32_t nsub, uint64_t seed, int64_t bound, const int32_t* color_override, int32_t* label,
                          int64_t* w, int32_t* rounds_run, int64_t* visits) {
    int32_t rr = 0;
    for (int32_t r = 0; r < rounds; ++r) {
        int64_t moves = 0;
        for (int32_t s = 0; s < nsub; ++s)
            moves += orc_subround_within(g, block, phase, level, r, s, nsub, seed, bound, color_override, label, w,
                                         visits, NULL);
        rr = r + 1;
        if (moves == 0) break;
    }
    if (rounds_run) *rounds_run = rr;
    return 0;
}

/* Size-constrained clustering: every node starts in its own cluster (label =
 * node id), cluster weights w(x) = c(x) (Section 3.1).  With a block array,
 * a node only joins clusters of its own block (Section 4.4, Iterated
 * Multilevel Schemes): singletons lie in one block each, and only same-block
 * neighbours are looked at, so every cluster stays inside one block. */
int32_t orc_cluster_within(const orc_graph* g, const int32_t* block, int64_t U, int32_t rounds, int32_t nsub,
                           uint64_t seed, int32_t level, const int32_t* color_override, int32_t* labels,
                           int32_t* rounds_run, int64_t* visits) {
    if (!g || g->n < 0 || rounds < 0 || nsub < 1) return -1;
    int32_t n = g->n;
    int64_t* w = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) {
        labels[v] = v;
        w[v] = node_w(g, v);
    }
    run_rounds(g, block, ORC_CLUSTER, level, rounds, nsub, seed, U, color_override, labels, w, rounds_run, visits);
    free(w);
    return 0;
}

/* Degree-ordered sub-rounds (Section 3.1: visiting nodes by increasing
 * degree lets low-degree nodes settle first and improves quality and time;
 * Section 4.1: used while coarsening only).  The nodes with at least one
 * neighbour to look at are ranked by (degree, id), both ascending, and cut
 * into nsub consecutive groups of equal size (group s: ranks r with
 * floor(r * nsub / count) = s), group s forming sub-round s.  The degree
 * counts the neighbours the node looks at (same-block ones with a block
 * array).  Nodes with none never move and are put in sub-round 0. */
typedef struct { int64_t deg; int32_t v; } deg_node;

static int cmp_deg(const void* x, const void* y) {
    const deg_node* p = (const deg_node*)x;
    const deg_node* q = (const deg_node*)y;
    if (p->deg != q->deg) return p->deg < q->deg ? -1 : 1;
    return (p->v > q->v) - (p->v < q->v);
}

void orc_degree_colors(const orc_graph* g, const int32_t* block, int32_t nsub, int32_t* color) {
    int32_t n = g->n;
    deg_node* D = (deg_node*)malloc((size_t)(n > 0 ? n : 1) * sizeof(deg_node));
    int64_t cnt = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t d = 0;
        for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i) d += in_block(block, v, g->adjncy[i]);
        color[v] = 0;
        if (d > 0) {
            D[cnt].deg = d;
            D[cnt].v = v;
            ++cnt;
        }
    }
    qsort(D, (size_t)cnt, sizeof(deg_node), cmp_deg);
    for (int64_t r = 0; r < cnt; ++r) color[D[r].v] = (int32_t)(r * nsub / cnt);
    free(D);
}

int32_t orc_cluster(const orc_graph* g, int64_t U, int32_t rounds, int32_t nsub, uint64_t seed,
                    int32_t level, const int32_t* color_override, int32_t* labels, int32_t* rounds_run,
                    int64_t* visits) {
    return orc_cluster_within(g, NULL, U, rounds, nsub, seed, level, color_override, labels, rounds_run, visits);
}

/* SCLaP as local search on a k-way partition with bound Lmax (Section 3.1,
 * last paragraph; Section 4.5). */
int32_t orc_refine(const orc_graph* g, int32_t k, int64_t Lmax, int32_t rounds, int32_t nsub, uint64_t seed,
                   int32_t level, const int32_t* color_override, int32_t* part, int32_t* rounds_run,
                   int64_t* visits) {
    if (!g || g->n < 0 || k < 1 || rounds < 0 || nsub < 1) return -1;
    int64_t* w = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    for (int32_t v = 0; v < g->n; ++v) {
        if (part[v] < 0 || part[v] >= k) { free(w); return -1; }
        w[part[v]] += node_w(g, v);
    }
    run_rounds(g, NULL, ORC_REFINE, level, rounds, nsub, seed, Lmax, color_override, part, w, rounds_run, visits);
    free(w);
    return 0;
}

/* ----------------------------------------------------------- contraction */

/*
 * Contract a clustering (Section 3.1, contraction definition; Section 4.3):
 * each cluster becomes one coarse node of weight equal to the sum of its
 * members; the coarse edge between two clusters carries the total weight of
 * the fine edges between them; intra-cluster edges vanish.  Coarse ids:
 * q(x) = number of used labels smaller than x, C(v) = q(label(v)).
 */
int32_t orc_contract(const orc_graph* g, const int32_t* labels, int32_t* C, int32_t* n_coarse,
                     int64_t* cxadj, int32_t* cadj, int32_t* cadjw, int32_t* cvw, int64_t* S_coarse) {
    int32_t n = g->n;
    for (int32_t v = 0; v < n; ++v)
        if (labels[v] < 0 || labels[v] >= n) return -1;
    char* used = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t* q = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) used[labels[v]] = 1;
    int32_t nc = 0;
    for (int32_t x = 0; x < n; ++x) {
        q[x] = nc;
        nc += used[x];
    }
    for (int32_t v = 0; v < n; ++v) C[v] = q[labels[v]];
    for (int32_t i = 0; i < nc; ++i) cvw[i] = 0;
    for (int32_t v = 0; v < n; ++v) cvw[C[v]] += (int32_t)node_w(g, v);
    int64_t S = n > 0 ? g->xadj[n] : 0;
    trip* T = (trip*)malloc((size_t)(S > 0 ? S : 1) * sizeof(trip));
    int64_t m = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t i = g->xadj[u]; i < g->xadj[u + 1]; ++i) {
            int32_t cu = C[u], cv = C[g->adjncy[i]];
            if (cu == cv) continue;
            T[m].a = cu; T[m].b = cv; T[m].c = edge_w(g, i);
            ++m;
        }
    qsort(T, (size_t)m, sizeof(trip), cmp_trip);
    int64_t out = 0;
    for (int32_t i = 0; i <= nc; ++i) cxadj[i] = 0;
    for (int64_t i = 0; i < m;) {
        int64_t a = T[i].a, b = T[i].b, s = 0;
        while (i < m && T[i].a == a && T[i].b == b) s += T[i++].c;
        cadj[out] = (int32_t)b;
        cadjw[out] = (int32_t)s;
        cxadj[a + 1]++;
        ++out;
    }
    for (int32_t i = 0; i < nc; ++i) cxadj[i + 1] += cxadj[i];
    free(T);
    free(used);
    free(q);
    *n_coarse = nc;
    *S_coarse = out;
    return 0;
}

/* Uncoarsening (Section 3.1, Section 4.3): a fine node takes the block of its
 * coarse representative. */
void orc_project(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part) {
    for (int32_t v = 0; v < n; ++v) part[v] = coarse_part[C[v]];
}

/* Objective and block weights (Section 2.1): cut = sum over undirected edges
 * whose ends lie in different blocks; bw[b] = c(V_b). */
int32_t orc_cut(const orc_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw) {
    if (k < 1) return -1;
    for (int32_t b = 0; b < k; ++b) bw[b] = 0;
    int64_t s = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        if (part[v] < 0 || part[v] >= k) return -1;
        bw[part[v]] += node_w(g, v);
        for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i)
            if (part[g->adjncy[i]] != part[v]) s += edge_w(g, i);
    }
    *cut = s / 2;
    return 0;
}

/* --------------------------------------------------- initial partitioning */

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/*
 * Plain host initial partitioner for the coarsest graph (stands in for the
 * evolutionary algorithm of Section 2.3 / Section 4.5):
 *   1. for b = 0..k-2, grow block b by breadth-first search, each search
 *      seeded at the smallest unassigned node of positive degree that still
 *      fits, neighbours visited in ascending id order, a node taken iff
 *      w(b) + c(v) <= T; seeds are tried until no unassigned node of positive
 *      degree fits;
 *   2. every node still unassigned (isolated nodes included), in ascending id
 *      order, goes to the currently lightest block (lowest block id on ties).
 */
int32_t orc_initial_partition(const orc_graph* g, int32_t k, int64_t T, int32_t* part) {
    if (k < 1) return -1;
    int32_t n = g->n;
    int64_t* wb = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) {
        part[v] = -1;
        if (g->xadj[v + 1] - g->xadj[v] > maxd) maxd = g->xadj[v + 1] - g->xadj[v];
    }
    int32_t* nb = (int32_t*)malloc((size_t)(maxd > 0 ? maxd : 1) * sizeof(int32_t));
    for (int32_t b = 0; b + 1 < k; ++b) {
        for (int32_t s = 0; s < n; ++s) {
            if (part[s] >= 0 || g->xadj[s + 1] == g->xadj[s]) continue;
            if (wb[b] + node_w(g, s) > T) continue;
            part[s] = b;
            wb[b] += node_w(g, s);
            int32_t head = 0, tail = 0;
            queue[tail++] = s;
            while (head < tail) {
                int32_t u = queue[head++];
                int64_t d = g->xadj[u + 1] - g->xadj[u];
                memcpy(nb, g->adjncy + g->xadj[u], (size_t)d * sizeof(int32_t));
                qsort(nb, (size_t)d, sizeof(int32_t), cmp_i32);
                for (int64_t i = 0; i < d; ++i) {
                    int32_t x = nb[i];
                    if (part[x] >= 0) continue;
                    if (wb[b] + node_w(g, x) > T) continue;
                    part[x] = b;
                    wb[b] += node_w(g, x);
                    queue[tail++] = x;
                }
            }
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        if (part[v] >= 0) continue;
        int32_t bmin = 0;
        for (int32_t b = 1; b < k; ++b)
            if (wb[b] < wb[bmin]) bmin = b;
        part[v] = bmin;
        wb[bmin] += node_w(g, v);
    }
    free(nb);
    free(queue);
    free(wb);
    return 0;
}

/*
 * Initial partition by label propagation from seeds (a deterministic
 * stand-in for the evolutionary partitioner of Section 4.5, built from the
 * size-constrained label propagation of Section 3.1):
 *   1. seeds: the min(k, #nodes with neighbours) nodes with neighbours of
 *      smallest (H(seed, 5, level, v), v); seed i starts block i;
 *   2. every other node starts in a pool, label k, whose weight carries an
 *      offset BIG = 2^30 > Lmax: the pool is never an eligible target and
 *      always overloaded, so by the overloaded-block rule each pool node
 *      joins its best eligible neighbouring block (none: it stays);
 *   3. `rounds` label-propagation rounds under Lmax with k + 1 labels, with
 *      the refinement rules and hash phase 2 (ORC_INITIAL);
 *   4. the nodes still in the pool (isolated ones among them), in id order,
 *      fill the blocks' remaining room max(0, T - w(b)) in block order: the
 *      node whose exclusive prefix weight is P goes to the first block whose
 *      cumulative room exceeds P (block k - 1 if none does).
 * Requires Lmax < 2^30 and c(V) < 2^30 (returns -1 otherwise).
 */
typedef struct { uint64_t h; int32_t v; } seed_key;

static int cmp_seed_key(const void* x, const void* y) {
    const seed_key* p = (const seed_key*)x;
    const seed_key* q = (const seed_key*)y;
    if (p->h != q->h) return p->h < q->h ? -1 : 1;
    return (p->v > q->v) - (p->v < q->v);
}

int32_t orc_initial_partition_lp(const orc_graph* g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed,
                                 int32_t level, int32_t rounds, int32_t nsub, int32_t* part, int32_t* rounds_run,
                                 int64_t* visits) {
    const int64_t BIG = (int64_t)1 << 30;
    int32_t n = g->n;
    int64_t cV = total_node_weight(g);
    if (k < 1 || nsub < 1 || rounds < 0 || Lmax >= BIG || cV >= BIG) return -1;
    seed_key* S = (seed_key*)malloc((size_t)(n > 0 ? n : 1) * sizeof(seed_key));
    int32_t npos = 0;
    for (int32_t v = 0; v < n; ++v) {
        part[v] = k;
        if (g->xadj[v + 1] == g->xadj[v]) continue;
        uint64_t words[4] = {seed, 5, (uint64_t)(uint32_t)level, (uint64_t)(uint32_t)v};
        S[npos].h = orc_hash(words, 4);
        S[npos].v = v;
        ++npos;
    }
    qsort(S, (size_t)npos, sizeof(seed_key), cmp_seed_key);
    for (int32_t i = 0; i < k && i < npos; ++i) part[S[i].v] = i;
    free(S);
    int64_t* w = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) w[part[v]] += node_w(g, v);
    w[k] += BIG;
    run_rounds(g, NULL, ORC_INITIAL, level, rounds, nsub, seed, Lmax, NULL, part, w, rounds_run, visits);
    /* the pool fills the remaining room of the blocks in block order */
    int64_t* cum = (int64_t*)malloc((size_t)k * sizeof(int64_t));
    int64_t run = 0;
    for (int32_t b = 0; b < k; ++b) {
        run += w[b] < T ? T - w[b] : 0;
        cum[b] = run;
    }
    int64_t P = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (part[v] != k) continue;
        int32_t b = 0;
        while (b < k && cum[b] <= P) ++b;
        part[v] = b < k ? b : k - 1;
        P += node_w(g, v);
    }
    free(cum);
    free(w);
    return 0;
}

/* ------------------------------------------------------------ multilevel */

void orc_default_options(orc_options* o) {
    o->coarsen_rounds = 10;
    o->refine_rounds = 10;
    o->subrounds = 4;
    o->cluster_divisor = 18;
    o->coarsest_nodes = 10000;
    o->max_levels = ORC_MAX_LEVELS;
    o->vcycles = 1;
    o->degree_order = 0;
    o->initial = 0;
}

typedef struct {
    int32_t n;
    int64_t* xadj;
    int32_t* adj;
    int32_t* adjw;
    int32_t* vw;
    int32_t* C;   /* map to the next coarser level */
    int32_t* blk; /* block of each node in the carried partition (later cycles) */
} level_t;

/* Seed of multilevel cycle c: the caller's seed for the first, a hash of
 * (seed, 4, c) for later ones, so each cycle draws fresh colours and ties. */
uint64_t orc_cycle_seed(uint64_t seed, int32_t cycle) {
    if (cycle == 0) return seed;
    uint64_t words[3] = {seed, 4, (uint64_t)(uint32_t)cycle};
    return orc_hash(words, 3);
}

/*
 * Multilevel partitioning (Section 4.5): cluster with SCLaP under U and
 * contract, level by level, while the graph has more than `coarsest_nodes`
 * nodes; keep a level only if it is smaller and continue only while it shrinks
 * by at least 5%; partition the coarsest graph; then at every level from the
 * coarsest to the finest project the partition and refine it with SCLaP under
 * Lmax.
 *
 * Iterated V-cycles (Section 4.4, Miscellanea: Iterated Multilevel Schemes): every cycle
 * after the first clusters inside the blocks of the previous cycle's result,
 * so no cut edge is contracted, each coarse node inherits the block of its
 * members, and the inherited partition of the coarsest graph (same cut and
 * block weights as the input partition) replaces the initial partitioner.
 * The result of the last cycle is returned.
 */
int32_t orc_partition(const orc_graph* g, int32_t k, double eps, uint64_t seed, const orc_options* opt_in,
                      int32_t* part, int64_t* cut, int64_t* bw, orc_stats* stats) {
    orc_options opt;
    if (opt_in) opt = *opt_in;
    else orc_default_options(&opt);
    if (!g || k < 1 || !(eps >= 0.0) || eps > 1000.0) return -1;
    if (opt.subrounds < 1 || opt.cluster_divisor < 1 || opt.max_levels < 0 || opt.max_levels > ORC_MAX_LEVELS ||
        opt.coarsen_rounds < 0 || opt.refine_rounds < 0 || opt.vcycles < 1 || opt.initial < 0 || opt.initial > 1)
        return -1;
    int32_t st = orc_validate(g);
    if (st != 0) return st;
    orc_stats local;
    orc_stats* S = stats ? stats : &local;
    memset(S, 0, sizeof(*S));
    int32_t n0 = g->n;
    int64_t cV = total_node_weight(g);
    int64_t Lmax = orc_lmax(cV, k, eps);
    int64_t W = cV / ((int64_t)opt.cluster_divisor * k);
    int64_t S0 = n0 > 0 ? g->xadj[n0] : 0;
    int32_t* prev = NULL; /* result of the previous cycle */

    for (int32_t cyc = 0; cyc < opt.vcycles; ++cyc) {
        uint64_t sd = orc_cycle_seed(seed, cyc);
        int64_t visits = S->visits;
        memset(S, 0, sizeof(*S));
        S->visits = visits;
        level_t L[ORC_MAX_LEVELS + 1];
        memset(L, 0, sizeof(L));
        /* level 0 views the input; materialise weights for uniform access */
        L[0].n = n0;
        L[0].xadj = (int64_t*)g->xadj;
        L[0].adj = (int32_t*)g->adjncy;
        L[0].adjw = (int32_t*)malloc((size_t)(S0 > 0 ? S0 : 1) * sizeof(int32_t));
        L[0].vw = (int32_t*)malloc((size_t)(n0 > 0 ? n0 : 1) * sizeof(int32_t));
        L[0].blk = prev;
        for (int64_t i = 0; i < S0; ++i) L[0].adjw[i] = (int32_t)edge_w(g, i);
        for (int32_t v = 0; v < n0; ++v) L[0].vw[v] = (int32_t)node_w(g, v);
        S->level_n[0] = n0;
        S->level_S[0] = S0;

        int32_t lev = 0;
        while (L[lev].n > opt.coarsest_nodes && lev < opt.max_levels) {
            orc_graph G = {L[lev].n, L[lev].xadj, L[lev].adj, L[lev].vw, L[lev].adjw};
            int32_t n = G.n;
            int64_t cmax = 0;
            for (int32_t v = 0; v < n; ++v)
                if (G.vwgt[v] > cmax) cmax = G.vwgt[v];
            int64_t U = cmax > W ? cmax : W;
            int32_t* labels = (int32_t*)malloc((size_t)n * sizeof(int32_t));
            int32_t rr = 0;
            int32_t* dcol = NULL;
            if (opt.degree_order) {
                dcol = (int32_t*)malloc((size_t)n * sizeof(int32_t));
                orc_degree_colors(&G, L[lev].blk, opt.subrounds, dcol);
            }
            orc_cluster_within(&G, L[lev].blk, U, opt.coarsen_rounds, opt.subrounds, sd, lev, dcol, labels, &rr,
                               &S->visits);
            free(dcol);
            S->cluster_rounds[lev] = rr;
            int64_t Sl = G.xadj[n];
            level_t nx;
            memset(&nx, 0, sizeof(nx));
            int32_t* Cmap = (int32_t*)malloc((size_t)n * sizeof(int32_t));
            nx.xadj = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
            nx.adj = (int32_t*)malloc((size_t)(Sl > 0 ? Sl : 1) * sizeof(int32_t));
            nx.adjw = (int32_t*)malloc((size_t)(Sl > 0 ? Sl : 1) * sizeof(int32_t));
            nx.vw = (int32_t*)malloc((size_t)n * sizeof(int32_t));
            int64_t Sc = 0;
            orc_contract(&G, labels, Cmap, &nx.n, nx.xadj, nx.adj, nx.adjw, nx.vw, &Sc);
            free(labels);
            if (nx.n >= n) { /* no shrink: discard the new level */
                free(Cmap); free(nx.xadj); free(nx.adj); free(nx.adjw); free(nx.vw);
                break;
            }
            if (L[lev].blk) { /* a coarse node lies in the block of its members */
                nx.blk = (int32_t*)malloc((size_t)(nx.n > 0 ? nx.n : 1) * sizeof(int32_t));
                for (int32_t v = 0; v < n; ++v) nx.blk[Cmap[v]] = L[lev].blk[v];
            }
            L[lev].C = Cmap;
            L[lev + 1] = nx;
            ++lev;
            S->level_n[lev] = nx.n;
            S->level_S[lev] = Sc;
            if (20LL * nx.n > 19LL * n) break; /* stalled: shrank by less than 5% */
        }
        S->levels = lev;

        /* partition of the coarsest graph: the initial partitioner in the
         * first cycle, the inherited blocks in later ones */
        int64_t T = (cV + k - 1) / k;
        int32_t* cur = (int32_t*)malloc((size_t)(L[lev].n > 0 ? L[lev].n : 1) * sizeof(int32_t));
        if (L[lev].blk) {
            memcpy(cur, L[lev].blk, (size_t)L[lev].n * sizeof(int32_t));
        } else if (opt.initial == 1) {
            orc_graph G = {L[lev].n, L[lev].xadj, L[lev].adj, L[lev].vw, L[lev].adjw};
            int32_t rr = 0;
            if (orc_initial_partition_lp(&G, k, T, Lmax, sd, lev, opt.refine_rounds, opt.subrounds, cur, &rr,
                                         &S->visits) != 0) {
                free(cur);
                for (int32_t l = 0; l <= lev; ++l) {
                    if (l > 0) { free(L[l].xadj); free(L[l].adj); free(L[l].blk); }
                    free(L[l].adjw); free(L[l].vw); free(L[l].C);
                }
                free(prev);
                return -1;
            }
        } else {
            orc_graph G = {L[lev].n, L[lev].xadj, L[lev].adj, L[lev].vw, L[lev].adjw};
            orc_initial_partition(&G, k, T, cur);
        }
        for (int32_t l = lev; l >= 0; --l) {
            if (l < lev) {
                int32_t* fine = (int32_t*)malloc((size_t)(L[l].n > 0 ? L[l].n : 1) * sizeof(int32_t));
                orc_project(L[l].n, L[l].C, cur, fine);
                free(cur);
                cur = fine;
            }
            orc_graph G = {L[l].n, L[l].xadj, L[l].adj, L[l].vw, L[l].adjw};
            int32_t rr = 0;
            orc_refine(&G, k, Lmax, opt.refine_rounds, opt.subrounds, sd, l, NULL, cur, &rr, &S->visits);
            S->refine_rounds[l] = rr;
        }
        for (int32_t l = 0; l <= lev; ++l) {
            if (l > 0) { free(L[l].xadj); free(L[l].adj); free(L[l].blk); }
            free(L[l].adjw); free(L[l].vw); free(L[l].C);
        }
        free(prev);
        prev = cur;
    }
    memcpy(part, prev, (size_t)n0 * sizeof(int32_t));
    free(prev);
    orc_cut(g, part, k, cut, bw);
    for (int32_t b = 0; b < k; ++b)
        if (bw[b] > Lmax) return 1;
    return 0;
}
