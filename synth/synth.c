/*
 * Seeded synthetic graph generators (inputs only).
 *
 * This module produces the synthetic stand-ins for the paper's benchmark
 * graphs (Section 5, Table I: web graphs, social networks, random geometric
 * graphs).  It holds none of the partitioning method's arithmetic: it only
 * draws random edges and assembles a symmetric CSR.  Both the CPU oracle and
 * the GPU library consume what it writes; neither shares any other code.
 *
 * Random numbers: a counter-based SplitMix64 stream (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).  Draw i of
 * the stream with key K is the SplitMix64 output function applied to
 * K + (i+1)*0x9E3779B97F4A7C15, i.e. exactly the i-th output of a SplitMix64
 * generator seeded with K.  Every draw is addressed by its index, so results
 * do not depend on thread count or scheduling.
 *
 * Output CSR: xadj int64[n+1], adjncy int32[S], adjwgt int32[S], vwgt int32[n];
 * symmetric, no self-loops, no duplicate neighbours, rows sorted ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* i-th output of a SplitMix64 stream seeded with key */
static inline uint64_t draw(uint64_t key, uint64_t i) { return sm_out(key + (i + 1) * SM_GAMMA); }

/* derive an independent stream key from (seed, tag) */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) { return draw(seed ^ (tag * 0xD1B54A32D192ED03ULL), tag); }

uint64_t synth_draw(uint64_t key, uint64_t i) { return draw(key, i); }

/* ------------------------------------------------------------------------- */
/* CSR assembly from an undirected edge list.                                 */
/* ------------------------------------------------------------------------- */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Build a symmetric CSR from m undirected pairs (src[i], dst[i]).  Self-loops
 * are dropped, both directions are inserted, duplicates are merged.  Returns S
 * (number of directed slots) and allocates *adj (caller frees with
 * synth_free).  xadj must hold n+1 entries.
 */
static int64_t build_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         int64_t* xadj, int32_t** adj_out) {
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        if (src[i] == dst[i]) continue;
        cnt[src[i]]++;
        cnt[dst[i]]++;
    }
    xadj[0] = 0;
    for (int32_t v = 0; v < n; ++v) xadj[v + 1] = xadj[v] + cnt[v];
    int64_t S0 = xadj[n];
    int32_t* adj = (int32_t*)malloc((size_t)(S0 > 0 ? S0 : 1) * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) cnt[v] = xadj[v];
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        adj[cnt[u]++] = v;
        adj[cnt[v]++] = u;
    }
    /* sort rows and drop duplicates; new row lengths go to cnt */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = xadj[v], e = xadj[v + 1];
        if (e - b > 1) qsort(adj + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t w = b;
        for (int64_t i = b; i < e; ++i)
            if (i == b || adj[i] != adj[i - 1]) adj[w++] = adj[i];
        cnt[v] = w - b;
    }
    /* compact */
    int64_t pos = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = xadj[v];
        if (pos != b) memmove(adj + pos, adj + b, (size_t)cnt[v] * sizeof(int32_t));
        xadj[v] = pos;
        pos += cnt[v];
    }
    xadj[n] = pos;
    free(cnt);
    *adj_out = adj;
    return pos;
}

void synth_free(void* p) { free(p); }

/*
 * Edge weights: w(u,v) = 1 + (draw(key_w, min(u,v) * n + max(u,v)) mod 4), so
 * the two directions of an edge always carry the same weight.  With
 * weighted == 0 every weight is 1.
 */
static void fill_weights(int32_t n, const int64_t* xadj, const int32_t* adj, int32_t* adjwgt,
                         int weighted, uint64_t seed) {
    uint64_t kw = stream_key(seed, 3);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v)
        for (int64_t i = xadj[v]; i < xadj[v + 1]; ++i) {
            if (!weighted) { adjwgt[i] = 1; continue; }
            uint64_t a = (uint64_t)(v < adj[i] ? v : adj[i]);
            uint64_t b = (uint64_t)(v < adj[i] ? adj[i] : v);
            adjwgt[i] = 1 + (int32_t)(draw(kw, a * (uint64_t)n + b) & 3ULL);
        }
}

/* ------------------------------------------------------------------------- */
/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004), no noise, no id permutation.    */
/* ------------------------------------------------------------------------- */
/*
 * Draw ef * 2^scale edges.  Each recursion level picks a quadrant with
 * probabilities a, b, c, d = 1-a-b-c using 16 bits of a 64-bit draw (4
 * levels per draw).  Node ids are < 2^scale; with n_keep < 2^scale, edges
 * with an endpoint >= n_keep are discarded (used for non-power-of-two n).
 * Returns S, fills xadj[n_keep+1], allocates *adj and *adjwgt.
 */
int64_t synth_rmat(int32_t scale, int32_t n_keep, int64_t n_edges, double a, double b, double c,
                   uint64_t seed, int weighted, int64_t* xadj, int32_t** adj, int32_t** adjwgt) {
    uint64_t key = stream_key(seed, 1);
    uint32_t ta = (uint32_t)llround(a * 65536.0);
    uint32_t tab = (uint32_t)llround((a + b) * 65536.0);
    uint32_t tabc = (uint32_t)llround((a + b + c) * 65536.0);
    int32_t draws_per_edge = (scale + 3) / 4;
    int32_t* src = (int32_t*)malloc((size_t)n_edges * sizeof(int32_t));
    int32_t* dst = (int32_t*)malloc((size_t)n_edges * sizeof(int32_t));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_edges; ++e) {
        uint32_t u = 0, v = 0;
        uint64_t r = 0;
        for (int32_t l = 0; l < scale; ++l) {
            if ((l & 3) == 0) r = draw(key, (uint64_t)e * (uint64_t)draws_per_edge + (uint64_t)(l >> 2));
            uint32_t q = (uint32_t)(r & 0xFFFFu);
            r >>= 16;
            uint32_t row = (q >= tab) ? 1u : 0u;         /* c or d */
            uint32_t col = (q >= ta && q < tab) || q >= tabc ? 1u : 0u; /* b or d */
            u = (u << 1) | row;
            v = (v << 1) | col;
        }
        if ((int64_t)u >= n_keep || (int64_t)v >= n_keep) { u = 0; v = 0; } /* dropped as self-loop */
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
    }
    int64_t S = build_csr(n_keep, n_edges, src, dst, xadj, adj);
    free(src);
    free(dst);
    *adjwgt = (int32_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(int32_t));
    fill_weights(n_keep, xadj, *adj, *adjwgt, weighted, seed);
    return S;
}

/* ------------------------------------------------------------------------- */
/* Barabasi-Albert preferential attachment.                                   */
/* ------------------------------------------------------------------------- */
/*
 * Nodes 0..m-1 start unconnected.  Node m attaches to 0..m-1.  Every later
 * node v picks m distinct targets, each drawn uniformly from the list of all
 * endpoints of edges created so far (so a node is chosen with probability
 * proportional to its degree), rejecting duplicates.
 */
int64_t synth_ba(int32_t n, int32_t m, uint64_t seed, int weighted, int64_t* xadj, int32_t** adj,
                 int32_t** adjwgt) {
    uint64_t key = stream_key(seed, 2);
    uint64_t ctr = 0;
    int64_t max_edges = (n > m) ? (int64_t)(n - m) * m : 0;
    int32_t* src = (int32_t*)malloc((size_t)(max_edges > 0 ? max_edges : 1) * sizeof(int32_t));
    int32_t* dst = (int32_t*)malloc((size_t)(max_edges > 0 ? max_edges : 1) * sizeof(int32_t));
    int32_t* ends = (int32_t*)malloc((size_t)(2 * max_edges + 1) * sizeof(int32_t));
    int32_t* pick = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t ne = 0, nends = 0;
    for (int32_t v = m; v < n; ++v) {
        int32_t got = 0;
        if (v == m) {
            for (int32_t t = 0; t < m; ++t) pick[got++] = t;
        } else {
            while (got < m) {
                int32_t t = ends[draw(key, ctr++) % (uint64_t)nends];
                int dup = 0;
                for (int32_t j = 0; j < got; ++j) dup |= (pick[j] == t);
                if (!dup) pick[got++] = t;
            }
        }
        for (int32_t j = 0; j < got; ++j) {
            src[ne] = v;
            dst[ne] = pick[j];
            ++ne;
            ends[nends++] = v;
            ends[nends++] = pick[j];
        }
    }
    int64_t S = build_csr(n, ne, src, dst, xadj, adj);
    free(src);
    free(dst);
    free(ends);
    free(pick);
    *adjwgt = (int32_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(int32_t));
    fill_weights(n, xadj, *adj, *adjwgt, weighted, seed);
    return S;
}

/* ------------------------------------------------------------------------- */
/* 2D random geometric graph (the paper's rggX family, Section 5).           */
/* ------------------------------------------------------------------------- */
/*
 * n points with 31-bit integer coordinates in [0, 2^31)^2; u and v are
 * adjacent iff their squared integer distance is < r_int^2 where
 * r_int = floor(radius * 2^31).  Integer arithmetic keeps it exact.
 */
int64_t synth_rgg(int32_t n, double radius, uint64_t seed, int weighted, int64_t* xadj,
                  int32_t** adj, int32_t** adjwgt) {
    uint64_t key = stream_key(seed, 4);
    const double SCALE = 2147483648.0;
    uint64_t r = (uint64_t)floor(radius * SCALE);
    if (r < 1) r = 1;
    uint64_t r2 = r * r;
    uint32_t* x = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    uint32_t* y = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) {
        uint64_t d = draw(key, (uint64_t)i);
        x[i] = (uint32_t)(d & 0x7FFFFFFFu);
        y[i] = (uint32_t)((d >> 32) & 0x7FFFFFFFu);
    }
    /* grid of cells of side >= r */
    int64_t g = (int64_t)(SCALE / (double)r);
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    uint64_t cw = ((uint64_t)1 << 31) / (uint64_t)g + 1; /* cell width >= r */
    int64_t ncell = g * g;
    int64_t* cstart = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t* cell_of = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        int64_t cx = (int64_t)(x[i] / cw), cy = (int64_t)(y[i] / cw);
        cell_of[i] = (int32_t)(cy * g + cx);
        cstart[cell_of[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    int32_t* members = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t* fill = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, cstart, (size_t)ncell * sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i) members[fill[cell_of[i]]++] = i;
    free(fill);
    /* collect pairs u < v */
    int64_t cap = (int64_t)n * 8 + 16, ne = 0;
    int32_t* src = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* dst = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    for (int32_t u = 0; u < n; ++u) {
        int64_t cx = cell_of[u] % g, cy = cell_of[u] / g;
        for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
                int64_t nx = cx + dx, ny = cy + dy;
                if (nx < 0 || ny < 0 || nx >= g || ny >= g) continue;
                int64_t c = ny * g + nx;
                for (int64_t j = cstart[c]; j < cstart[c + 1]; ++j) {
                    int32_t v = members[j];
                    if (v <= u) continue;
                    int64_t ddx = (int64_t)x[u] - (int64_t)x[v];
                    int64_t ddy = (int64_t)y[u] - (int64_t)y[v];
                    uint64_t d2 = (uint64_t)(ddx * ddx) + (uint64_t)(ddy * ddy);
                    if (d2 < r2) {
                        if (ne == cap) {
                            cap *= 2;
                            src = (int32_t*)realloc(src, (size_t)cap * sizeof(int32_t));
                            dst = (int32_t*)realloc(dst, (size_t)cap * sizeof(int32_t));
                        }
                        src[ne] = u;
                        dst[ne] = v;
                        ++ne;
                    }
                }
            }
    }
    free(x);
    free(y);
    free(cstart);
    free(cell_of);
    free(members);
    int64_t S = build_csr(n, ne, src, dst, xadj, adj);
    free(src);
    free(dst);
    *adjwgt = (int32_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(int32_t));
    fill_weights(n, xadj, *adj, *adjwgt, weighted, seed);
    return S;
}

/* Copy a library-allocated array into a caller buffer and free it. */
void synth_take_i32(int32_t* src, int32_t* dst, int64_t count) {
    if (count > 0) memcpy(dst, src, (size_t)count * sizeof(int32_t));
    free(src);
}
