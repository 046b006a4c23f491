// Multilevel drivers for gfx950: one graph (Section 4.5) and a batch of
// independent graphs, plus the host initial partitioner of the coarsest graph.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <future>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include <immintrin.h>

#include "driver.hpp"
#include "profile.hpp"

namespace sclap {

// ----------------------------------------------------------------- options

Opts resolve(const sclap_options* o) {
    Opts r;
    if (!o) return r;
    r.coarsen_rounds = o->coarsen_rounds;
    r.refine_rounds = o->refine_rounds;
    r.nsub = o->subrounds;
    r.divisor = o->cluster_divisor;
    r.coarsest = o->coarsest_nodes;
    r.max_levels = o->max_levels;
    r.validate = o->validate;
    r.color_override = o->color_override;
    if (o->lane_max_degree > 0) r.tune.lane_max = o->lane_max_degree;
    if (o->wave_max_degree > 0) r.tune.wave_max = o->wave_max_degree;
    if (o->block_max_degree > 0) r.tune.block_max = o->block_max_degree;
    if (o->hub_part_limit > 0) r.tune.hub_part_limit = o->hub_part_limit;
    if (o->hub_region_cap > 0) r.tune.hub_region_cap = o->hub_region_cap;
    if (o->select_small_max > 0) r.tune.select_small_max = o->select_small_max;
    if (o->select_launches < 0) fail(SCLAP_ERR_INVALID, "select_launches must be >= 0");
    r.tune.select_launches = o->select_launches;
    if (o->graph_capture < -1 || o->graph_capture > 1) fail(SCLAP_ERR_INVALID, "graph_capture must be -1, 0 or 1");
    r.tune.capture = o->graph_capture;
    if (o->fused_eval < -1 || o->fused_eval > 1) fail(SCLAP_ERR_INVALID, "fused_eval must be -1, 0 or 1");
    r.tune.fuse = o->fused_eval;
    if (o->block_table != 0 && o->block_table != 10240 && o->block_table != 16384)
        fail(SCLAP_ERR_INVALID, "block_table must be 0, 10240 or 16384");
    if (o->block_table != 0) r.tune.block_table = o->block_table;
    r.tune.skip_quiet = o->skip_quiet < 0 ? -1 : (o->skip_quiet > 0 ? 1 : 0);
    r.vcycles = o->vcycles == 0 ? 1 : o->vcycles;
    r.degree_order = o->degree_order != 0 ? 1 : 0;
    r.bucket_mean = o->contract_bucket_mean;
    r.initial = o->initial_partitioner;
    if (r.initial < 0 || r.initial > 1) fail(SCLAP_ERR_INVALID, "initial_partitioner must be 0 or 1");
    if (r.bucket_mean < 0) fail(SCLAP_ERR_INVALID, "contract_bucket_mean must be >= 0");
    if (r.vcycles < 1 || r.vcycles > 64) fail(SCLAP_ERR_INVALID, "vcycles must be in 1..64");
    if (r.coarsen_rounds < 0 || r.refine_rounds < 0) fail(SCLAP_ERR_INVALID, "round counts must be >= 0");
    if (r.nsub < 1 || r.nsub > 16) fail(SCLAP_ERR_INVALID, "subrounds must be in 1..16");
    if (r.divisor < 1) fail(SCLAP_ERR_INVALID, "cluster_divisor must be >= 1");
    if (r.coarsest < 0) fail(SCLAP_ERR_INVALID, "coarsest_nodes must be >= 0");
    if (r.max_levels < 0 || r.max_levels > SCLAP_MAX_LEVELS) fail(SCLAP_ERR_INVALID, "max_levels must be in 0..64");
    return r;
}

// Device view of a caller graph with device pointers; reads S = xadj[n].
DevGraph dev_view(const sclap_graph* g, hipStream_t s) {
    if (!g) fail(SCLAP_ERR_INVALID, "graph is NULL");
    if (g->n < 0) fail(SCLAP_ERR_INVALID, "n < 0");
    DevGraph d;
    d.n = g->n;
    d.xadj = g->xadj;
    d.adj = g->adjncy;
    d.ew = g->adjwgt;
    d.vw = g->vwgt;
    if (g->n > 0) {
        if (!g->xadj) fail(SCLAP_ERR_INVALID, "xadj is NULL");
        HIPCHK(hipMemcpyAsync(&d.S, g->xadj + g->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (d.S < 0) fail(SCLAP_ERR_INVALID, "xadj[n] < 0");
        if (d.S > 0 && !g->adjncy) fail(SCLAP_ERR_INVALID, "adjncy is NULL");
    }
    return d;
}

void check_graph(const DevGraph& g, bool validate, int64_t* cV, int64_t* cmax, hipStream_t s) {
    if (validate) {
        const int st = validate_graph(g, cV, cmax, s);
        if (st == SCLAP_ERR_INVALID) fail(st, "invalid graph (offsets, ids, self-loops or weights)");
        if (st == SCLAP_ERR_NOT_SYMMETRIC) fail(st, "graph is not symmetric");
        if (st == SCLAP_ERR_OVERFLOW) fail(st, "node or edge weight total exceeds 2^31-1");
        if (st != 0) fail(st, "graph validation failed");
    } else {
        node_weight_stats(g, cV, cmax, s);
    }
}

int64_t lmax_of(int64_t cV, int32_t k, double eps) {
    const int64_t T = (cV + k - 1) / k;
    const int64_t ppm = std::llround(eps * 1e6);
    return T + (T * ppm) / 1000000;
}

void check_k_eps(int32_t k, double eps) {
    if (k < 1) fail(SCLAP_ERR_INVALID, "k must be >= 1");
    if (!(eps >= 0.0) || eps > 1000.0) fail(SCLAP_ERR_INVALID, "eps must be in [0, 1000]");
}

// ------------------------------------------------- host initial partition

namespace {

// Runs f(i) for i in [0, count) on up to `threads` host threads.
template <typename F>
void parallel_for(int32_t count, int32_t threads, F f) {
    threads = std::max(1, std::min(threads, count));
    if (threads == 1) {
        for (int32_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<int32_t> next{0};
    std::vector<std::exception_ptr> errs(threads);
    std::vector<std::thread> pool;
    for (int32_t t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            try {
                for (int32_t i = next++; i < count; i = next++) f(i);
            } catch (...) {
                errs[t] = std::current_exception();
            }
        });
    for (auto& th : pool) th.join();
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

// Smallest index >= from whose value is <= cap, over a segment tree of mins.
struct MinTree {  // node weights are int32; INT32_MAX marks an erased leaf
    int64_t size = 1;
    std::vector<int32_t> t;
    explicit MinTree(const std::vector<int64_t>& a) {
        while (size < static_cast<int64_t>(a.size())) size <<= 1;
        t.assign(2 * static_cast<size_t>(size), INT32_MAX);
        for (size_t i = 0; i < a.size(); ++i) t[size + i] = static_cast<int32_t>(a[i]);
        for (int64_t i = size - 1; i > 0; --i) t[i] = std::min(t[2 * i], t[2 * i + 1]);
    }
    void erase(int64_t i) {
        int64_t p = i + size;
        t[p] = INT32_MAX;
        for (p >>= 1; p > 0; p >>= 1) {
            const int32_t m = std::min(t[2 * p], t[2 * p + 1]);
            if (m == t[p]) break;  // ancestors keep their minima
            t[p] = m;
        }
    }
    // smallest index >= from whose weight is <= cap, or -1: from the leaf,
    // climb while on a right child, step to the right sibling until one holds
    // a fitting leaf, then descend to its leftmost fitting leaf (the next
    // seed is usually close, so this climbs only a few levels)
    int32_t first_le(int64_t from, int64_t cap) const {
        if (from < 0) from = 0;
        if (from >= size) return -1;
        int64_t p = from + size;
        if (t[p] <= cap) return static_cast<int32_t>(from);
        while (true) {
            while (p & 1) {
                p >>= 1;
                if (p <= 1) return -1;
            }
            ++p;
            if (t[p] <= cap) break;
        }
        while (p < size) {
            p <<= 1;
            if (t[p] > cap) ++p;
        }
        return static_cast<int32_t>(p - size);
    }
    int64_t min() const { return t[1] == INT32_MAX ? INT64_MAX : t[1]; }
};

// Binary min-heap of packed (weight << 32 | block) keys: the lightest block,
// lowest id on ties, is at the root.
struct BlockHeap {
    std::vector<uint64_t> h;
    static uint64_t key(int64_t w, int32_t b) { return (static_cast<uint64_t>(w) << 32) | static_cast<uint32_t>(b); }
    explicit BlockHeap(const std::vector<int64_t>& wb) { reset(wb); }
    // rebuilds the heap from the block weights (storage reused)
    void reset(const std::vector<int64_t>& wb) {
        h.resize(wb.size());
        for (size_t b = 0; b < wb.size(); ++b) h[b] = key(wb[b], static_cast<int32_t>(b));
        std::make_heap(h.begin(), h.end(), std::greater<uint64_t>());
    }
    int32_t top() const { return static_cast<int32_t>(h[0] & 0xFFFFFFFFu); }
    // adds c to the root's weight and restores the heap order
    void add_to_top(int64_t c) {
        if (c == 0) return;
        const uint64_t x = h[0] + (static_cast<uint64_t>(c) << 32);
        size_t i = 0;
        const size_t n = h.size();
        while (true) {
            size_t l = 2 * i + 1;
            if (l >= n) break;
            if (l + 1 < n && h[l + 1] < h[l]) ++l;
            if (h[l] >= x) break;
            h[i] = h[l];
            i = l;
        }
        h[i] = x;
    }
};

}  // namespace

// Untaken-neighbour masks of a row, eight slots per byte (bit q of byte j for
// slot 8j + q of the first 8 * nb slots): set when the neighbour's bit in the
// taken bitmap is clear or its id is outside [0, ncore).  AVX2 gathers of the
// bitmap words where the CPU has them, one slot at a time otherwise.  Bits
// only go from clear to set while a row is walked, so a mask computed before
// the walk may only over-report, and every reported slot is checked again.
__attribute__((target("avx2"))) void untaken_masks_avx2(const int32_t* row, size_t nb, const uint32_t* taken32,
                                                       uint32_t ncore, uint8_t* masks) {
    const __m256i bias = _mm256_set1_epi32(static_cast<int>(0x80000000u));
    const __m256i ncb = _mm256_xor_si256(_mm256_set1_epi32(static_cast<int>(ncore)), bias);
    const __m256i low5 = _mm256_set1_epi32(31);
    const __m256i one = _mm256_set1_epi32(1);
    for (size_t j = 0; j < nb; ++j) {
        const __m256i x = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(row + 8 * j));
        const __m256i inb = _mm256_cmpgt_epi32(ncb, _mm256_xor_si256(x, bias));  // x < ncore, unsigned
        const __m256i idx = _mm256_and_si256(_mm256_srli_epi32(x, 5), inb);    // outside: word 0
        const __m256i w = _mm256_i32gather_epi32(reinterpret_cast<const int*>(taken32), idx, 4);
        const __m256i bit = _mm256_and_si256(_mm256_srlv_epi32(w, _mm256_and_si256(x, low5)), one);
        const __m256i want = _mm256_or_si256(_mm256_cmpeq_epi32(bit, _mm256_setzero_si256()),
                                             _mm256_andnot_si256(inb, _mm256_set1_epi32(-1)));
        masks[j] = static_cast<uint8_t>(_mm256_movemask_ps(_mm256_castsi256_ps(want)));
    }
}

void untaken_masks_scalar(const int32_t* row, size_t nb, const uint64_t* taken, uint32_t ncore, uint8_t* masks) {
    for (size_t j = 0; j < nb; ++j) {
        uint32_t m = 0;
        for (int q = 0; q < 8; ++q) {
            const uint32_t x = static_cast<uint32_t>(row[8 * j + q]);
            const uint64_t word = x < ncore ? taken[x >> 6] : 0ULL;
            m |= static_cast<uint32_t>(~(word >> (x & 63)) & 1ULL) << q;
        }
        masks[j] = static_cast<uint8_t>(m);
    }
}

// Grows blocks 0..k-2 by breadth-first search up to T each (seeds: smallest
// unassigned node of positive degree that fits; neighbours in ascending id
// order), then deals every remaining node, in id order, to the currently
// lightest block (lowest id on ties).  Weights fit 31 bits (c(V) <= 2^31-1).

void host_initial_partition(int32_t n, const int64_t* xadj, const int32_t* adj, const int32_t* vw, int32_t k,
                            int64_t T, int32_t* part, bool rows_sorted, bool adj_ranked, int32_t threads) {
    auto T0 = Clock::now();
    const unsigned hw = std::thread::hardware_concurrency();
    const int32_t nthr = threads > 0 ? threads : static_cast<int32_t>(std::min(16u, hw ? hw : 1u));
    // id ranges of whole 64-node words, one task each
    const size_t words = (static_cast<size_t>(n) + 63) / 64;
    const int32_t ntask = n < (1 << 20) ? 1 : 4 * nthr;
    auto task_words = [&](int32_t t, size_t& w0, size_t& w1) {
        w0 = words * t / ntask;
        w1 = words * (t + 1) / ntask;
    };
    std::vector<int64_t> wb(static_cast<size_t>(k), 0);
    // seed candidates: nodes of positive degree, in id order; a bitmap with
    // per-word prefix counts gives a node's index among them in O(1)
    std::vector<uint64_t> has_deg(words, 0);
    std::vector<int32_t> rank_base(words + 1, 0);
    std::vector<int32_t> task_cnt(static_cast<size_t>(ntask) + 1, 0);
    parallel_for(ntask, nthr, [&](int32_t t) {
        size_t w0, w1;
        task_words(t, w0, w1);
        int32_t cnt = 0;
        for (size_t w = w0; w < w1; ++w) {
            uint64_t bits = 0;
            const int32_t v0 = static_cast<int32_t>(w * 64);
            const int32_t v1 = std::min<int32_t>(n, v0 + 64);
            for (int32_t v = v0; v < v1; ++v) {
                part[v] = -1;
                if (xadj[v + 1] > xadj[v]) bits |= 1ULL << (v - v0);
            }
            has_deg[w] = bits;
            cnt += __builtin_popcountll(bits);
        }
        task_cnt[t + 1] = cnt;
    });
    for (int32_t t = 0; t < ntask; ++t) task_cnt[t + 1] += task_cnt[t];
    std::vector<int32_t> seed_node(static_cast<size_t>(task_cnt[ntask]));
    std::vector<int64_t> seed_w(seed_node.size());
    parallel_for(ntask, nthr, [&](int32_t t) {
        size_t w0, w1;
        task_words(t, w0, w1);
        int32_t r = task_cnt[t];
        for (size_t w = w0; w < w1; ++w) {
            rank_base[w] = r;
            for (uint64_t bits = has_deg[w]; bits; bits &= bits - 1) {
                const int32_t v = static_cast<int32_t>(w * 64) + __builtin_ctzll(bits);
                seed_node[r] = v;
                seed_w[r] = vw ? vw[v] : 1;
                ++r;
            }
        }
    });
    rank_base[words] = task_cnt[ntask];
    auto seed_rank = [&](int32_t v) {
        const size_t i = static_cast<size_t>(v) >> 6;
        return rank_base[i] + __builtin_popcountll(has_deg[i] & ((1ULL << (v & 63)) - 1));
    };
    const double t_pre = ms_since(T0);
    MinTree seeds(seed_w);
    const double t_tree = ms_since(T0);
    // Growth runs on the positive-degree nodes renumbered by rank (a
    // monotone renumbering, so seeds and neighbours keep their order and the
    // result is the same): its random accesses then hit arrays of the
    // core's size instead of n.  Nodes of degree 0 are never reached.
    const int32_t ncore = static_cast<int32_t>(seed_node.size());
    const int64_t S = n > 0 ? xadj[n] : 0;
    // the renumbered rows live in a per-thread buffer kept between calls:
    // first-touch page faults of a fresh buffer cost more than the mapping
    thread_local std::unique_ptr<int32_t[]> cadj_buf;
    thread_local size_t cadj_cap = 0;
    if (!adj_ranked && cadj_cap < static_cast<size_t>(std::max<int64_t>(S, 1))) {
        cadj_buf.reset();
        cadj_cap = static_cast<size_t>(std::max<int64_t>(S, 1));
        cadj_buf.reset(new int32_t[cadj_cap]);  // every entry used is written below
    }
    const int32_t* const cadj = adj_ranked ? adj : cadj_buf.get();
    int32_t* const cadj_w = cadj_buf.get();
    std::vector<int64_t> cx(static_cast<size_t>(ncore) + 1);
    std::vector<int32_t> cw32(static_cast<size_t>(ncore));
    std::atomic<int> bad{0};
    parallel_for(ntask, nthr, [&](int32_t t) {
        const int32_t i0 = static_cast<int32_t>(static_cast<int64_t>(ncore) * t / ntask);
        const int32_t i1 = static_cast<int32_t>(static_cast<int64_t>(ncore) * (t + 1) / ntask);
        for (int32_t i = i0; i < i1; ++i) {
            const int32_t v = seed_node[i];
            cx[i] = xadj[v];
            cw32[i] = static_cast<int32_t>(seed_w[i]);
            if (adj_ranked) continue;
            for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
                const int32_t x = adj[e];
                // a neighbour without neighbours of its own: the graph is not symmetric
                if (x < 0 || x >= n || !((has_deg[static_cast<size_t>(x) >> 6] >> (x & 63)) & 1ULL)) {
                    bad.store(1, std::memory_order_relaxed);
                    cadj_w[e] = 0;
                } else {
                    cadj_w[e] = seed_rank(x);
                }
            }
        }
    });
    if (bad.load()) fail(SCLAP_ERR_NOT_SYMMETRIC, "initial partition: a neighbour id is out of range or has no neighbours");
    cx[ncore] = S;
    const double t_seed = ms_since(T0);
    std::vector<uint64_t> ctaken((static_cast<size_t>(ncore) + 63) / 64 + 1, 0);
    static const bool use_avx2 = __builtin_cpu_supports("avx2");
    std::vector<uint8_t> masks;
    std::vector<int32_t> nb;
    std::vector<uint64_t> rowbits;  // scratch bitmap of the core for ordering unsorted rows
    // core nodes in the order blocks take them; each search's queue is the
    // tail of this list that it appended (a node is queued at most once)
    std::vector<int32_t> order(static_cast<size_t>(ncore) + 1);
    std::vector<size_t> bstart(static_cast<size_t>(k) + 1, 0);
    size_t ntaken = 0;
    bool nonsym = false;
    for (int32_t b = 0; b + 1 < k; ++b) {
        bstart[b] = ntaken;
        int64_t wcur = wb[b];
        auto take = [&](int32_t c) {
            ctaken[static_cast<size_t>(c) >> 6] |= 1ULL << (c & 63);
            wcur += cw32[c];
            seeds.erase(c);
            order[ntaken++] = c;
        };
        int32_t from = 0;
        while (true) {
            const int32_t si = seeds.first_le(from, T - wcur);
            if (si < 0) break;
            size_t head = ntaken;
            take(si);
            while (head < ntaken) {
                // every node a search can reach has positive degree, so once
                // the lightest such unassigned node does not fit, stop
                if (seeds.min() > T - wcur) break;
                const int32_t u = order[head++];
                // rows are visited in queue order, far apart in memory: fetch
                // the row a few places ahead in the queue early
                if (head + 6 < ntaken) {
                    const int64_t p = cx[order[head + 6]];
                    __builtin_prefetch(cadj + p);
                    __builtin_prefetch(cadj + p + 16);
                }
                const int32_t* row = cadj + cx[u];
                const int32_t* row_end = cadj + cx[u + 1];
                if (!rows_sorted && !std::is_sorted(row, row_end)) {
                    // ascending copy of the row: through a bitmap of the core
                    // when the row is dense in its id range (equal ids
                    // collapse, which the walk below would skip anyway),
                    // else by sorting
                    const auto mm = std::minmax_element(row, row_end);
                    const int32_t lo = *mm.first, hi = *mm.second;
                    const size_t d = static_cast<size_t>(row_end - row);
                    nb.clear();
                    if (lo >= 0 && hi < ncore &&
                        static_cast<size_t>((hi >> 6) - (lo >> 6) + 1) <= 4 * d) {
                        if (rowbits.empty()) rowbits.assign((static_cast<size_t>(ncore) + 63) / 64, 0);
                        for (const int32_t* it = row; it != row_end; ++it)
                            rowbits[static_cast<size_t>(*it) >> 6] |= 1ULL << (*it & 63);
                        for (int32_t wd = lo >> 6; wd <= (hi >> 6); ++wd) {
                            for (uint64_t bits = rowbits[wd]; bits; bits &= bits - 1)
                                nb.push_back(wd * 64 + __builtin_ctzll(bits));
                            rowbits[wd] = 0;
                        }
                    } else {
                        nb.assign(row, row_end);
                        std::sort(nb.begin(), nb.end());
                    }
                    row = nb.data();
                    row_end = nb.data() + nb.size();
                }
                // eight neighbours at a time: masks of the untaken ones for the
                // whole row, then the set bits in order (each rechecked, since
                // taking one can affect a later equal neighbour)
                auto visit = [&](int32_t x) {
                    if (static_cast<uint32_t>(x) >= static_cast<uint32_t>(ncore)) {  // -1 from core_ranks:
                        nonsym = true;                                                // not symmetric
                        return;
                    }
                    if ((ctaken[static_cast<size_t>(x) >> 6] >> (x & 63)) & 1ULL) return;
                    if (wcur + cw32[x] > T) return;
                    take(x);
                };
                const size_t nb = static_cast<size_t>(row_end - row) / 8;
                if (masks.size() < nb) masks.resize(nb);
                if (use_avx2)
                    untaken_masks_avx2(row, nb, reinterpret_cast<const uint32_t*>(ctaken.data()),
                                       static_cast<uint32_t>(ncore), masks.data());
                else
                    untaken_masks_scalar(row, nb, ctaken.data(), static_cast<uint32_t>(ncore), masks.data());
                for (size_t j = 0; j < nb; ++j) {
                    uint32_t m = masks[j];
                    while (m) {
                        const int q = __builtin_ctz(m);
                        m &= m - 1;
                        visit(row[8 * j + q]);
                    }
                }
                for (const int32_t* it = row + 8 * nb; it != row_end; ++it) visit(*it);
            }
            from = si + 1;
        }
        wb[b] = wcur;
    }
    bstart[k > 1 ? k - 1 : 0] = ntaken;
    if (nonsym || bad.load()) fail(SCLAP_ERR_NOT_SYMMETRIC, "initial partition: a neighbour has no neighbours");
    parallel_for(std::max(k - 1, 1), ntask == 1 ? 1 : nthr, [&](int32_t b) {  // small graphs: this thread
        if (b + 1 >= k) return;
        for (size_t i = bstart[b]; i < bstart[b + 1]; ++i) part[seed_node[order[i]]] = b;
    });
    const double t_bfs = ms_since(T0);
    // unassigned nodes in id order (compacted per task, then concatenated)
    std::fill(task_cnt.begin(), task_cnt.end(), 0);
    parallel_for(ntask, nthr, [&](int32_t t) {
        size_t w0, w1;
        task_words(t, w0, w1);
        int32_t cnt = 0;
        const int32_t v1 = std::min<int32_t>(n, static_cast<int32_t>(w1 * 64));
        for (int32_t v = static_cast<int32_t>(w0 * 64); v < v1; ++v) cnt += part[v] < 0;
        task_cnt[t + 1] = cnt;
    });
    for (int32_t t = 0; t < ntask; ++t) task_cnt[t + 1] += task_cnt[t];
    const size_t nrest = static_cast<size_t>(task_cnt[ntask]);
    std::unique_ptr<int32_t[]> rest_buf(new int32_t[std::max<size_t>(nrest, 1)]);  // filled below
    int32_t* const rest = rest_buf.get();
    parallel_for(ntask, nthr, [&](int32_t t) {
        size_t w0, w1;
        task_words(t, w0, w1);
        int32_t r = task_cnt[t];
        const int32_t v1 = std::min<int32_t>(n, static_cast<int32_t>(w1 * 64));
        for (int32_t v = static_cast<int32_t>(w0 * 64); v < v1; ++v)
            if (part[v] < 0) rest[r++] = v;
    });
    const double t_rest = ms_since(T0);
    auto cw = [&](int32_t v) -> int64_t { return vw ? vw[v] : 1; };
    // runs of equal weight in the leftover order: their starts, found in
    // parallel (a run is dealt as one unit below)
    std::vector<std::vector<size_t>> task_starts(static_cast<size_t>(ntask));
    if (vw) {
        parallel_for(ntask, nthr, [&](int32_t t) {
            const size_t a0 = nrest * static_cast<size_t>(t) / ntask, a1 = nrest * static_cast<size_t>(t + 1) / ntask;
            for (size_t q = std::max<size_t>(a0, 1); q < a1; ++q)
                if (vw[rest[q]] != vw[rest[q - 1]]) task_starts[t].push_back(q);
        });
    }
    std::vector<size_t> run_end;  // end of each run, in order
    for (const auto& ts : task_starts) run_end.insert(run_end.end(), ts.begin(), ts.end());
    run_end.push_back(nrest);
    // blocks by (weight, id); kept across runs and repaired by insertion
    // (a run changes the weights of a few blocks only), rebuilt after the
    // node-by-node path
    std::vector<int32_t> ord(static_cast<size_t>(k)), ord_next(static_cast<size_t>(k));
    bool ord_ok = false;
    auto lighter = [&](int32_t x, int32_t y) { return wb[x] != wb[y] ? wb[x] < wb[y] : x < y; };
    auto order_blocks = [&]() {
        if (!ord_ok) {
            for (int32_t b = 0; b < k; ++b) ord[b] = b;
            std::sort(ord.begin(), ord.end(), lighter);
            ord_ok = true;
            return;
        }
        for (int32_t a = 1; a < k; ++a) {
            const int32_t x = ord[a];
            int32_t q = a - 1;
            while (q >= 0 && lighter(x, ord[q])) {
                ord[q + 1] = ord[q];
                --q;
            }
            ord[q + 1] = x;
        }
    };
    BlockHeap heap(wb);  // kept in step with wb by the node-by-node path
    bool heap_ok = true;
    // a dealt run: node t of rest[i, i + take) goes to plan_ord[at + t mod gsz];
    // the block weights are advanced here and the labels written afterwards,
    // in parallel
    struct DealPlan {
        size_t i, take, at;
        int32_t gsz;
    };
    std::vector<DealPlan> plans;
    std::vector<int32_t> plan_ord;
    size_t i = 0;
    size_t nruns = 0, nheap = 0;
    while (i < nrest) {
        const int64_t c = cw(rest[i]);
        const size_t j = run_end[nruns];
        ++nruns;
        if (c == 0 || k > 4096 || j - i < 4 * static_cast<size_t>(k)) {  // node by node
            nheap += j - i;
            if (ord_ok && j - i <= 2) {
                // a node or two (typically one heavier node between runs of
                // equal weight): with the order repaired (a dealt run leaves
                // it stale), the lightest block is ord[0]; it moves right
                // past the blocks that are now lighter, keeping the order
                order_blocks();
                for (; i < j; ++i) {
                    const int32_t b = ord[0];
                    part[rest[i]] = b;
                    wb[b] += c;
                    int32_t q = 0;
                    while (q + 1 < k && lighter(ord[q + 1], b)) {
                        ord[q] = ord[q + 1];
                        ++q;
                    }
                    ord[q] = b;
                }
                heap_ok = false;
                continue;
            }
            if (!heap_ok) {
                heap.reset(wb);
                heap_ok = true;
            }
            ord_ok = false;
            for (; i < j; ++i) {
                const int32_t b = heap.top();
                part[rest[i]] = b;
                wb[b] += c;
                heap.add_to_top(c);
            }
            continue;
        }
        heap_ok = false;
        while (i < j) {
            order_blocks();
            const int64_t m0 = wb[ord[0]];
            int32_t gsz = 1;
            while (gsz < k && wb[ord[gsz]] < m0 + c) ++gsz;
            size_t take = j - i;
            if (gsz < k) {
                const int32_t X = ord[gsz];
                const int64_t wx = wb[X];
                uint64_t before = 0;
                for (int32_t t = 0; t < gsz; ++t) {
                    const int32_t g = ord[t];
                    const int64_t d = wx - wb[g];  // >= 0: g is not heavier than X
                    if (c == 1) {
                        before += static_cast<uint64_t>(d + (g < X ? 1 : 0));
                    } else {
                        const int64_t q = d / c, r = d - q * c;
                        before += static_cast<uint64_t>(q + (r != 0 ? 1 : 0) + ((r == 0 && g < X) ? 1 : 0));
                    }
                }
                take = std::min<size_t>(take, static_cast<size_t>(before));
            }
            // node t of the run goes to ord[t mod gsz]
            plans.push_back(DealPlan{i, take, plan_ord.size(), gsz});
            plan_ord.insert(plan_ord.end(), ord.begin(), ord.begin() + gsz);
            for (int32_t g = 0; g < gsz; ++g)
                wb[ord[g]] += c * static_cast<int64_t>(take / gsz + (static_cast<size_t>(g) < take % gsz ? 1 : 0));
            // the order is now three sorted runs (the blocks that took one
            // node more, the rest of the group, the blocks outside it): one
            // three-way merge restores it
            {
                const int32_t r = static_cast<int32_t>(take % static_cast<size_t>(gsz));
                int32_t a = 0, b2 = r, c2 = gsz;
                for (int32_t o = 0; o < k; ++o) {
                    int32_t w = -1, from = -1;
                    if (a < r) {
                        w = ord[a];
                        from = 0;
                    }
                    if (b2 < gsz && (from < 0 || lighter(ord[b2], w))) {
                        w = ord[b2];
                        from = 1;
                    }
                    if (c2 < k && (from < 0 || lighter(ord[c2], w))) {
                        w = ord[c2];
                        from = 2;
                    }
                    ord_next[o] = w;
                    if (from == 0) ++a;
                    else if (from == 1) ++b2;
                    else ++c2;
                }
                ord.swap(ord_next);
            }
            i += take;
        }
    }
    // labels of the dealt runs: nodes split evenly over the threads
    if (!plans.empty()) {
        std::vector<size_t> pstart(plans.size() + 1, 0);
        for (size_t q = 0; q < plans.size(); ++q) pstart[q + 1] = pstart[q] + plans[q].take;
        const size_t total = pstart.back();
        const int32_t nt = total < (1u << 20) ? 1 : 4 * nthr;  // starting threads costs more below
        parallel_for(nt, nthr, [&](int32_t t) {
            const size_t a0 = total * static_cast<size_t>(t) / nt, a1 = total * static_cast<size_t>(t + 1) / nt;
            size_t q = static_cast<size_t>(std::upper_bound(pstart.begin(), pstart.end(), a0) - pstart.begin()) - 1;
            for (size_t a = a0; a < a1; ++q) {
                const DealPlan& P = plans[q];
                const size_t t0 = a - pstart[q];
                const size_t t1 = std::min(P.take, a1 - pstart[q]);
                const int32_t* r0 = rest + P.i;
                const int32_t* o = plan_ord.data() + P.at;
                const size_t gsz = static_cast<size_t>(P.gsz);
                size_t g = t0 % gsz;
                for (size_t x = t0; x < t1; ++x) {
                    part[r0[x]] = o[g];
                    if (++g == gsz) g = 0;
                }
                a = pstart[q] + t1;
            }
        });
    }
    static const bool trace = std::getenv("SCLAP_TRACE") != nullptr;
    if (trace)
        fprintf(stderr,
                "[sclap] host partition phases: scan %.1f, tree %.1f, core %.1f (%d nodes), growth %.1f, rest %.1f "
                "(%zu nodes), dealing %.1f ms (%zu runs, %zu nodes one by one)\n",
                t_pre, t_tree - t_pre, t_seed - t_tree, ncore, t_bfs - t_seed, t_rest - t_bfs, nrest,
                ms_since(T0) - t_rest, nruns, nheap);
}

// ------------------------------------------------------------ multilevel

namespace {

bool trace_on() {
    static const bool on = std::getenv("SCLAP_TRACE") != nullptr;
    return on;
}

// Page-locked host staging for the coarsest graph.  One buffer is kept for
// the process and reused by whichever call holds it (pinning fresh memory on
// every call costs more than the copy it speeds up); a call that finds it
// busy uses ordinary uninitialised host memory instead.
class HostStage {
  public:
    explicit HostStage(size_t bytes) : lk_(mu(), std::try_to_lock) {
        if (lk_.owns_lock()) {
            if (cap() < bytes) {
                if (buf()) (void)hipHostFree(buf());
                buf() = nullptr;
                cap() = 0;
                void* p = nullptr;
                if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess) {
                    buf() = static_cast<char*>(p);
                    cap() = bytes;
                } else {
                    (void)hipGetLastError();
                }
            }
            if (buf()) {
                data_ = buf();
                return;
            }
            lk_.unlock();
        }
        own_.reset(new char[bytes]);
        data_ = own_.get();
    }
    char* data() const { return data_; }
    bool pinned() const { return lk_.owns_lock(); }

  private:
    static std::mutex& mu() {
        static std::mutex m;
        return m;
    }
    static char*& buf() {
        static char* b = nullptr;
        return b;
    }
    static size_t& cap() {
        static size_t c = 0;
        return c;
    }
    std::unique_lock<std::mutex> lk_;
    std::unique_ptr<char[]> own_;
    char* data_ = nullptr;
};

}  // namespace

namespace {

struct Level {
    OwnedDevGraph own;
    DevGraph g;
    DBuf<int32_t> C;  // map to the next coarser level
};

}  // namespace

double ms_since(Clock::time_point t) { return std::chrono::duration<double, std::milli>(Clock::now() - t).count(); }

namespace {

// Weight arrays that hold only ones are dropped (read as implicit ones), so
// the level-0 rounds do not stream them.
void drop_unit_weights(DevGraph& g, hipStream_t s) {
    if (g.ew && all_in_range(g.ew, g.S, 1, 2, s)) g.ew = nullptr;
    if (g.vw && all_in_range(g.vw, g.n, 1, 2, s)) g.vw = nullptr;
}

}  // namespace

namespace {

// One multilevel cycle (Section 4.5).  blk0 (device) is null in the first
// cycle; in later ones it holds the previous cycle's partition: clustering
// then stays inside its blocks (on the subgraph of intra-block slots), every
// coarse node inherits the block of its members, and the inherited partition
// of the coarsest graph replaces the initial partitioner (it has the cut and
// the block weights of blk0, since no cut edge was contracted).  blk0 may
// alias part_out.  Per-level statistics describe this cycle; visits and
// times add up.
void multilevel_cycle(const DevGraph& g0, int32_t k, int64_t cV, int64_t cmax0, int64_t Lmax, uint64_t seed,
                      const Opts& o, const int32_t* blk0, int32_t* part_out, sclap_stats* st, double& lp_ms,
                      hipStream_t s) {
    const int64_t W = cV / (static_cast<int64_t>(o.divisor) * k);
    std::memset(st->level_n, 0, sizeof(st->level_n));
    std::memset(st->level_S, 0, sizeof(st->level_S));
    std::memset(st->cluster_rounds, 0, sizeof(st->cluster_rounds));
    std::memset(st->refine_rounds, 0, sizeof(st->refine_rounds));
    std::vector<Level> L(1);
    std::vector<DBuf<int32_t>> blk(1);  // inherited blocks of levels >= 1
    auto blk_of = [&](int32_t l) -> const int32_t* { return l == 0 ? blk0 : blk[l].get(); };
    L[0].g = g0;
    st->level_n[0] = g0.n;
    st->level_S[0] = g0.S;
    auto t_coarsen = Clock::now();
    int32_t lev = 0;
    while (L[lev].g.n > o.coarsest && lev < o.max_levels) {
        const DevGraph G = L[lev].g;
        const int32_t n = G.n;
        int64_t cvl = 0, cmax = cmax0;
        if (lev > 0) node_weight_stats(G, &cvl, &cmax, s);
        const int64_t U = std::max(cmax, W);
        DBuf<int32_t> labels(n, s), w(n, s);
        iota_u32(reinterpret_cast<uint32_t*>(labels.get()), n, s);
        label_weights(G, labels.get(), w.get(), n, s);
        OwnedDevGraph inside;
        DevGraph Gc = G;  // the graph clustering looks at
        if (blk0) {
            within_blocks(G, blk_of(lev), inside, s);
            Gc = inside.view();
            Gc.vw = G.vw;
        }
        DBuf<int32_t> dcol;
        if (o.degree_order) {
            dcol.alloc(n, s);
            degree_colors(Gc, 1, nullptr, nullptr, nullptr, o.nsub, dcol.get(), s);
        }
        auto t_lp = Clock::now();
        const LPResult r = run_lp(Gc, kCluster, lev, seed, o.nsub, o.coarsen_rounds, U, labels.get(), w.get(), n,
                                  dcol.get(), o.tune, s);
        lp_ms += ms_since(t_lp);
        inside = OwnedDevGraph();
        st->visits += r.visits;
        st->cluster_rounds[lev] = r.rounds_run;
        w.release();
        DBuf<int32_t> C(n, s);
        Level nx;
        contract(G, labels.get(), C.get(), nx.own, s, nullptr, 0, nullptr, false, o.bucket_mean);
        if (nx.own.n >= n) break;  // no shrink: keep the current level as the coarsest
        DBuf<int32_t> cb;
        if (blk0) {
            cb.alloc(std::max(nx.own.n, 1), s);
            inherit_blocks(n, C.get(), blk_of(lev), cb.get(), s);
        }
        L[lev].C = std::move(C);
        nx.g = nx.own.view();
        L.push_back(std::move(nx));
        blk.push_back(std::move(cb));
        ++lev;
        st->level_n[lev] = L[lev].g.n;
        st->level_S[lev] = L[lev].g.S;
        if (20LL * L[lev].g.n > 19LL * n) break;  // stalled
    }
    st->levels = lev;
    // inner levels keep their rows unordered; the initial partition grows
    // blocks along ascending neighbour ids, so order the coarsest graph's rows
    if (lev > 0 && !blk0 && o.initial == 0) sort_rows(L[lev].own, s);
    HIPCHK(hipStreamSynchronize(s));
    st->ms_coarsen += ms_since(t_coarsen);

    auto t_init = Clock::now();
    const DevGraph Gc = L[lev].g;
    const int32_t nc = Gc.n;
    DBuf<int32_t> cur;
    int32_t* curp = part_out;
    if (lev > 0) {
        cur.alloc(nc, s);
        curp = cur.get();
    }
    if (blk0) {
        // the inherited partition of the coarsest graph
        if (nc > 0 && curp != blk_of(lev))
            HIPCHK(hipMemcpyAsync(curp, blk_of(lev), nc * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    } else if (o.initial == 1) {
        // on the device: label propagation from hashed seeds
        const int64_t T = (cV + k - 1) / k;
        const LPResult r = device_initial_partition(Gc, k, T, Lmax, seed, lev, o.nsub, o.refine_rounds, o.tune, curp, s);
        st->visits += r.visits;
    } else {
        // initial partition of the coarsest graph on the host
        const size_t bx = (static_cast<size_t>(nc) + 1) * sizeof(int64_t);
        const size_t ba = static_cast<size_t>(std::max<int64_t>(Gc.S, 1)) * sizeof(int32_t);
        const size_t bn = static_cast<size_t>(std::max(nc, 1)) * sizeof(int32_t);
        HostStage stage(bx + ba + 2 * bn);
        int64_t* hx = reinterpret_cast<int64_t*>(stage.data());
        int32_t* ha = reinterpret_cast<int32_t*>(stage.data() + bx);
        int32_t* hv = reinterpret_cast<int32_t*>(stage.data() + bx + ba);
        int32_t* hp = reinterpret_cast<int32_t*>(stage.data() + bx + ba + bn);
        DBuf<int32_t> ranked;  // the adjacency renumbered to the positive-degree core
        if (nc > 0) {
            HIPCHK(hipMemcpyAsync(hx, Gc.xadj, bx, hipMemcpyDeviceToHost, s));
            if (Gc.S > 0) {
                ranked.alloc(Gc.S, s);
                core_ranks(Gc, ranked.get(), s);
                HIPCHK(hipMemcpyAsync(ha, ranked.get(), Gc.S * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            }
            if (Gc.vw) HIPCHK(hipMemcpyAsync(hv, Gc.vw, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        const double ms_d2h = ms_since(t_init);
        const int64_t T = (cV + k - 1) / k;
        // rows of contracted levels are sorted by construction
        host_initial_partition(nc, hx, ha, Gc.vw ? hv : nullptr, k, T, hp, lev > 0, true);
        const double ms_ip = ms_since(t_init) - ms_d2h;
        if (nc > 0) HIPCHK(hipMemcpyAsync(curp, hp, nc * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // the staging buffer is released below
        if (trace_on())
            fprintf(stderr, "[sclap] initial partition: n=%d S=%lld pinned=%d copy-in %.1f ms, partition %.1f ms\n",
                    nc, static_cast<long long>(Gc.S), stage.pinned() ? 1 : 0, ms_d2h, ms_ip);
    }
    HIPCHK(hipStreamSynchronize(s));
    st->ms_initial += ms_since(t_init);

    auto t_ref = Clock::now();
    DBuf<int32_t> w(k, s);
    for (int32_t l = lev; l >= 0; --l) {
        const DevGraph G = L[l].g;
        if (l < lev) {
            DBuf<int32_t> fine;
            int32_t* finep = part_out;
            if (l > 0) {
                fine.alloc(G.n, s);
                finep = fine.get();
            }
            project(G.n, L[l].C.get(), curp, finep, s);
            cur = std::move(fine);
            curp = finep;
            L[l + 1].own = OwnedDevGraph();  // the coarser graph is no longer needed
            blk[l + 1].release();
            L[l].C.release();
        }
        label_weights(G, curp, w.get(), k, s);
        auto t_lp = Clock::now();
        const LPResult r = run_lp(G, kRefine, l, seed, o.nsub, o.refine_rounds, Lmax, curp, w.get(), k, nullptr,
                                  o.tune, s);
        lp_ms += ms_since(t_lp);
        st->visits += r.visits;
        st->refine_rounds[l] = r.rounds_run;
    }
    HIPCHK(hipStreamSynchronize(s));
    st->ms_refine += ms_since(t_ref);
}

}  // namespace

uint64_t cycle_seed(uint64_t seed, int32_t cycle) {
    if (cycle == 0) return seed;
    return hash_prefix({seed, 4, static_cast<uint64_t>(static_cast<uint32_t>(cycle))});
}

int partition_impl(const DevGraph& g0_in, int32_t k, double eps, uint64_t seed, const Opts& o, int32_t* part_out,
                   int64_t* cut, int64_t* bw, sclap_stats* stats, hipStream_t s) {
    DevGraph g0 = g0_in;
    check_k_eps(k, eps);
    if (!part_out && g0.n > 0) fail(SCLAP_ERR_INVALID, "part is NULL");
    if (!cut || !bw) fail(SCLAP_ERR_INVALID, "cut / block_w is NULL");
    int64_t cV = 0, cmax0 = 0;
    check_graph(g0, o.validate != 0, &cV, &cmax0, s);
    drop_unit_weights(g0, s);
    sclap_stats local;
    sclap_stats* st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    const int64_t Lmax = lmax_of(cV, k, eps);
    double lp_ms = 0;
    for (int32_t c = 0; c < o.vcycles; ++c)
        multilevel_cycle(g0, k, cV, cmax0, Lmax, cycle_seed(seed, c), o, c == 0 ? nullptr : part_out, part_out, st,
                         lp_ms, s);
    auto t_cut = Clock::now();
    cut_and_weights(g0, part_out, k, cut, bw, s);
    st->ms_refine += ms_since(t_cut);
    st->ms_lp = lp_ms;
    for (int32_t b = 0; b < k; ++b)
        if (bw[b] > Lmax) return SCLAP_WARN_IMBALANCED;
    return SCLAP_OK;
}

// ------------------------------------------------------------- tuning

LPTuning autotune(const DevGraph& g_in, int32_t k, const Opts& o, hipStream_t s) {
    check_k_eps(k, 0.0);
    DevGraph g = g_in;
    int64_t cV = 0, cmax = 0;
    check_graph(g, false, &cV, &cmax, s);
    drop_unit_weights(g, s);
    LPTuning best = o.tune;
    if (g.n == 0) return best;
    const int64_t U = std::max(cmax, cV / (static_cast<int64_t>(o.divisor) * k));
    const int64_t Lmax = lmax_of(cV, k, 0.03);
    DBuf<int32_t> labels(g.n, s), w(std::max<int64_t>(g.n, k), s);
    std::vector<int32_t> hpart(g.n);
    for (int32_t v = 0; v < g.n; ++v) hpart[v] = static_cast<int32_t>(static_cast<int64_t>(v) * k / g.n);
    DBuf<int32_t> part0(g.n, s), part(g.n, s);
    HIPCHK(hipMemcpyAsync(part0.get(), hpart.data(), g.n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // The objective: one clustering round from singletons plus one refinement
    // round of a k-way partition (contiguous id ranges), the faster of two
    // timings.  Neither depends on the knobs' values, only their time does.
    auto measure = [&](const LPTuning& t) {
        double ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            iota_u32(reinterpret_cast<uint32_t*>(labels.get()), g.n, s);
            label_weights(g, labels.get(), w.get(), g.n, s);
            HIPCHK(hipMemcpyAsync(part.get(), part0.get(), g.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipEventRecord(e0, s));
            run_lp(g, kCluster, 0, 1, o.nsub, 1, U, labels.get(), w.get(), g.n, nullptr, t, s);
            label_weights(g, part.get(), w.get(), k, s);
            run_lp(g, kRefine, 0, 1, o.nsub, 1, Lmax, part.get(), w.get(), k, nullptr, t, s);
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float f = 0;
            HIPCHK(hipEventElapsedTime(&f, e0, e1));
            ms = std::min(ms, static_cast<double>(f));
        }
        return ms;
    };
    // Coordinate search from the library defaults.  The degree thresholds
    // decide which kernel, and so which LDS table, a row gets: one lane and
    // registers (degree <= lane_max), 16, 32 or 64 lanes with 64-, 128- and
    // 512-entry tables (<= wave_max), one workgroup with 2048-, 8192- or
    // 10240-entry tables (<= block_max), above that the hub chunks; the table
    // size of the longest-row workgroup bucket (10240 or 16384 entries) is
    // searched as well; the capture choice decides whether the rounds run as
    // one HIP graph.  A value is taken only if it is at least 3 % faster than
    // the current best.
    best.lane_max = 16;
    best.wave_max = 256;
    best.block_max = 8192;
    best.block_table = 10240;
    double best_ms = measure(best);
    auto try_values = [&](int32_t LPTuning::*field, std::initializer_list<int32_t> values) {
        const int32_t keep = best.*field;
        for (int32_t val : values) {
            if (val == keep) continue;
            LPTuning t = best;
            t.*field = val;
            const double ms = measure(t);
            if (ms < 0.97 * best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    };
    try_values(&LPTuning::capture, {1, -1});
    try_values(&LPTuning::block_max, {1024, 2048, 4096});
    try_values(&LPTuning::wave_max, {32, 64, 128});
    try_values(&LPTuning::lane_max, {4, 8});
    try_values(&LPTuning::block_table, {16384});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// ------------------------------------------------------------- batches
//
// Many graphs partitioned together: the graphs of a batch are one CSR with a
// node range per graph and no edge between ranges.  Every level runs each
// kernel once for all graphs; hashes, orders and bounds are per graph
// (graph-local ids, own seed, U and Lmax), so every graph gets exactly the
// result it gets alone.  A graph leaves the coarsening loop by its own stop
// rule; later levels hold only the graphs still coarsening.

namespace {

struct BatchLevel {
    OwnedDevGraph own;
    DevGraph g;
    std::vector<int32_t> ids;  // batch index of each member graph
    std::vector<int32_t> nb;   // first node of each member, then n
    std::vector<int64_t> sb;   // first slot of each member, then S
    DBuf<int32_t> gid;         // [n] batch index of each node
    DBuf<int32_t> C;           // [n] node of the next level, -1 where the graph ends here
};

template <typename T>
void upload_vec(DBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
    if (h.empty()) return;
    HIPCHK(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Host initial partitions of a batch, overlapped with coarsening.  As soon
// as coarsening decides which graphs end at a level, their slices are packed
// on the device (neighbours as core ranks) and copied to pinned host memory,
// one copy per array, and a task of its own partitions them (one graph per
// host thread, largest first) while the device coarsens the levels below;
// the levels decided last (usually two at the end of coarsening) run side by
// side.  Refinement of a level waits only for that level's partitions, which
// go back in one copy and are scattered into the level's layout on the
// device.
class HostIpPipeline {
  public:
    // stage_bytes bounds the packed levels together (every graph ends at one
    // level, no larger there than at level 0)
    HostIpPipeline(size_t stage_bytes, const int32_t* k, const std::vector<int64_t>& T, const std::vector<int32_t>& kb,
                   hipStream_t s)
        : stage_(stage_bytes), cap_(stage_bytes), k_(k), T_(T), kb_(kb), s_(s) {
        const unsigned hw = std::thread::hardware_concurrency();
        threads_ = static_cast<int32_t>(std::min(16u, hw ? hw : 1u));
        lv_.resize(static_cast<size_t>(SCLAP_MAX_LEVELS) + 1);
        HIPCHK(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking));
    }
    HostIpPipeline(const HostIpPipeline&) = delete;
    HostIpPipeline& operator=(const HostIpPipeline&) = delete;
    ~HostIpPipeline() {
        closed_.store(true);
        for (auto& L : lv_)
            if (L && L->task.valid()) L->task.wait();
        (void)hipStreamSynchronize(cs_);  // copies still reading the packed levels
        for (auto& L : lv_)
            if (L && L->ev) (void)hipEventDestroy(L->ev);
        (void)hipStreamDestroy(cs_);
    }

    // The members `members` (indices into B) end at level l.
    void stage(int32_t l, const BatchLevel& B, const std::vector<int32_t>& members) {
        std::unique_ptr<Level> lv(new Level);
        Level& L = *lv;
        L.ready = L.done.get_future().share();
        const int32_t Mk = static_cast<int32_t>(members.size());
        L.nnb.push_back(0);
        L.nsb.push_back(0);
        std::vector<int64_t> osb;
        for (int32_t m : members) {
            L.gids.push_back(B.ids[m]);
            L.onb.push_back(B.nb[m]);
            osb.push_back(B.sb[m]);
            L.nnb.push_back(L.nnb.back() + (B.nb[m + 1] - B.nb[m]));
            L.nsb.push_back(L.nsb.back() + (B.sb[m + 1] - B.sb[m]));
        }
        L.n = L.nnb[Mk];
        const int64_t S = L.nsb[Mk];
        if (L.n > 0) {
            L.dx.alloc(static_cast<size_t>(L.n) + Mk, s_);
            L.da.alloc(static_cast<size_t>(std::max<int64_t>(S, 1)), s_);
            if (B.g.vw) L.dv.alloc(L.n, s_);
            pack_members_for_host(B.g, L.onb, osb, L.nnb, L.nsb, L.dx.get(), L.da.get(), L.dv.get(), s_);  // syncs
            L.x = take<int64_t>(static_cast<size_t>(L.n) + Mk);
            L.a = take<int32_t>(static_cast<size_t>(S));
            L.v = B.g.vw ? take<int32_t>(L.n) : nullptr;
            L.p = take<int32_t>(L.n);
            // on a stream of their own, beside the coarsening of the next level
            HIPCHK(hipMemcpyAsync(L.x, L.dx.get(), (static_cast<size_t>(L.n) + Mk) * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, cs_));
            if (S > 0)
                HIPCHK(hipMemcpyAsync(L.a, L.da.get(), static_cast<size_t>(S) * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      cs_));
            if (L.v) HIPCHK(hipMemcpyAsync(L.v, L.dv.get(), L.n * sizeof(int32_t), hipMemcpyDeviceToHost, cs_));
            HIPCHK(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
            HIPCHK(hipEventRecord(L.ev, cs_));
            // where the partitions go back: nnb | onb on the device
            L.dnb.alloc(2 * static_cast<size_t>(Mk) + 1, s_);
            HIPCHK(hipMemcpyAsync(L.dnb.get(), L.nnb.data(), (Mk + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s_));
            HIPCHK(hipMemcpyAsync(L.dnb.get() + Mk + 1, L.onb.data(), Mk * sizeof(int32_t), hipMemcpyHostToDevice,
                                  s_));
        }
        L.t_staged = ms_since(t0_);
        Level* lp = lv.get();
        lv_[l] = std::move(lv);
        lp->task = std::async(std::launch::async, [this, lp, l] { work(*lp, l); });
    }

    // Waits for level l's partitions and writes them into part (the level's
    // layout, labels in the batch's block space).  Returns the ms waited.
    double finish(int32_t l, int32_t* part) {
        Level* L = lv_[l].get();  // staged by this thread
        if (!L) fail(SCLAP_ERR_INVALID, "batch level without initial partitions");
        const auto t = Clock::now();
        L->ready.get();  // rethrows the helper's error
        const double waited = ms_since(t);
        if (L->n > 0) {
            L->dp.alloc(L->n, s_);
            HIPCHK(hipMemcpyAsync(L->dp.get(), L->p, L->n * sizeof(int32_t), hipMemcpyHostToDevice, s_));
            unpack_members(L->dp.get(), L->n, static_cast<int32_t>(L->onb.size()), L->dnb.get(), part, s_);
        }
        return waited;
    }

  private:
    struct Level {
        int32_t n = 0;
        std::vector<int32_t> gids, onb, nnb;  // batch index, old and packed node base of each member
        std::vector<int64_t> nsb;             // packed slot base
        DBuf<int64_t> dx;                     // packed on the device
        DBuf<int32_t> da, dv, dnb, dp;
        int64_t* x = nullptr;  // pinned host copies
        int32_t *a = nullptr, *v = nullptr, *p = nullptr;
        hipEvent_t ev = nullptr;  // the copies to the host have landed
        double t_staged = 0, t_start = 0, t_copied = 0, t_done = 0;  // ms since the pipeline started
        std::promise<void> done;
        std::shared_future<void> ready;
        std::future<void> task;  // the host partitioning of this level
    };

    template <typename T>
    T* take(size_t count) {
        const size_t bytes = (count * sizeof(T) + 7) & ~static_cast<size_t>(7);
        if (used_ + bytes > cap_) fail(SCLAP_ERR_INVALID, "batch staging area too small");
        T* p = reinterpret_cast<T*>(stage_.data() + used_);
        used_ += bytes;
        return p;
    }

    void work(Level& L, int32_t l) {
        try {
            L.t_start = ms_since(t0_);
            if (L.n > 0 && !closed_.load()) {
                HIPCHK(hipEventSynchronize(L.ev));
                L.t_copied = ms_since(t0_);
                partition(L);
            }
            L.t_done = ms_since(t0_);
            if (trace_on())
                fprintf(stderr, "[sclap] batch host partitions L%d: %zu graphs, %d nodes; staged %.1f, started %.1f, "
                        "copied %.1f, done %.1f ms\n", l, L.gids.size(), L.n, L.t_staged, L.t_start, L.t_copied,
                        L.t_done);
            L.done.set_value();
        } catch (...) {
            L.done.set_exception(std::current_exception());
        }
    }

    void partition(Level& L) {
        const int32_t Mk = static_cast<int32_t>(L.gids.size());
        std::vector<int32_t> order(Mk);
        for (int32_t m = 0; m < Mk; ++m) order[m] = m;
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            return L.nnb[x + 1] - L.nnb[x] > L.nnb[y + 1] - L.nnb[y];
        });
        parallel_for(Mk, threads_, [&](int32_t i) {
            const int32_t m = order[i];
            const int32_t nm = L.nnb[m + 1] - L.nnb[m];
            if (nm == 0) return;
            const int32_t g = L.gids[m];
            int32_t* pp = L.p + L.nnb[m];
            // rows of inner levels are unordered; neighbours come as core ranks
            host_initial_partition(nm, L.x + L.nnb[m] + m, L.a + L.nsb[m], L.v ? L.v + L.nnb[m] : nullptr, k_[g], T_[g],
                                   pp, false, true, 1);
            for (int32_t q = 0; q < nm; ++q) pp[q] += kb_[g];  // labels of the batch's block space
        });
    }

    HostStage stage_;
    Clock::time_point t0_ = Clock::now();
    size_t cap_, used_ = 0;
    const int32_t* k_;
    const std::vector<int64_t>& T_;
    const std::vector<int32_t>& kb_;
    hipStream_t s_;
    hipStream_t cs_ = nullptr;  // copies to the host (default priority)
    int32_t threads_ = 1;
    std::vector<std::unique_ptr<Level>> lv_;
    std::atomic<bool> closed_{false};  // being destroyed: levels not yet started are skipped
};

__global__ void pool_init_kernel(int32_t n, const int32_t* __restrict__ gid, const int32_t* __restrict__ pool,
                                 int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) part[v] = pool[gid[v]];
}

__global__ void seed_flag_kernel(int32_t n, const int64_t* __restrict__ xadj, const int32_t* __restrict__ gid,
                                 const uint8_t* __restrict__ act, int32_t* __restrict__ flag) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) flag[v] = (act[gid[v]] && xadj[v + 1] > xadj[v]) ? 1 : 0;
}

__global__ void batch_seed_keys_kernel(int32_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ rank,
                                       const int32_t* __restrict__ gid, const int32_t* __restrict__ nbase,
                                       const uint64_t* __restrict__ prefix, uint64_t* __restrict__ keys,
                                       uint32_t* __restrict__ vals, int32_t* __restrict__ gcount) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n || !flag[v]) return;
    const int32_t g = gid[v];
    keys[rank[v]] = mix64(prefix[g] ^ static_cast<uint64_t>(static_cast<uint32_t>(v - nbase[g])));
    vals[rank[v]] = static_cast<uint32_t>(v);
    atomicAdd(&gcount[g], 1);
}

__global__ void gid_keys_kernel(int32_t m, const uint32_t* __restrict__ vals, const int32_t* __restrict__ gid,
                                uint64_t* __restrict__ keys) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) keys[i] = static_cast<uint32_t>(gid[vals[i]]);
}

__global__ void batch_place_seeds_kernel(int32_t m, const uint32_t* __restrict__ vals, const int32_t* __restrict__ gid,
                                         const int32_t* __restrict__ start, const int32_t* __restrict__ kg,
                                         const int32_t* __restrict__ kb2, int32_t* __restrict__ part) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t v = static_cast<int32_t>(vals[i]);
    const int32_t g = gid[v];
    const int32_t r = i - start[g];
    if (r < kg[g]) part[v] = kb2[g] + r;
}

__global__ void pool_offset_kernel(int32_t G, const uint8_t* __restrict__ act, const int32_t* __restrict__ pool,
                                   int32_t* __restrict__ w, int32_t add) {
    const int32_t g = blockIdx.x * 256 + threadIdx.x;
    if (g < G && act[g]) w[pool[g]] += add;
}

__global__ void batch_pool_weight_kernel(int32_t n, const int32_t* __restrict__ gid, const uint8_t* __restrict__ act,
                                         const int32_t* __restrict__ pool, const int32_t* __restrict__ part,
                                         const int32_t* __restrict__ vw, int32_t* __restrict__ pw) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t g = gid[v];
    pw[v] = (act[g] && part[v] == pool[g]) ? (vw ? vw[v] : 1) : 0;
}

// blocks of the graphs that end here, in the batch's block space: pool nodes
// fill the remaining room of their graph's blocks by their prefix weight
__global__ void batch_deal_kernel(int32_t n, const int32_t* __restrict__ gid, const uint8_t* __restrict__ act,
                                  const int32_t* __restrict__ nbase, const int32_t* __restrict__ kg,
                                  const int32_t* __restrict__ kb2, const int32_t* __restrict__ kb,
                                  const int64_t* __restrict__ P, const int64_t* __restrict__ cum,
                                  int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t g = gid[v];
    if (!act[g]) return;
    int32_t local = part[v] - kb2[g];
    const int32_t k = kg[g];
    if (local == k) {
        const int64_t p = P[v] - P[nbase[g]];
        const int64_t* c = cum + kb2[g];
        int32_t lo = 0, hi = k;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (c[mid] > p) hi = mid;
            else lo = mid + 1;
        }
        local = lo < k ? lo : k - 1;
    }
    part[v] = kb[g] + local;
}

// The device initial partitioner for every graph of a batch level whose
// coarsest level this is (ending[g]), as device_initial_partition does for one
// graph: each graph gets k_g + 1 labels (its pool last) in a label space of
// its own, its seeds from its own hash, its own bound and rooms.  Writes the
// ending graphs' blocks, in the batch's block space, into part; the other
// nodes of the level are left for the projection.
LPResult batch_device_initial(const DevGraph& g, const int32_t* gid, const std::vector<int32_t>& ids,
                              const std::vector<int32_t>& nb, int32_t level, int32_t G, const int32_t* k,
                              const std::vector<int32_t>& kb, const std::vector<int64_t>& T,
                              const std::vector<int64_t>& cV, const std::vector<int64_t>& Lmax,
                              const std::vector<uint8_t>& ending, const std::vector<uint64_t>& cseed,
                              const uint64_t* d_seed, const int64_t* d_bound, const Opts& o, int32_t* part,
                              hipStream_t s) {
    constexpr int64_t kBig = int64_t(1) << 30;
    const int32_t n = g.n;
    std::vector<int32_t> kb2(static_cast<size_t>(G) + 1, 0), pool(G), nbase(G, 0), kg(k, k + G);
    for (int32_t x = 0; x < G; ++x) {
        kb2[x + 1] = kb2[x] + k[x] + 1;
        pool[x] = kb2[x] + k[x];
    }
    const int32_t K2 = kb2[G];
    std::vector<int32_t> lg(static_cast<size_t>(K2));
    for (int32_t x = 0; x < G; ++x)
        for (int32_t b = kb2[x]; b < kb2[x + 1]; ++b) lg[b] = x;
    std::vector<uint8_t> act(G, 0);
    std::vector<uint64_t> prefix(G, 0);
    int32_t max_labels = 1;
    for (size_t m = 0; m < ids.size(); ++m) {
        const int32_t x = ids[m];
        nbase[x] = nb[m];
        if (!ending[x]) continue;
        if (Lmax[x] >= kBig || cV[x] >= kBig) fail(SCLAP_ERR_INVALID, "device initial partition needs Lmax and c(V) below 2^30");
        act[x] = 1;
        prefix[x] = hash_prefix({cseed[x], 5, static_cast<uint64_t>(static_cast<uint32_t>(level))});
        max_labels = std::max(max_labels, k[x] + 1);
    }
    DBuf<int32_t> d_kb2(static_cast<size_t>(G) + 1, s), d_pool(G, s), d_nbase(G, s), d_kg(G, s), d_kb(G, s),
        d_lg(std::max(K2, 1), s), d_gcount(G, s), d_start(G, s);
    DBuf<uint8_t> d_act(G, s);
    DBuf<uint64_t> d_prefix(G, s);
    upload_vec(d_kb2, kb2, s);
    upload_vec(d_pool, pool, s);
    upload_vec(d_nbase, nbase, s);
    upload_vec(d_kg, kg, s);
    upload_vec(d_kb, std::vector<int32_t>(kb.begin(), kb.begin() + G), s);
    upload_vec(d_lg, lg, s);
    upload_vec(d_act, act, s);
    upload_vec(d_prefix, prefix, s);
    fill_i32(d_gcount.get(), 0, G, s);
    pool_init_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, d_pool.get(), part);
    LAUNCHCHK();
    // seeds: per graph the k smallest (hash, id) among its nodes with neighbours
    DBuf<int32_t> flag(n, s), rank(n, s), tot(1, s);
    seed_flag_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g.xadj, gid, d_act.get(), flag.get());
    LAUNCHCHK();
    exclusive_scan_i32(flag.get(), rank.get(), n, tot.get(), s);
    int32_t ncand = 0;
    HIPCHK(hipMemcpyAsync(&ncand, tot.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ncand > 0) {
        DBuf<uint64_t> keys(ncand, s), ktmp(ncand, s);
        DBuf<uint32_t> vals(ncand, s), vtmp(ncand, s);
        batch_seed_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, flag.get(), rank.get(), gid, d_nbase.get(),
                                                                d_prefix.get(), keys.get(), vals.get(),
                                                                d_gcount.get());
        LAUNCHCHK();
        RadixScratch rs;
        radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), ncand, 0, 64, rs, s);
        gid_keys_kernel<<<grid_for(ncand, 256), 256, 0, s>>>(ncand, vals.get(), gid, keys.get());
        LAUNCHCHK();
        radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), ncand, 0,
                         std::max(1, bits_for(static_cast<uint64_t>(std::max(G - 1, 1)))), rs, s);
        std::vector<int32_t> gc(G), start(G, 0);
        HIPCHK(hipMemcpyAsync(gc.data(), d_gcount.get(), G * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int32_t x = 1; x < G; ++x) start[x] = start[x - 1] + gc[x - 1];
        upload_vec(d_start, start, s);
        batch_place_seeds_kernel<<<grid_for(ncand, 256), 256, 0, s>>>(ncand, vals.get(), gid, d_start.get(),
                                                                      d_kg.get(), d_kb2.get(), part);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(s));  // start is read by the upload above
    }
    DBuf<int32_t> w(std::max(K2, 1), s);
    label_weights(g, part, w.get(), K2, s);
    pool_offset_kernel<<<grid_for(G, 256), 256, 0, s>>>(G, d_act.get(), d_pool.get(), w.get(), static_cast<int32_t>(kBig));
    LAUNCHCHK();
    MultiGraph mg;
    mg.G = G;
    mg.gid = gid;
    mg.lgid = d_lg.get();
    mg.max_labels = max_labels;
    mg.nbase = d_nbase.get();
    mg.lbase = d_kb2.get();
    mg.bound = d_bound;
    mg.seed = d_seed;
    mg.active = d_act.get();
    const LPResult r = run_lp(g, kInitial, level, 0, o.nsub, o.refine_rounds, 0, part, w.get(), K2, nullptr, o.tune, s,
                              &mg);
    // pools fill their graph's remaining room
    std::vector<int32_t> hw(static_cast<size_t>(std::max(K2, 1)));
    HIPCHK(hipMemcpyAsync(hw.data(), w.get(), std::max(K2, 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int64_t> cum(static_cast<size_t>(std::max(K2, 1)), 0);
    for (int32_t x = 0; x < G; ++x) {
        if (!act[x]) continue;
        int64_t run = 0;
        for (int32_t b = 0; b < k[x]; ++b) {
            const int64_t wb = hw[kb2[x] + b];
            run += wb < T[x] ? T[x] - wb : 0;
            cum[kb2[x] + b] = run;
        }
    }
    DBuf<int64_t> d_cum(std::max(K2, 1), s), P(n, s), ptot(1, s);
    upload_vec(d_cum, cum, s);
    batch_pool_weight_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, d_act.get(), d_pool.get(), part, g.vw,
                                                              flag.get());
    LAUNCHCHK();
    exclusive_scan_i32_to_i64(flag.get(), P.get(), n, ptot.get(), s);
    batch_deal_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, d_act.get(), d_nbase.get(), d_kg.get(), d_kb2.get(),
                                                       d_kb.get(), P.get(), d_cum.get(), part);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));  // the host vectors uploaded above stay alive until here
    return r;
}


}  // namespace

int partition_batch_impl(const DevGraph& g0_in, int32_t G, const int32_t* node_base, const int32_t* k,
                         const double* eps, const uint64_t* seed, const Opts& o_in, int32_t* part_out, int64_t* cut,
                         int64_t* bw, sclap_batch_stats* stats, hipStream_t s) {
    Opts o = o_in;
    DevGraph g0 = g0_in;
    // many small graphs converge early: skipping their quiet nodes pays off
    if (o.tune.skip_quiet == 0) o.tune.skip_quiet = 1;
    if (G < 1) fail(SCLAP_ERR_INVALID, "count must be >= 1");
    if (!node_base || !k || !eps || !seed) fail(SCLAP_ERR_INVALID, "node_base, k, eps or seed is NULL");
    if (node_base[0] != 0 || node_base[G] != g0.n) fail(SCLAP_ERR_INVALID, "node_base must run from 0 to n");
    std::vector<int32_t> kb(static_cast<size_t>(G) + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        if (node_base[g + 1] < node_base[g]) fail(SCLAP_ERR_INVALID, "node_base must be non-decreasing");
        check_k_eps(k[g], eps[g]);
        if (static_cast<int64_t>(kb[g]) + k[g] > (1 << 30)) fail(SCLAP_ERR_INVALID, "sum of k too large");
        kb[g + 1] = kb[g] + k[g];
    }
    const int32_t K = kb[G];
    if (!part_out && g0.n > 0) fail(SCLAP_ERR_INVALID, "part is NULL");
    if (!cut || !bw) fail(SCLAP_ERR_INVALID, "cut / block_w is NULL");
    sclap_batch_stats local;
    sclap_batch_stats* st = stats ? stats : &local;
    int32_t* graph_levels = st->graph_levels;
    std::memset(st, 0, sizeof(*st));
    st->graph_levels = graph_levels;
    auto t_coarsen = Clock::now();
    double lp_ms = 0;

    std::vector<BatchLevel> L(1);
    {
        BatchLevel& B = L[0];
        B.g = g0;
        B.ids.resize(G);
        for (int32_t g = 0; g < G; ++g) B.ids[g] = g;
        B.nb.assign(node_base, node_base + G + 1);
        B.sb = member_slot_bases(g0.xadj, B.nb, s);
        B.gid.alloc(std::max(g0.n, 1), s);
        member_ids(g0.n, B.nb, B.ids, B.gid.get(), s);
    }
    if (o.validate) {
        int64_t cVu = 0, cmu = 0;
        check_graph(g0, true, &cVu, &cmu, s);
        if (!members_closed(g0, L[0].nb, L[0].sb, s)) fail(SCLAP_ERR_INVALID, "an edge joins two graphs of the batch");
    }
    drop_unit_weights(g0, s);
    L[0].g = g0;
    std::vector<int64_t> cV(G), cmax0(G);
    graph_node_stats(g0.n, L[0].gid.get(), g0.vw, G, cV.data(), cmax0.data(), s);
    std::vector<int64_t> Lmax(G), W(G), T(G);
    for (int32_t g = 0; g < G; ++g) {
        if (cV[g] > 2147483647LL) fail(SCLAP_ERR_OVERFLOW, "node weight total of a graph exceeds 2^31-1");
        Lmax[g] = lmax_of(cV[g], k[g], eps[g]);
        W[g] = cV[g] / (static_cast<int64_t>(o.divisor) * k[g]);
        T[g] = (cV[g] + k[g] - 1) / k[g];
    }

    // per-graph device parameters
    DBuf<uint64_t> d_seed(G, s);
    DBuf<int64_t> d_bound(G, s);
    DBuf<int32_t> d_lbase(G, s), d_nbase(G, s), d_kb(G, s);
    DBuf<uint8_t> d_active(G, s);
    upload_vec(d_kb, std::vector<int32_t>(kb.begin(), kb.begin() + G), s);
    std::vector<int32_t> lgid(std::max(K, 1));
    for (int32_t g = 0; g < G; ++g)
        for (int32_t b = kb[g]; b < kb[g + 1]; ++b) lgid[b] = g;
    DBuf<int32_t> d_lgid(std::max(K, 1), s);
    upload_vec(d_lgid, lgid, s);
    DBuf<int32_t> w(std::max(K, 1), s);

    // Multilevel cycles (Section 4.4, Iterated Multilevel Schemes): from the second on, part_out holds the
    // previous cycle's partition in the batch's block space; clustering stays
    // inside its blocks and the inherited coarsest partitions replace the
    // initial partitioner, as in multilevel_cycle.
    for (int32_t cyc = 0; cyc < o.vcycles; ++cyc) {
        const int32_t* carry = cyc == 0 ? nullptr : part_out;
        std::vector<uint64_t> cseed(G);
        for (int32_t g = 0; g < G; ++g) cseed[g] = cycle_seed(seed[g], cyc);
        upload_vec(d_seed, cseed, s);
        L.resize(1);
        std::vector<DBuf<int32_t>> bblk(1);  // inherited blocks of levels >= 1
        auto blk_of = [&](int32_t l) -> const int32_t* { return l == 0 ? carry : bblk[l].get(); };
        t_coarsen = Clock::now();
        // host initial partitions (first cycle; later ones inherit theirs),
        // computed while coarsening goes on
        std::unique_ptr<HostIpPipeline> pipe;
        if (!carry && o.initial != 1) {
            auto r8 = [](size_t x) { return (x + 7) & ~static_cast<size_t>(7); };
            const size_t n0 = static_cast<size_t>(g0.n), S0 = static_cast<size_t>(g0.S);
            const size_t bytes = r8((n0 + G) * sizeof(int64_t)) + r8(S0 * sizeof(int32_t)) +
                                 2 * r8(n0 * sizeof(int32_t)) + 4 * 8 * (static_cast<size_t>(SCLAP_MAX_LEVELS) + 1);
            pipe.reset(new HostIpPipeline(bytes, k, T, kb, s));
        }

        // ---- coarsening
        std::vector<uint8_t> cont(G, 1);
        int32_t lev = 0;
        while (true) {
            const int32_t M = static_cast<int32_t>(L[lev].ids.size());
            std::vector<uint8_t> act(G, 0);
            bool any = false;
            for (int32_t m = 0; m < M; ++m) {
                const int32_t g = L[lev].ids[m];
                const int32_t nm = L[lev].nb[m + 1] - L[lev].nb[m];
                if (cont[g] && nm > o.coarsest && lev < o.max_levels) {
                    act[g] = 1;
                    any = true;
                }
            }
            if (!any) {  // every graph of this level ends here
                if (pipe) {
                    std::vector<int32_t> all(M);
                    for (int32_t m = 0; m < M; ++m) all[m] = m;
                    pipe->stage(lev, L[lev], all);
                }
                break;
            }
            BatchLevel& B = L[lev];
            const int32_t n = B.g.n;
            std::vector<int64_t> cvl(G), cm = cmax0;
            if (lev > 0) graph_node_stats(n, B.gid.get(), B.g.vw, G, cvl.data(), cm.data(), s);
            std::vector<int64_t> bound(G, 0);
            std::vector<int32_t> base(G, 0);
            for (int32_t m = 0; m < M; ++m) {
                const int32_t g = B.ids[m];
                bound[g] = std::max(cm[g], W[g]);
                base[g] = B.nb[m];
            }
            upload_vec(d_bound, bound, s);
            upload_vec(d_lbase, base, s);
            upload_vec(d_nbase, base, s);
            upload_vec(d_active, act, s);
            DBuf<int32_t> labels(n, s), wl(n, s);
            iota_u32(reinterpret_cast<uint32_t*>(labels.get()), n, s);
            label_weights(B.g, labels.get(), wl.get(), n, s);
            MultiGraph mg;
            mg.G = G;
            mg.gid = B.gid.get();
            mg.lgid = B.gid.get();  // cluster labels are node ids
            mg.nbase = d_nbase.get();
            mg.lbase = d_lbase.get();
            mg.bound = d_bound.get();
            mg.seed = d_seed.get();
            mg.active = d_active.get();
            OwnedDevGraph inside;
            DevGraph Gc = B.g;  // the graph clustering looks at
            if (carry) {
                within_blocks(B.g, blk_of(lev), inside, s);
                Gc = inside.view();
                Gc.vw = B.g.vw;
            }
            DBuf<int32_t> dcol;
            if (o.degree_order) {
                std::vector<int32_t> gcnt(G, 0);
                for (int32_t m = 0; m < M; ++m) gcnt[B.ids[m]] = B.nb[m + 1] - B.nb[m];
                DBuf<int32_t> d_gcnt(G, s);
                upload_vec(d_gcnt, gcnt, s);
                dcol.alloc(n, s);
                degree_colors(Gc, G, B.gid.get(), d_nbase.get(), d_gcnt.get(), o.nsub, dcol.get(), s);
                HIPCHK(hipStreamSynchronize(s));  // gcnt is read by the upload above
            }
            auto t_lp = Clock::now();
            const LPResult r = run_lp(Gc, kCluster, lev, 0, o.nsub, o.coarsen_rounds, 0, labels.get(), wl.get(), n,
                                      dcol.get(), o.tune, s, &mg);
            lp_ms += ms_since(t_lp);
            inside = OwnedDevGraph();
            st->visits += r.visits;
            wl.release();
            // contraction of the whole level; member m's coarse nodes start at cb[m]
            DBuf<int32_t> probe(M + 1, s), qb(M + 1, s), C(n, s);
            upload_vec(probe, B.nb, s);
            OwnedDevGraph coarse;
            contract(B.g, labels.get(), C.get(), coarse, s, probe.get(), M + 1, qb.get(), false, o.bucket_mean);
            std::vector<int32_t> cb(M + 1);
            HIPCHK(hipMemcpyAsync(cb.data(), qb.get(), (M + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            labels.release();
            std::vector<int32_t> keep;
            for (int32_t m = 0; m < M; ++m) {
                const int32_t g = B.ids[m];
                if (!act[g]) {
                    cont[g] = 0;
                    continue;
                }
                const int64_t nm = B.nb[m + 1] - B.nb[m], nc = cb[m + 1] - cb[m];
                if (nc >= nm) {  // no shrink: this level stays the graph's coarsest
                    cont[g] = 0;
                    continue;
                }
                keep.push_back(m);
                if (20 * nc > 19 * nm) cont[g] = 0;  // stalled
            }
            if (pipe) {  // the graphs not kept end at this level
                std::vector<int32_t> ending;
                size_t q = 0;
                for (int32_t m = 0; m < M; ++m) {
                    if (q < keep.size() && keep[q] == m) {
                        ++q;
                        continue;
                    }
                    ending.push_back(m);
                }
                pipe->stage(lev, B, ending);
            }
            if (keep.empty()) break;
            BatchLevel N;
            const std::vector<int64_t> csb = member_slot_bases(coarse.xadj.get(), cb, s);
            N.nb.push_back(0);
            N.sb.push_back(0);
            std::vector<int32_t> onb;
            std::vector<int64_t> osb;
            for (int32_t m : keep) {
                N.ids.push_back(B.ids[m]);
                N.nb.push_back(N.nb.back() + (cb[m + 1] - cb[m]));
                N.sb.push_back(N.sb.back() + (csb[m + 1] - csb[m]));
                onb.push_back(cb[m]);
                osb.push_back(csb[m]);
            }
            if (static_cast<int32_t>(keep.size()) == M) {
                N.own = std::move(coarse);
            } else {
                compact_members(coarse.view(), onb, osb, N.nb, N.sb, N.own, s);
                coarse = OwnedDevGraph();
            }
            N.g = N.own.view();
            N.gid.alloc(std::max(N.g.n, 1), s);
            member_ids(N.g.n, N.nb, N.ids, N.gid.get(), s);
            std::vector<int32_t> delta(G, INT_MIN);
            for (size_t j = 0; j < keep.size(); ++j) delta[N.ids[j]] = N.nb[j] - cb[keep[j]];
            remap_members(n, B.gid.get(), delta, C.get(), s);
            DBuf<int32_t> cbl;
            if (carry) {
                cbl.alloc(std::max(N.g.n, 1), s);
                inherit_blocks(n, C.get(), blk_of(lev), cbl.get(), s);
            }
            B.C = std::move(C);
            L.push_back(std::move(N));  // B is not used after this
            bblk.push_back(std::move(cbl));
            ++lev;
        }
        const int32_t top = lev;
        std::vector<int32_t> last(G, 0);
        for (int32_t l = 0; l <= top; ++l)
            for (size_t m = 0; m < L[l].ids.size(); ++m) last[L[l].ids[m]] = l;
        st->levels = top;
        if (st->graph_levels)
            for (int32_t g = 0; g < G; ++g) st->graph_levels[g] = last[g];
        HIPCHK(hipStreamSynchronize(s));
        st->ms_coarsen += ms_since(t_coarsen);
        if (trace_on() && pipe) fprintf(stderr, "[sclap] batch coarsening done at %.1f ms\n", ms_since(t_coarsen));

        // ---- initial partitions: on the host (staged during coarsening
        // above), or on the device level by level in the refinement loop
        const bool dev_ip = o.initial == 1 && !carry;
        std::vector<uint8_t> ends_dev(static_cast<size_t>(top) + 1, 0);
        if (dev_ip)
            for (int32_t g = 0; g < G; ++g) ends_dev[last[g]] = 1;
        std::vector<double> ms_wait(static_cast<size_t>(top) + 1, 0.0);

        // ---- refinement from the top level down
        auto t_ref = Clock::now();
        upload_vec(d_bound, Lmax, s);
        upload_vec(d_active, std::vector<uint8_t>(G, 1), s);
        DBuf<int32_t> cur;
        double ip_ms = 0;
        for (int32_t l = top; l >= 0; --l) {
            BatchLevel& B = L[l];
            const int32_t n = B.g.n;
            DBuf<int32_t> mine;
            int32_t* part = part_out;
            if (l > 0) {
                mine.alloc(std::max(n, 1), s);
                part = mine.get();
            }
            if (carry && part != blk_of(l) && n > 0)  // graphs ending here keep their inherited blocks
                HIPCHK(hipMemcpyAsync(part, blk_of(l), n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            // graphs ending here: their initial partitions (the other ranges
            // are overwritten by the projection next)
            if (pipe) {
                ms_wait[l] = pipe->finish(l, part);
                ip_ms += ms_wait[l];
            }
            if (ends_dev[l] && n > 0) {
                std::vector<uint8_t> endg(G, 0);
                for (size_t m = 0; m < B.ids.size(); ++m)
                    if (last[B.ids[m]] == l) endg[B.ids[m]] = 1;
                auto t_ip = Clock::now();
                const LPResult ri = batch_device_initial(B.g, B.gid.get(), B.ids, B.nb, l, G, k, kb, T, cV, Lmax, endg,
                                                         cseed, d_seed.get(), d_bound.get(), o, part, s);
                st->visits += ri.visits;
                ip_ms += ms_since(t_ip);
            }
            if (l < top) project_kept(n, B.C.get(), cur.get(), part, s);
            std::vector<int32_t> base(G, 0);
            for (size_t m = 0; m < B.ids.size(); ++m) base[B.ids[m]] = B.nb[m];
            upload_vec(d_nbase, base, s);
            label_weights(B.g, part, w.get(), K, s);
            MultiGraph mg;
            mg.G = G;
            mg.gid = B.gid.get();
            mg.lgid = d_lgid.get();
            mg.max_labels = *std::max_element(k, k + G);
            mg.nbase = d_nbase.get();
            mg.lbase = d_kb.get();
            mg.bound = d_bound.get();
            mg.seed = d_seed.get();
            mg.active = d_active.get();
            auto t_lp = Clock::now();
            const LPResult r =
                run_lp(B.g, kRefine, l, 0, o.nsub, o.refine_rounds, 0, part, w.get(), K, nullptr, o.tune, s, &mg);
            lp_ms += ms_since(t_lp);
            st->visits += r.visits;
            HIPCHK(hipStreamSynchronize(s));  // the staging uploaded above must stay alive until here
            cur = std::move(mine);
            if (l < top) {
                L[l + 1] = BatchLevel();
                bblk[l + 1].release();
            }
            B.C.release();
        }
        HIPCHK(hipStreamSynchronize(s));
        st->ms_refine += ms_since(t_ref) - ip_ms;
        st->ms_initial += ip_ms;
        if (trace_on()) {
            fprintf(stderr, "[sclap] batch initial partitions: ms waited per level:");
            for (int32_t l = top; l >= 0; --l) fprintf(stderr, " L%d %.1f", l, ms_wait[l]);
            fprintf(stderr, "\n");
        }
    }  // cycles
    auto t_fin = Clock::now();
    std::vector<int32_t> hw_(std::max(K, 1));
    HIPCHK(hipMemcpyAsync(hw_.data(), w.get(), std::max(K, 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    graph_cuts(g0, part_out, L[0].gid.get(), G, cut, s);  // synchronises
    shift_by_graph(g0.n, L[0].gid.get(), d_kb.get(), -1, part_out, s);
    HIPCHK(hipStreamSynchronize(s));
    int status = SCLAP_OK;
    for (int32_t g = 0; g < G; ++g)
        for (int32_t b = kb[g]; b < kb[g + 1]; ++b) {
            bw[b] = hw_[b];
            if (bw[b] > Lmax[g]) status = SCLAP_WARN_IMBALANCED;
        }
    st->ms_refine += ms_since(t_fin);
    st->ms_lp = lp_ms;
    return status;
}

}  // namespace sclap
