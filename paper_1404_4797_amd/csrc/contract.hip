// Cluster contraction on gfx950 (Section 3.1 contraction definition; Section
// 4.3 relabelling and quotient graph).
//
// Coarse ids are the ranks of the used labels (mark + exclusive scan).  The
// quotient graph is built row by row instead of by one global sort:
//   1. count, per fine node u, the slots u->v with C(u) != C(v), and add the
//      counts up per coarse row (one atomic per node: in the multilevel path
//      a cluster has at most U members, however many slots its rows hold);
//   2. scan the row counts into row offsets, give every node a block of its
//      row and scatter (C(v), w) of every such slot into its node's block
//      (each wave's run of a row reserves its part with one atomic);
//   3. sort each row by C(v) and merge equal neighbours, summing weights:
//      rows of up to 64 entries in the registers of one wave (bitonic network
//      over lanes), up to 4096 in the LDS of one workgroup, longer rows by a
//      radix sort of (row, C(v)) keys over just those rows;
//   4. scan the merged row lengths into the coarse offsets and copy.
// The result is canonical (rows ascend by neighbour id) whatever order the
// atomics of step 2 produced.
#include <climits>

#include "graph_ops.hpp"
#include "profile.hpp"
#include "tiles.hpp"

namespace sclap {

namespace {

constexpr int kWaveRow = 64;     // rows up to this length: one wave
constexpr int kBlockRow = 4096;  // up to this length: one workgroup, LDS sort

__global__ void mark_used_kernel(int32_t n, const int32_t* __restrict__ labels, int32_t* __restrict__ used) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) used[labels[v]] = 1;
}

__global__ void map_kernel(int32_t n, const int32_t* __restrict__ labels, const int32_t* __restrict__ q,
                           const int32_t* __restrict__ vw, int32_t* __restrict__ C, int32_t* __restrict__ cvw) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t cv = q[labels[v]];
    C[v] = cv;
    const int32_t c = vw ? vw[v] : 1;
    if (c) atomicAdd(&cvw[cv], c);
}

// probe_out[i] = number of used labels below probe[i] (probe[i] in [0, n]).
__global__ void probe_kernel(const int32_t* __restrict__ probe, int32_t nprobe, const int32_t* __restrict__ q,
                             int32_t n, const int32_t* __restrict__ total, int32_t* __restrict__ out) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < nprobe) out[i] = probe[i] < n ? q[probe[i]] : *total;
}

__device__ __forceinline__ int32_t block_sum_i32_256(int32_t v) {
    __shared__ int32_t sred[4];
    v = wave_sum(v);
    if (lane_id() == 0) sred[threadIdx.x >> 6] = v;
    __syncthreads();
    const int32_t t = sred[0] + sred[1] + sred[2] + sred[3];
    __syncthreads();
    return t;
}

// Runs of equal keys over consecutive lanes: lead = first lane of this lane's
// run, end = one past its last lane.
__device__ __forceinline__ void wave_runs(int32_t key, int& lead, int& end) {
    const int lane = lane_id();
    const int32_t prev = __shfl_up(key, 1, 64);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const uint64_t upto = (2ULL << lane) - 1;  // lanes 0..lane (all lanes for lane 63)
    lead = 63 - __clzll(static_cast<long long>(heads & upto));
    const uint64_t after = heads & ~upto;
    end = after ? __ffsll(static_cast<long long>(after)) - 1 : 64;
}

// Step 1: inter-cluster slots per fine node, cross[u] (one atomic per wave and
// row run: rows are contiguous in slot order); keeps C(v) of every slot for
// step 2, which then reads it in slot order instead of gathering it again.
__global__ void __launch_bounds__(kTileThreads) cross_count_kernel(const int64_t* __restrict__ xadj,
                                                                   const int32_t* __restrict__ adj, int32_t n,
                                                                   int64_t S, const int32_t* __restrict__ C,
                                                                   int32_t* __restrict__ cross,
                                                                   int32_t* __restrict__ cvs, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
    tile_owners(xadj, trow, static_cast<int64_t>(blockIdx.x), i0, i1, owner);
    const int lane = lane_id();
    for (int r = 0; r < kTilePer; ++r) {
        const int64_t i = i0 + r * kTileThreads + threadIdx.x;
        int32_t u = -1;
        bool e = false;
        if (i < i1) {
            u = owner[i - i0];
            const int32_t cv = C[adj[i]];
            cvs[i] = cv;
            e = C[u] != cv;
        }
        int lead, end;
        wave_runs(u, lead, end);
        const uint64_t em = __ballot(e);
        const uint64_t run = ((end == 64 ? 0ULL : (1ULL << end)) - 1) & ~((1ULL << lead) - 1);
        const int cnt = __popcll(em & run);
        if (lane == lead && u >= 0 && cnt) atomicAdd(&cross[u], cnt);
    }
}

// Per fine node: its coarse row grows by cross[u] ...
__global__ void row_count_kernel(int32_t n, const int32_t* __restrict__ C, const int32_t* __restrict__ cross,
                                 int32_t* __restrict__ rowcnt) {
    const int32_t u = blockIdx.x * 256 + threadIdx.x;
    if (u < n && cross[u]) atomicAdd(&rowcnt[C[u]], cross[u]);
}

// ... and, once rows are placed, each node reserves its block of the row.
__global__ void node_base_kernel(int32_t n, const int32_t* __restrict__ C, const int32_t* __restrict__ cross,
                                 const int64_t* __restrict__ rowoff, int32_t* __restrict__ fill,
                                 int64_t* __restrict__ nbase) {
    const int32_t u = blockIdx.x * 256 + threadIdx.x;
    if (u < n && cross[u]) nbase[u] = rowoff[C[u]] + atomicAdd(&fill[C[u]], cross[u]);
}

// Step 2: (C(v), w) of every inter-cluster slot into its node's block of the
// coarse row; each wave run of a row reserves its part of the block.
__global__ void __launch_bounds__(kTileThreads) row_scatter_kernel(const int64_t* __restrict__ xadj,
                                                                   const int32_t* __restrict__ cvs,
                                                                   const int32_t* __restrict__ ew, int32_t n, int64_t S,
                                                                   const int32_t* __restrict__ C,
                                                                   const int64_t* __restrict__ nbase,
                                                                   int32_t* __restrict__ nfill,
                                                                   int32_t* __restrict__ tk, int32_t* __restrict__ tw, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
    tile_owners(xadj, trow, static_cast<int64_t>(blockIdx.x), i0, i1, owner);
    const int lane = lane_id();
    for (int r = 0; r < kTilePer; ++r) {
        const int64_t i = i0 + r * kTileThreads + threadIdx.x;
        int32_t u = -1, cv = 0;
        bool e = false;
        if (i < i1) {
            u = owner[i - i0];
            cv = cvs[i];
            e = C[u] != cv;
        }
        int lead, end;
        wave_runs(u, lead, end);
        const uint64_t em = __ballot(e);
        const uint64_t run = ((end == 64 ? 0ULL : (1ULL << end)) - 1) & ~((1ULL << lead) - 1);
        const int cnt = __popcll(em & run);
        int32_t base = 0;
        if (lane == lead && u >= 0 && cnt) base = atomicAdd(&nfill[u], cnt);
        base = __shfl(base, lead, 64);
        if (e) {
            const int64_t at = nbase[u] + base + __popcll(em & run & ((1ULL << lane) - 1));
            tk[at] = cv;
            tw[at] = ew ? ew[i] : 1;
        }
    }
}

// Rows by length: 0 or 1 entries are final as they are; the others go to the
// wave, workgroup or long-row lists.
// (each workgroup takes kClassifyIters * 256 consecutive rows at a time and
// appends to each list with one atomic: the three counters are few and hot)
constexpr int kClassifyIters = 16;

__global__ void __launch_bounds__(256) row_classify_kernel(int32_t nc, const int32_t* __restrict__ rowcnt,
                                                           int32_t* __restrict__ dcnt, int32_t* __restrict__ lists,
                                                           int32_t cap, uint32_t* __restrict__ counts) {
    for (int32_t base = blockIdx.x * (kClassifyIters * 256); base < nc; base += gridDim.x * (kClassifyIters * 256)) {
        uint32_t m[3] = {0, 0, 0};
        int32_t lens[kClassifyIters];
#pragma unroll
        for (int it = 0; it < kClassifyIters; ++it) {
            const int32_t r = base + it * 256 + static_cast<int32_t>(threadIdx.x);
            lens[it] = r < nc ? rowcnt[r] : -1;
        }
#pragma unroll
        for (int it = 0; it < kClassifyIters; ++it) {
            const int32_t r = base + it * 256 + static_cast<int32_t>(threadIdx.x);
            const int32_t len = lens[it];
            if (len < 0) continue;
            if (len <= 1) {
                dcnt[r] = len;
                continue;
            }
            m[len <= kWaveRow ? 0 : (len <= kBlockRow ? 1 : 2)] |= 1u << it;
        }
        for (int c = 0; c < 3; ++c) {
            uint32_t bits = m[c];
            uint32_t j = block_append_count(static_cast<uint32_t>(__popc(bits)), &counts[c]);
            while (bits) {
                const int it = __ffs(bits) - 1;
                bits &= bits - 1;
                lists[static_cast<int64_t>(c) * cap + j++] = base + it * 256 + static_cast<int32_t>(threadIdx.x);
            }
        }
    }
}

// Rows of 2..64 entries: one wave per row sorts (C(v), w) over its lanes with a
// bitonic network and writes the merged row to the row's start.
__global__ void __launch_bounds__(256) wave_rows_kernel(const int32_t* __restrict__ list, uint32_t count,
                                                        const int64_t* __restrict__ rowoff,
                                                        const int32_t* __restrict__ rowcnt, int32_t* __restrict__ tk,
                                                        int32_t* __restrict__ tw, int32_t* __restrict__ dcnt) {
    const uint32_t wv = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (wv >= count) return;  // uniform per wave
    const int lane = lane_id();
    const int32_t row = list[wv];
    const int64_t b = rowoff[row];
    const int32_t len = rowcnt[row];
    uint32_t key = lane < len ? static_cast<uint32_t>(tk[b + lane]) : 0xFFFFFFFFu;
    int32_t w = lane < len ? tw[b + lane] : 0;
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t ok = __shfl_xor(key, j, 64);
            const int32_t ow = __shfl_xor(w, j, 64);
            const bool up = (lane & k) == 0;
            const bool low = (lane & j) == 0;
            const bool take = low == up ? ok < key : ok > key;
            if (take) {
                key = ok;
                w = ow;
            }
        }
    }
    // merge equal neighbours: inclusive sums over the lanes, then per run
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool valid = lane < len;
    const bool head = valid && (lane == 0 || prev != key);
    int64_t incl = w;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const uint64_t heads = __ballot(head);
    const uint64_t upto = (2ULL << lane) - 1;
    const uint64_t after = heads & ~upto;
    const int last = (after ? __ffsll(static_cast<long long>(after)) - 1 : len) - 1;  // last lane of this run
    const int64_t at_last = __shfl(incl, last < 0 ? 0 : last, 64);
    if (head) {
        const int pos = __popcll(heads & (upto >> 1));
        tk[b + pos] = static_cast<int32_t>(key);
        tw[b + pos] = static_cast<int32_t>(at_last - incl + w);
    }
    if (lane == 0) dcnt[row] = __popcll(heads);
}

// Rows of 65..4096 entries: one workgroup per row, bitonic sort of
// (C(v) << 32 | w) in LDS, then the merged row to the row's start.
__global__ void __launch_bounds__(256) block_rows_kernel(const int32_t* __restrict__ list,
                                                         const int64_t* __restrict__ rowoff,
                                                         const int32_t* __restrict__ rowcnt, int32_t* __restrict__ tk,
                                                         int32_t* __restrict__ tw, int32_t* __restrict__ dcnt) {
    __shared__ uint64_t sk[kBlockRow];
    __shared__ int32_t s_cnt[256];
    const int tid = threadIdx.x;
    const int32_t row = list[blockIdx.x];
    const int64_t b = rowoff[row];
    const int32_t len = rowcnt[row];
    int32_t P = 128;
    while (P < len) P <<= 1;
    for (int32_t j = tid; j < P; j += 256)
        sk[j] = j < len ? (static_cast<uint64_t>(static_cast<uint32_t>(tk[b + j])) << 32) |
                              static_cast<uint32_t>(tw[b + j])
                        : ~0ULL;
    for (int32_t k = 2; k <= P; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int32_t i = tid; i < P; i += 256) {
                const int32_t p = i ^ j;
                if (p > i) {
                    const uint64_t x = sk[i], y = sk[p];
                    if ((x > y) == ((i & k) == 0)) {
                        sk[i] = y;
                        sk[p] = x;
                    }
                }
            }
        }
    }
    __syncthreads();
    // each thread owns a contiguous segment of the sorted row
    const int32_t per = (len + 255) / 256;
    const int32_t s0 = tid * per < len ? tid * per : len;
    const int32_t s1 = s0 + per < len ? s0 + per : len;
    int32_t mine = 0;
    for (int32_t i = s0; i < s1; ++i)
        if (i == 0 || (sk[i] >> 32) != (sk[i - 1] >> 32)) ++mine;
    s_cnt[tid] = mine;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const int32_t c = s_cnt[t];
            s_cnt[t] = run;
            run += c;
        }
        dcnt[row] = run;
    }
    __syncthreads();
    int32_t pos = s_cnt[tid];
    for (int32_t i = s0; i < s1; ++i) {
        const uint64_t key = sk[i] >> 32;
        if (i != 0 && key == (sk[i - 1] >> 32)) continue;
        int64_t sum = 0;
        for (int32_t j = i; j < len && (sk[j] >> 32) == key; ++j) sum += static_cast<int32_t>(sk[j] & 0xFFFFFFFFu);
        tk[b + pos] = static_cast<int32_t>(key);
        tw[b + pos] = static_cast<int32_t>(sum);
        ++pos;
    }
}

// Rows longer than 4096 entries: keys (long-row index << bn | C(v)) over just
// those rows, radix sorted, then merged per row.
__global__ void long_lens_kernel(const int32_t* __restrict__ list, uint32_t nl, const int32_t* __restrict__ rowcnt,
                                 int32_t* __restrict__ nchunks, int32_t chunk) {
    const uint32_t l = blockIdx.x * 256 + threadIdx.x;
    if (l < nl) nchunks[l] = (rowcnt[list[l]] + chunk - 1) / chunk;
}

constexpr int kLongChunk = 8192;  // entries merged in LDS per workgroup before the sort
constexpr int kDedupThreads = 1024;

// Long-row chunks: chunk c of all long rows belongs to row list[crow[c]] and
// is that row's chunk number c - cfirst[crow[c]].
__global__ void long_chunks_kernel(uint32_t nl, const int64_t* __restrict__ cfirst, int32_t* __restrict__ crow) {
    const uint32_t l = blockIdx.x;
    if (l >= nl) return;
    for (int64_t c = cfirst[l] + threadIdx.x; c < cfirst[l + 1]; c += 256) crow[c] = static_cast<int32_t>(l);
}

// Merges equal neighbours inside one chunk in an LDS table and writes the
// chunk's distinct (C(v), summed w) back to the chunk's start.  Sums fit 32
// bits: a partial sum never exceeds the coarse edge's weight, and the edge
// weight total is checked to fit 31 bits.  Long rows of contracted hubs
// repeat their neighbours many times, so large chunks shrink what the
// bucket passes after this one move.
__global__ void __launch_bounds__(kDedupThreads) long_dedup_kernel(const int32_t* __restrict__ list,
                                                                   const int32_t* __restrict__ crow,
                                                                   const int64_t* __restrict__ cfirst,
                                                                   const int64_t* __restrict__ rowoff,
                                                                   const int32_t* __restrict__ rowcnt,
                                                                   int32_t* __restrict__ tk, int32_t* __restrict__ tw,
                                                                   int32_t* __restrict__ ccnt) {
    constexpr int kT = 2 * kLongChunk;
    constexpr int kW = kDedupThreads / kWave;
    __shared__ int32_t keys[kT];
    __shared__ uint32_t sums[kT];
    __shared__ int32_t s_w[kW];
    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t l = crow[c];
    const int32_t row = list[l];
    const int64_t j0 = (c - cfirst[l]) * kLongChunk;
    const int64_t len = rowcnt[row];
    const int32_t cnt = static_cast<int32_t>(j0 + kLongChunk < len ? kLongChunk : len - j0);
    const int64_t b = rowoff[row] + j0;
    for (int j = tid; j < kT; j += kDedupThreads) {
        keys[j] = -1;
        sums[j] = 0;
    }
    __syncthreads();
    for (int j = tid; j < cnt; j += kDedupThreads) {
        const int32_t x = tk[b + j];
        uint32_t h = slot_hash(static_cast<uint32_t>(x)) & (kT - 1);
        while (true) {
            const int32_t prev = atomicCAS(&keys[h], -1, x);
            if (prev == -1 || prev == x) break;
            h = (h + 1) & (kT - 1);
        }
        atomicAdd(&sums[h], static_cast<uint32_t>(tw[b + j]));
    }
    __syncthreads();
    // exclusive prefix of the occupied slots, kPer consecutive slots per thread
    constexpr int kPer = kT / kDedupThreads;
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) mine += keys[tid * kPer + j] >= 0;
    int32_t incl = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= o) incl += t;
    }
    if (lane_id() == kWave - 1) s_w[tid / kWave] = incl;
    __syncthreads();
    int32_t pos = incl - mine;
    for (int w = 0; w < tid / kWave; ++w) pos += s_w[w];
    if (tid == kDedupThreads - 1) ccnt[c] = pos + mine;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int e = tid * kPer + j;
        if (keys[e] < 0) continue;
        tk[b + pos] = keys[e];
        tw[b + pos] = static_cast<int32_t>(sums[e]);
        ++pos;
    }
}

// Sort keys (long-row index << bn | C(v)) over the merged chunk entries, one
// chunk per workgroup.
__global__ void __launch_bounds__(256) long_keys_kernel(const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ crow,
                                                        const int64_t* __restrict__ cfirst,
                                                        const int32_t* __restrict__ ccnt,
                                                        const int64_t* __restrict__ coff,
                                                        const int64_t* __restrict__ rowoff,
                                                        const int32_t* __restrict__ tk, const int32_t* __restrict__ tw,
                                                        int bn, uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
    const int64_t c = blockIdx.x;
    const int32_t l = crow[c];
    const int64_t src = rowoff[list[l]] + (c - cfirst[l]) * kLongChunk;
    const int64_t dst = coff[c];
    for (int32_t j = threadIdx.x; j < ccnt[c]; j += 256) {
        keys[dst + j] = (static_cast<uint64_t>(l) << bn) | static_cast<uint32_t>(tk[src + j]);
        vals[dst + j] = static_cast<uint32_t>(tw[src + j]);
    }
}

// loff[l] = coff[cfirst[l]]: first sort key of long row l
__global__ void long_offsets_kernel(uint32_t nl, const int64_t* __restrict__ cfirst, const int64_t* __restrict__ coff,
                                    int64_t* __restrict__ loff) {
    const uint32_t l = blockIdx.x * 256 + threadIdx.x;
    if (l <= nl) loff[l] = coff[cfirst[l]];
}

// heads of equal-key runs, and the weights as int64 for the prefix sums
__global__ void long_heads_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t m,
                                  int32_t* __restrict__ head, int64_t* __restrict__ psum) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < m) {
        head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
        psum[i] = static_cast<int32_t>(vals[i]);
    }
}

// Heads write the neighbour at the row-local distinct index and remember
// where the run starts; the last entry of a run writes its summed weight.
// pos: exclusive scan of head; psum: inclusive scan of the weights.
__global__ void long_runs_kernel(const int32_t* __restrict__ list, const int64_t* __restrict__ loff,
                                 const int64_t* __restrict__ rowoff, const uint64_t* __restrict__ keys, int64_t m,
                                 const int32_t* __restrict__ head, const int64_t* __restrict__ pos, int bn,
                                 int64_t* __restrict__ run_start, int32_t* __restrict__ tk,
                                 int32_t* __restrict__ dcnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m) return;
    const uint64_t key = keys[i];
    const uint32_t l = static_cast<uint32_t>(key >> bn);
    const int32_t row = list[l];
    const int64_t first = pos[loff[l]];  // distinct index of the row's first run
    const int64_t d = pos[i] + head[i] - 1;
    if (head[i]) {
        run_start[d] = i;
        tk[rowoff[row] + (d - first)] = static_cast<int32_t>(key & ((1ULL << bn) - 1));
    }
    if (i + 1 == loff[l + 1]) dcnt[row] = static_cast<int32_t>(d + 1 - first);
}

__global__ void long_tails_kernel(const int32_t* __restrict__ list, const int64_t* __restrict__ loff,
                                  const int64_t* __restrict__ rowoff, const uint64_t* __restrict__ keys, int64_t m,
                                  const int32_t* __restrict__ head, const int64_t* __restrict__ pos,
                                  const int64_t* __restrict__ psum, int bn, const int64_t* __restrict__ run_start,
                                  int32_t* __restrict__ tw) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m) return;
    const uint64_t key = keys[i];
    if (i + 1 < m && keys[i + 1] == key) return;  // not the last entry of its run
    const uint32_t l = static_cast<uint32_t>(key >> bn);
    const int32_t row = list[l];
    const int64_t first = pos[loff[l]];
    const int64_t d = pos[i] + head[i] - 1;
    const int64_t st = run_start[d];
    tw[rowoff[row] + (d - first)] = static_cast<int32_t>(psum[i] - (st > 0 ? psum[st - 1] : 0));
}

// Unsorted merge of rows of 65..4096 entries: one workgroup per row sums
// equal neighbours in an LDS table of kT >= 2 len slots and writes the
// distinct entries (in table order) to the row's start.  Rows are grouped by
// length so that short rows get small tables (less to clear, more workgroups
// per CU).
template <int kT>
__global__ void __launch_bounds__(256) block_hash_rows_kernel(const int32_t* __restrict__ list,
                                                              const int64_t* __restrict__ rowoff,
                                                              const int32_t* __restrict__ rowcnt,
                                                              int32_t* __restrict__ tk, int32_t* __restrict__ tw,
                                                              int32_t* __restrict__ dcnt) {
    __shared__ int32_t keys[kT];
    __shared__ int32_t sums[kT];
    __shared__ int32_t s_w[4];
    const int tid = threadIdx.x;
    const int32_t row = list[blockIdx.x];
    const int64_t b = rowoff[row];
    const int32_t len = rowcnt[row];
    for (int j = tid; j < kT; j += 256) {
        keys[j] = -1;
        sums[j] = 0;
    }
    __syncthreads();
    for (int j = tid; j < len; j += 256) {
        const int32_t x = tk[b + j];
        uint32_t h = slot_hash(static_cast<uint32_t>(x)) & (kT - 1);
        while (true) {
            const int32_t prev = atomicCAS(&keys[h], -1, x);
            if (prev == -1 || prev == x) break;
            h = (h + 1) & (kT - 1);
        }
        atomicAdd(&sums[h], tw[b + j]);  // partial sums never exceed the final coarse weight
    }
    __syncthreads();
    // exclusive prefix of the occupied slots, kPer consecutive slots per thread
    constexpr int kPer = kT / 256;
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) mine += keys[tid * kPer + j] >= 0;
    int32_t incl = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= o) incl += t;
    }
    if (lane_id() == kWave - 1) s_w[tid / kWave] = incl;
    __syncthreads();
    int32_t pos = incl - mine;
    for (int w = 0; w < tid / kWave; ++w) pos += s_w[w];
    if (tid == 255) dcnt[row] = pos + mine;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int e = tid * kPer + j;
        if (keys[e] < 0) continue;
        tk[b + pos] = keys[e];
        tw[b + pos] = sums[e];
        ++pos;
    }
}

// Splits the workgroup-row list by length: class c holds rows of at most
// 256 << c entries (c = 0..4).  Each workgroup takes kClassifyIters * 256
// list entries at a time and appends to each class with one atomic.
__global__ void __launch_bounds__(256) block_row_split_kernel(const int32_t* __restrict__ list, uint32_t count,
                                                              const int32_t* __restrict__ rowcnt,
                                                              int32_t* __restrict__ out, uint32_t cap,
                                                              uint32_t* __restrict__ counts) {
    for (uint32_t base = blockIdx.x * (kClassifyIters * 256); base < count;
         base += gridDim.x * (kClassifyIters * 256)) {
        int32_t rows[kClassifyIters], lens[kClassifyIters];
#pragma unroll
        for (int it = 0; it < kClassifyIters; ++it) {
            const uint32_t i = base + it * 256 + threadIdx.x;
            rows[it] = i < count ? list[i] : -1;
        }
#pragma unroll
        for (int it = 0; it < kClassifyIters; ++it) lens[it] = rows[it] >= 0 ? rowcnt[rows[it]] : 0;
        uint32_t m[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int it = 0; it < kClassifyIters; ++it) {
            if (rows[it] < 0) continue;
            int cls = 0;
            while (cls < 4 && lens[it] > (256 << cls)) ++cls;
            m[cls] |= 1u << it;
        }
        for (int c = 0; c < 5; ++c) {
            uint32_t bits = m[c];
            uint32_t j = block_append_count(static_cast<uint32_t>(__popc(bits)), &counts[c]);
            while (bits) {
                const int it = __ffs(bits) - 1;
                bits &= bits - 1;
                out[static_cast<int64_t>(c) * cap + j++] = rows[it];
            }
        }
    }
}

// Unsorted merge of long rows after the chunk merge, by buckets: the merged
// chunk entries of long row l are spread over P_l = ceil(m_l / kBucketMean)
// buckets by a hash of the neighbour id (so equal ids meet in one bucket),
// scattered bucket by bucket into a staging array, merged per bucket in an
// LDS table by one workgroup, and copied back into the row.  Every step
// streams the entries once; nothing probes a table in HBM.  A bucket whose
// distinct neighbours do not fit its LDS table raises a flag, and the caller
// then merges the long rows through per-row HBM tables instead.
constexpr int kBucketMean = 1024;   // merged entries per bucket on average (default)
constexpr int kBucketTable = 4096;  // LDS table slots of one bucket merge
constexpr int kBucketLds = 4096;    // rows with up to this many buckets count and reserve in LDS

__device__ __forceinline__ uint32_t bucket_of(int32_t x, uint32_t P) {
    const uint32_t h = slot_hash(static_cast<uint32_t>(x) ^ 0x5BD1E995u);  // independent of the table slot
    return static_cast<uint32_t>((static_cast<uint64_t>(h) * P) >> 32);
}

__global__ void long_bucket_counts_kernel(uint32_t nl, const int64_t* __restrict__ loff, int32_t mean,
                                          const int32_t* __restrict__ list, const int64_t* __restrict__ cfirst,
                                          int32_t* __restrict__ dcnt, int32_t* __restrict__ nbk) {
    const uint32_t l = blockIdx.x * 256 + threadIdx.x;
    if (l >= nl) return;
    const int64_t m = loff[l + 1] - loff[l];
    if (cfirst[l + 1] - cfirst[l] == 1) {  // one chunk: its merge is the row's
        nbk[l] = 0;
        dcnt[list[l]] = static_cast<int32_t>(m);
        return;
    }
    // at most kBucketLds buckets: a row's buckets then count and reserve in
    // LDS; a bucket whose distinct neighbours overflow its table sends the
    // long rows to the HBM-table merge
    const int64_t q = m > mean ? (m + mean - 1) / mean : 1;
    nbk[l] = static_cast<int32_t>(q < kBucketLds ? q : kBucketLds);
}

// bucket q belongs to long row brow[q]
__global__ void long_bucket_rows_kernel(uint32_t nl, const int64_t* __restrict__ bfirst, int32_t* __restrict__ brow) {
    const uint32_t l = blockIdx.x;
    if (l >= nl) return;
    for (int64_t q = bfirst[l] + threadIdx.x; q < bfirst[l + 1]; q += 256) brow[q] = static_cast<int32_t>(l);
}

// Pass 1 (reserve = false): bucket sizes.  Pass 2 (reserve = true): every
// entry to its bucket's range of the staging arrays; each workgroup reserves
// its part of a bucket with one atomic per bucket it touches.
template <bool kReserve>
__global__ void __launch_bounds__(256) long_bucket_scatter_kernel(
    const int32_t* __restrict__ list, const int32_t* __restrict__ crow, const int64_t* __restrict__ cfirst,
    const int32_t* __restrict__ ccnt, const int64_t* __restrict__ rowoff, const int64_t* __restrict__ bfirst,
    const int32_t* __restrict__ tk, const int32_t* __restrict__ tw, int32_t* __restrict__ bcount,
    const int64_t* __restrict__ boff, int32_t* __restrict__ bfill, int32_t* __restrict__ sk,
    int32_t* __restrict__ sw) {
    __shared__ int32_t lcnt[kBucketLds];
    __shared__ int32_t lbase[kBucketLds];
    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t l = crow[c];
    const int64_t src = rowoff[list[l]] + (c - cfirst[l]) * kLongChunk;
    const int32_t cnt = ccnt[c];
    const int64_t b0 = bfirst[l];
    const uint32_t P = static_cast<uint32_t>(bfirst[l + 1] - b0);
    if (P == 0) return;  // a one-chunk row, merged already
    for (uint32_t j = tid; j < P; j += 256) lcnt[j] = 0;
    __syncthreads();
    for (int32_t j = tid; j < cnt; j += 256) atomicAdd(&lcnt[bucket_of(tk[src + j], P)], 1);
    __syncthreads();
    for (uint32_t j = tid; j < P; j += 256) {
        const int32_t k = lcnt[j];
        if (k == 0) continue;
        if (kReserve) {
            lbase[j] = atomicAdd(&bfill[b0 + j], k);
            lcnt[j] = 0;
        } else {
            atomicAdd(&bcount[b0 + j], k);
        }
    }
    if (!kReserve) return;
    __syncthreads();
    for (int32_t j = tid; j < cnt; j += 256) {
        const int32_t x = tk[src + j];
        const uint32_t q = bucket_of(x, P);
        const int64_t at = boff[b0 + q] + lbase[q] + atomicAdd(&lcnt[q], 1);
        sk[at] = x;
        sw[at] = tw[src + j];
    }
}

// One workgroup per bucket: equal neighbours summed in an LDS table, the
// distinct entries written back to the bucket's start, their number to qcnt.
__global__ void __launch_bounds__(256) long_bucket_merge_kernel(const int64_t* __restrict__ boff,
                                                                int32_t* __restrict__ sk, int32_t* __restrict__ sw,
                                                                int32_t* __restrict__ qcnt,
                                                                uint32_t* __restrict__ overflow) {
    __shared__ int32_t keys[kBucketTable];
    __shared__ int32_t sums[kBucketTable];
    __shared__ int32_t s_w[4];
    __shared__ int32_t s_full;
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x;
    const int64_t b = boff[q];
    const int32_t len = static_cast<int32_t>(boff[q + 1] - b);
    for (int j = tid; j < kBucketTable; j += 256) {
        keys[j] = -1;
        sums[j] = 0;
    }
    if (tid == 0) s_full = 0;
    __syncthreads();
    for (int j = tid; j < len; j += 256) {
        const int32_t x = sk[b + j];
        uint32_t h = slot_hash(static_cast<uint32_t>(x)) & (kBucketTable - 1);
        int probes = 0;
        while (true) {
            const int32_t prev = atomicCAS(&keys[h], -1, x);
            if (prev == -1 || prev == x) break;
            h = (h + 1) & (kBucketTable - 1);
            if (++probes == kBucketTable) break;  // table full
        }
        if (probes == kBucketTable) {
            s_full = 1;
            break;
        }
        atomicAdd(&sums[h], sw[b + j]);  // partial sums never exceed the final coarse weight
    }
    __syncthreads();
    if (s_full) {
        if (tid == 0) atomicOr(overflow, 1u);
        return;
    }
    // exclusive prefix of the occupied slots, kPer consecutive slots per thread
    constexpr int kPer = kBucketTable / 256;
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) mine += keys[tid * kPer + j] >= 0;
    int32_t incl = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= o) incl += t;
    }
    if (lane_id() == kWave - 1) s_w[tid / kWave] = incl;
    __syncthreads();
    int32_t pos = incl - mine;
    for (int w = 0; w < tid / kWave; ++w) pos += s_w[w];
    if (tid == 255) qcnt[q] = pos + mine;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int e = tid * kPer + j;
        if (keys[e] < 0) continue;
        sk[b + pos] = keys[e];
        sw[b + pos] = sums[e];
        ++pos;
    }
}

__global__ void __launch_bounds__(256) long_bucket_write_kernel(const int32_t* __restrict__ list,
                                                                const int32_t* __restrict__ brow,
                                                                const int64_t* __restrict__ bfirst,
                                                                const int64_t* __restrict__ boff,
                                                                const int64_t* __restrict__ qoff,
                                                                const int32_t* __restrict__ qcnt,
                                                                const int64_t* __restrict__ rowoff,
                                                                const int32_t* __restrict__ sk,
                                                                const int32_t* __restrict__ sw,
                                                                int32_t* __restrict__ tk, int32_t* __restrict__ tw,
                                                                int32_t* __restrict__ dcnt) {
    const int64_t q = blockIdx.x;
    const int32_t l = brow[q];
    const int32_t row = list[l];
    const int64_t q0 = bfirst[l];
    const int64_t dst = rowoff[row] + (qoff[q] - qoff[q0]);
    const int64_t src = boff[q];
    const int32_t cnt = qcnt[q];
    for (int32_t j = threadIdx.x; j < cnt; j += 256) {
        tk[dst + j] = sk[src + j];
        tw[dst + j] = sw[src + j];
    }
    if (q == q0 && threadIdx.x == 0) dcnt[row] = static_cast<int32_t>(qoff[bfirst[l + 1]] - qoff[q0]);
}

// Unsorted merge of long rows after the chunk merge: one open-addressing
// table in HBM per row (at least twice its merged entries, a power of two),
// filled with atomics, then compacted chunk by chunk.
constexpr int kTabChunk = 4096;

__global__ void long_table_sizes_kernel(uint32_t nl, const int64_t* __restrict__ loff, int64_t* __restrict__ tsz,
                                        int64_t* __restrict__ tch) {
    const uint32_t l = blockIdx.x * 256 + threadIdx.x;
    if (l >= nl) return;
    const int64_t want = 2 * (loff[l + 1] - loff[l]);
    int64_t t = kTabChunk;
    while (t < want) t <<= 1;
    tsz[l] = t;
    tch[l] = t / kTabChunk;
}

__global__ void __launch_bounds__(256) long_table_insert_kernel(const int32_t* __restrict__ list,
                                                                const int32_t* __restrict__ crow,
                                                                const int64_t* __restrict__ cfirst,
                                                                const int32_t* __restrict__ ccnt,
                                                                const int64_t* __restrict__ rowoff,
                                                                const int32_t* __restrict__ tk,
                                                                const int32_t* __restrict__ tw,
                                                                const int64_t* __restrict__ toff,
                                                                const int64_t* __restrict__ tsz,
                                                                int32_t* __restrict__ gk, int32_t* __restrict__ gv) {
    const int64_t c = blockIdx.x;  // one merged chunk per workgroup
    const int32_t l = crow[c];
    const int64_t src = rowoff[list[l]] + (c - cfirst[l]) * kLongChunk;
    int32_t* keys = gk + toff[l];
    int32_t* vals = gv + toff[l];
    const uint64_t mask = static_cast<uint64_t>(tsz[l]) - 1;
    for (int32_t j = threadIdx.x; j < ccnt[c]; j += 256) {
        const int32_t x = tk[src + j];
        uint64_t h = slot_hash(static_cast<uint32_t>(x)) & mask;
        while (true) {
            const int32_t prev = atomicCAS(&keys[h], -1, x);
            if (prev == -1 || prev == x) break;
            h = (h + 1) & mask;
        }
        atomicAdd(&vals[h], tw[src + j]);
    }
}

// table chunk q belongs to row tl[q]
__global__ void long_table_chunks_kernel(uint32_t nl, const int64_t* __restrict__ tcfirst, int32_t* __restrict__ tl) {
    const uint32_t l = blockIdx.x;
    if (l >= nl) return;
    for (int64_t q = tcfirst[l] + threadIdx.x; q < tcfirst[l + 1]; q += 256) tl[q] = static_cast<int32_t>(l);
}

__global__ void __launch_bounds__(256) long_table_count_kernel(const int32_t* __restrict__ tl,
                                                               const int64_t* __restrict__ tcfirst,
                                                               const int64_t* __restrict__ toff,
                                                               const int32_t* __restrict__ gk,
                                                               int32_t* __restrict__ qcnt) {
    const int64_t q = blockIdx.x;
    const int32_t l = tl[q];
    const int64_t base = toff[l] + (q - tcfirst[l]) * kTabChunk;
    int32_t c = 0;
    for (int j = threadIdx.x; j < kTabChunk; j += 256) c += gk[base + j] >= 0;
    c = block_sum_i32_256(c);
    if (threadIdx.x == 0) qcnt[q] = c;
}

__global__ void __launch_bounds__(256) long_table_write_kernel(const int32_t* __restrict__ list,
                                                               const int32_t* __restrict__ tl,
                                                               const int64_t* __restrict__ tcfirst,
                                                               const int64_t* __restrict__ toff,
                                                               const int64_t* __restrict__ qoff,
                                                               const int64_t* __restrict__ rowoff,
                                                               const int32_t* __restrict__ gk,
                                                               const int32_t* __restrict__ gv,
                                                               int32_t* __restrict__ tk, int32_t* __restrict__ tw,
                                                               int32_t* __restrict__ dcnt) {
    __shared__ int32_t s_cnt[256];
    const int64_t q = blockIdx.x;
    const int32_t l = tl[q];
    const int32_t row = list[l];
    const int64_t base = toff[l] + (q - tcfirst[l]) * kTabChunk;
    constexpr int kPer = kTabChunk / 256;
    const int tid = threadIdx.x;
    int32_t mine = 0;
    for (int j = 0; j < kPer; ++j) mine += gk[base + tid * kPer + j] >= 0;
    s_cnt[tid] = mine;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const int32_t x = s_cnt[t];
            s_cnt[t] = run;
            run += x;
        }
    }
    __syncthreads();
    int64_t pos = rowoff[row] + (qoff[q] - qoff[tcfirst[l]]) + s_cnt[tid];
    for (int j = 0; j < kPer; ++j) {
        const int64_t e = base + tid * kPer + j;
        if (gk[e] < 0) continue;
        tk[pos] = gk[e];
        tw[pos] = gv[e];
        ++pos;
    }
    if (q == tcfirst[l] && tid == 0) dcnt[row] = static_cast<int32_t>(qoff[tcfirst[l + 1]] - qoff[tcfirst[l]]);
}

__global__ void row_degrees_kernel(int32_t n, const int64_t* __restrict__ xadj, int32_t* __restrict__ deg) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) deg[v] = static_cast<int32_t>(xadj[v + 1] - xadj[v]);
}

// Step 4: the merged prefix of every row to its place in the coarse CSR.
__global__ void __launch_bounds__(kTileThreads) row_copy_kernel(const int64_t* __restrict__ rowoff, int32_t nc, int64_t m,
                                                                const int32_t* __restrict__ dcnt,
                                                                const int64_t* __restrict__ cxadj,
                                                                const int32_t* __restrict__ tk,
                                                                const int32_t* __restrict__ tw,
                                                                int32_t* __restrict__ cadj, int32_t* __restrict__ cew, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const int64_t i1 = i0 + kTile < m ? i0 + kTile : m;
    tile_owners(rowoff, trow, static_cast<int64_t>(blockIdx.x), i0, i1, owner);
    for (int r = 0; r < kTilePer; ++r) {
        const int64_t i = i0 + r * kTileThreads + threadIdx.x;
        if (i >= i1) continue;
        const int32_t row = owner[i - i0];
        const int64_t li = i - rowoff[row];
        if (li < dcnt[row]) {
            cadj[cxadj[row] + li] = tk[i];
            cew[cxadj[row] + li] = tw[i];
        }
    }
}

// Unsorted merge of the workgroup rows, by length class (table of 512 <<
// class slots).
void hash_block_rows(const int32_t* list, uint32_t count, const int64_t* rowoff, const int32_t* rowcnt,
                     int32_t* tk, int32_t* tw, int32_t* dcnt, hipStream_t s) {
    DBuf<int32_t> sub(5 * static_cast<size_t>(count), s);
    DBuf<uint32_t> cnt(5, s);
    fill_u32(cnt.get(), 0, 5, s);
    block_row_split_kernel<<<std::min(grid_for(count, 256 * kClassifyIters), 1024u), 256, 0, s>>>(
        list, count, rowcnt, sub.get(), count, cnt.get());
    LAUNCHCHK();
    uint32_t hc[5];
    HIPCHK(hipMemcpyAsync(hc, cnt.get(), sizeof(hc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int32_t* l = sub.get();
    if (hc[0]) block_hash_rows_kernel<512><<<hc[0], 256, 0, s>>>(l, rowoff, rowcnt, tk, tw, dcnt);
    if (hc[1]) block_hash_rows_kernel<1024><<<hc[1], 256, 0, s>>>(l + count, rowoff, rowcnt, tk, tw, dcnt);
    if (hc[2]) block_hash_rows_kernel<2048><<<hc[2], 256, 0, s>>>(l + 2 * count, rowoff, rowcnt, tk, tw, dcnt);
    if (hc[3]) block_hash_rows_kernel<4096><<<hc[3], 256, 0, s>>>(l + 3 * count, rowoff, rowcnt, tk, tw, dcnt);
    if (hc[4]) block_hash_rows_kernel<8192><<<hc[4], 256, 0, s>>>(l + 4 * count, rowoff, rowcnt, tk, tw, dcnt);
    LAUNCHCHK();
}

// Long rows (unsorted) merged by buckets; false if a bucket's distinct
// neighbours overflowed its LDS table (tk/tw untouched then).
bool bucket_merge_long_rows(uint32_t nl, const int32_t* llist, int64_t nch, const int32_t* crow,
                            const int64_t* cfirst, const int32_t* ccnt, const int64_t* loff, int64_t ml,
                            const int64_t* rowoff, int32_t* tk, int32_t* tw, int32_t* dcnt, int32_t mean,
                            hipStream_t s) {
    ProfScope ps("contract_long_buckets", 40.0 * static_cast<double>(ml), s);
    DBuf<int32_t> nbk(nl, s);
    DBuf<int64_t> bfirst(static_cast<size_t>(nl) + 1, s), tot(2, s);
    long_bucket_counts_kernel<<<grid_for(nl, 256), 256, 0, s>>>(nl, loff, mean, llist, cfirst, dcnt, nbk.get());
    LAUNCHCHK();
    exclusive_scan_i32_to_i64(nbk.get(), bfirst.get(), nl, tot.get(), s);
    int64_t NB = 0;
    HIPCHK(hipMemcpyAsync(&NB, tot.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (NB == 0) return true;  // every long row was one chunk
    fill_i64(bfirst.get() + nl, NB, 1, s);
    DBuf<int32_t> brow(NB, s), bcount(NB, s), bfill(NB, s), qcnt(NB, s);
    DBuf<int64_t> boff(static_cast<size_t>(NB) + 1, s), qoff(static_cast<size_t>(NB) + 1, s);
    DBuf<int32_t> sk(std::max<int64_t>(ml, 1), s), sw(std::max<int64_t>(ml, 1), s);
    DBuf<uint32_t> overflow(1, s);
    long_bucket_rows_kernel<<<nl, 256, 0, s>>>(nl, bfirst.get(), brow.get());
    LAUNCHCHK();
    fill_i32(bcount.get(), 0, NB, s);
    fill_i32(bfill.get(), 0, NB, s);
    fill_u32(overflow.get(), 0, 1, s);
    long_bucket_scatter_kernel<false><<<static_cast<unsigned>(nch), 256, 0, s>>>(
        llist, crow, cfirst, ccnt, rowoff, bfirst.get(), tk, tw, bcount.get(), nullptr, nullptr, nullptr, nullptr);
    LAUNCHCHK();
    exclusive_scan_i32_to_i64(bcount.get(), boff.get(), NB, tot.get(), s);
    HIPCHK(hipMemcpyAsync(boff.get() + NB, tot.get(), sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    long_bucket_scatter_kernel<true><<<static_cast<unsigned>(nch), 256, 0, s>>>(
        llist, crow, cfirst, ccnt, rowoff, bfirst.get(), tk, tw, nullptr, boff.get(), bfill.get(), sk.get(),
        sw.get());
    LAUNCHCHK();
    long_bucket_merge_kernel<<<static_cast<unsigned>(NB), 256, 0, s>>>(boff.get(), sk.get(), sw.get(), qcnt.get(),
                                                                      overflow.get());
    LAUNCHCHK();
    uint32_t over = 0;
    HIPCHK(hipMemcpyAsync(&over, overflow.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (over) return false;
    exclusive_scan_i32_to_i64(qcnt.get(), qoff.get(), NB, tot.get() + 1, s);
    HIPCHK(hipMemcpyAsync(qoff.get() + NB, tot.get() + 1, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    long_bucket_write_kernel<<<static_cast<unsigned>(NB), 256, 0, s>>>(llist, brow.get(), bfirst.get(), boff.get(),
                                                                      qoff.get(), qcnt.get(), rowoff, sk.get(),
                                                                      sw.get(), tk, tw, dcnt);
    LAUNCHCHK();
    return true;
}

}  // namespace

// Merges (and, if `sorted`, orders by neighbour id) every row r of the
// entries tk/tw[rowoff[r] .. rowoff[r] + rowcnt[r]) in place; dcnt[r]
// receives the number of distinct neighbours, written at the row's start.
void merge_rows(int32_t nc, int64_t m, const int64_t* rowoff, const int32_t* rowcnt, int32_t* tk, int32_t* tw,
                int32_t* dcnt, bool sorted, hipStream_t s, int32_t bucket_mean = 0) {
    DBuf<int32_t> lists(3 * static_cast<size_t>(nc), s);
    DBuf<uint32_t> counts(3, s);
    uint32_t hc[3] = {0, 0, 0};
    {
        ProfScope ps("contract_rows", 16.0 * static_cast<double>(m), s);
        fill_u32(counts.get(), 0, 3, s);
        row_classify_kernel<<<std::min(grid_for(nc, 256 * kClassifyIters), 1024u), 256, 0, s>>>(
            nc, rowcnt, dcnt, lists.get(), nc, counts.get());
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(hc, counts.get(), sizeof(hc), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hc[0] > 0) {
            wave_rows_kernel<<<grid_for(static_cast<int64_t>(hc[0]) * 64, 256), 256, 0, s>>>(
                lists.get(), hc[0], rowoff, rowcnt, tk, tw, dcnt);
            LAUNCHCHK();
        }
        if (hc[1] > 0) {
            if (sorted)
                block_rows_kernel<<<hc[1], 256, 0, s>>>(lists.get() + nc, rowoff, rowcnt, tk, tw, dcnt);
            else
                hash_block_rows(lists.get() + nc, hc[1], rowoff, rowcnt, tk, tw, dcnt, s);
            LAUNCHCHK();
        }
    }
    if (hc[2] > 0) {
        ProfScope ps("contract_long_rows", 0, s);
        const uint32_t nl = hc[2];
        const int32_t* llist = lists.get() + 2 * static_cast<size_t>(nc);
        // chunks of the long rows, each merged in LDS first
        DBuf<int32_t> lens(nl, s);
        DBuf<int64_t> cfirst(static_cast<size_t>(nl) + 1, s), ctot(1, s);
        long_lens_kernel<<<grid_for(nl, 256), 256, 0, s>>>(llist, nl, rowcnt, lens.get(), kLongChunk);
        LAUNCHCHK();
        exclusive_scan_i32_to_i64(lens.get(), cfirst.get(), nl, ctot.get(), s);
        int64_t nch = 0;
        HIPCHK(hipMemcpyAsync(&nch, ctot.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fill_i64(cfirst.get() + nl, nch, 1, s);
        DBuf<int32_t> crow(nch, s), ccnt(nch, s);
        DBuf<int64_t> coff(static_cast<size_t>(nch) + 1, s), mtot2(1, s), loff(static_cast<size_t>(nl) + 1, s);
        {
            ProfScope ps_m("contract_long_merge", 0, s);
            long_chunks_kernel<<<nl, 256, 0, s>>>(nl, cfirst.get(), crow.get());
            LAUNCHCHK();
            long_dedup_kernel<<<static_cast<unsigned>(nch), kDedupThreads, 0, s>>>(llist, crow.get(), cfirst.get(),
                                                                                   rowoff, rowcnt, tk, tw, ccnt.get());
            LAUNCHCHK();
        }
        exclusive_scan_i32_to_i64(ccnt.get(), coff.get(), nch, mtot2.get(), s);
        int64_t ml = 0;
        HIPCHK(hipMemcpyAsync(&ml, mtot2.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fill_i64(coff.get() + nch, ml, 1, s);
        long_offsets_kernel<<<grid_for(static_cast<int64_t>(nl) + 1, 256), 256, 0, s>>>(nl, cfirst.get(), coff.get(),
                                                                                         loff.get());
        LAUNCHCHK();
        if (!sorted && bucket_merge_long_rows(nl, llist, nch, crow.get(), cfirst.get(), ccnt.get(), loff.get(), ml,
                                              rowoff, tk, tw, dcnt, bucket_mean > 0 ? bucket_mean : kBucketMean, s))
            return;
        if (!sorted) {  // a bucket overflowed: per-row tables in HBM
            DBuf<int64_t> tsz(nl, s), tch(nl, s), toff(static_cast<size_t>(nl) + 1, s),
                tcfirst(static_cast<size_t>(nl) + 1, s);
            long_table_sizes_kernel<<<grid_for(nl, 256), 256, 0, s>>>(nl, loff.get(), tsz.get(), tch.get());
            LAUNCHCHK();
            // offsets: [0, inclusive sums]
            fill_i64(toff.get(), 0, 1, s);
            fill_i64(tcfirst.get(), 0, 1, s);
            inclusive_scan_i64(tsz.get(), toff.get() + 1, nl, s);
            inclusive_scan_i64(tch.get(), tcfirst.get() + 1, nl, s);
            int64_t hts[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(&hts[0], toff.get() + nl, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&hts[1], tcfirst.get() + nl, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const int64_t ttot = hts[0], nq = hts[1];
            DBuf<int32_t> gk(ttot, s), gv(ttot, s), tl(nq, s), qcnt(nq, s);
            DBuf<int64_t> qoff(static_cast<size_t>(nq) + 1, s), qt(1, s);
            fill_i32(gk.get(), -1, ttot, s);
            fill_i32(gv.get(), 0, ttot, s);
            {
                ProfScope ps_i("contract_long_insert", 0, s);
                long_table_insert_kernel<<<static_cast<unsigned>(nch), 256, 0, s>>>(
                    llist, crow.get(), cfirst.get(), ccnt.get(), rowoff, tk, tw, toff.get(), tsz.get(), gk.get(),
                    gv.get());
                LAUNCHCHK();
            }
            long_table_chunks_kernel<<<nl, 256, 0, s>>>(nl, tcfirst.get(), tl.get());
            LAUNCHCHK();
            long_table_count_kernel<<<static_cast<unsigned>(nq), 256, 0, s>>>(tl.get(), tcfirst.get(), toff.get(),
                                                                            gk.get(), qcnt.get());
            LAUNCHCHK();
            exclusive_scan_i32_to_i64(qcnt.get(), qoff.get(), nq, qt.get(), s);
            HIPCHK(hipMemcpyAsync(qoff.get() + nq, qt.get(), sizeof(int64_t), hipMemcpyDeviceToDevice, s));
            long_table_write_kernel<<<static_cast<unsigned>(nq), 256, 0, s>>>(llist, tl.get(), tcfirst.get(),
                                                                            toff.get(), qoff.get(), rowoff, gk.get(),
                                                                            gv.get(), tk, tw, dcnt);
            LAUNCHCHK();
            return;
        }
        const int bn = std::max(1, bits_for(static_cast<uint64_t>(nc - 1)));
        DBuf<uint64_t> keys(ml, s), ktmp(ml, s);
        DBuf<uint32_t> vals(ml, s), vtmp(ml, s);
        long_keys_kernel<<<static_cast<unsigned>(nch), 256, 0, s>>>(llist, crow.get(), cfirst.get(), ccnt.get(),
                                                                    coff.get(), rowoff, tk, tw, bn, keys.get(),
                                                                    vals.get());
        LAUNCHCHK();
        {
            ProfScope ps2("contract_long_sort", 0, s);
            RadixScratch rs;
            radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), ml, 0,
                             bn + std::max(1, bits_for(static_cast<uint64_t>(nl - 1))), rs, s);
        }
        DBuf<int32_t> head(ml, s);
        DBuf<int64_t> pos(ml, s), psum(ml, s), dtot(1, s), run_start(ml, s);
        ktmp.release();
        vtmp.release();
        long_heads_kernel<<<grid_for(ml, 256), 256, 0, s>>>(keys.get(), vals.get(), ml, head.get(), psum.get());
        LAUNCHCHK();
        exclusive_scan_i32_to_i64(head.get(), pos.get(), ml, dtot.get(), s);
        inclusive_scan_i64(psum.get(), psum.get(), ml, s);
        long_runs_kernel<<<grid_for(ml, 256), 256, 0, s>>>(llist, loff.get(), rowoff, keys.get(), ml,
                                                           head.get(), pos.get(), bn, run_start.get(), tk,
                                                           dcnt);
        LAUNCHCHK();
        long_tails_kernel<<<grid_for(ml, 256), 256, 0, s>>>(llist, loff.get(), rowoff, keys.get(), ml,
                                                            head.get(), pos.get(), psum.get(), bn, run_start.get(),
                                                            tw);
        LAUNCHCHK();
    }

}


void contract(const DevGraph& g, const int32_t* labels, int32_t* C, OwnedDevGraph& coarse, hipStream_t s,
              const int32_t* probe, int32_t nprobe, int32_t* probe_out, bool sorted, int32_t bucket_mean) {
    const int32_t n = g.n;
    if (n == 0) {
        coarse.n = 0;
        coarse.S = 0;
        coarse.xadj.alloc(1, s);
        fill_i64(coarse.xadj.get(), 0, 1, s);
        if (nprobe > 0) fill_i32(probe_out, 0, nprobe, s);
        return;
    }
    // coarse ids: ranks of the used labels
    DBuf<int32_t> q(n, s);
    DBuf<int32_t> total(1, s);
    fill_i32(q.get(), 0, n, s);
    mark_used_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, labels, q.get());
    LAUNCHCHK();
    exclusive_scan_i32(q.get(), q.get(), n, total.get(), s);
    if (nprobe > 0) {
        probe_kernel<<<grid_for(nprobe, 256), 256, 0, s>>>(probe, nprobe, q.get(), n, total.get(), probe_out);
        LAUNCHCHK();
    }
    int32_t nc = 0;
    HIPCHK(hipMemcpyAsync(&nc, total.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    coarse.n = nc;
    coarse.vw.alloc(nc, s);
    fill_i32(coarse.vw.get(), 0, nc, s);
    map_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, labels, q.get(), g.vw, C, coarse.vw.get());
    LAUNCHCHK();
    q.release();
    coarse.xadj.alloc(static_cast<size_t>(nc) + 1, s);
    const int64_t ntiles = (g.S + kTile - 1) / kTile;

    // 1 + 2: inter-cluster slots bucketed by coarse source row
    DBuf<int32_t> rowcnt(nc, s);
    DBuf<int64_t> rowoff(static_cast<size_t>(nc) + 1, s), mtot(1, s);
    fill_i32(rowcnt.get(), 0, nc, s);
    int64_t m = 0;
    DBuf<int32_t> cross(n, s);
    DBuf<int32_t> cvs(g.S > 0 ? g.S : 1, s);  // C(v) of every slot
    TileRows gtiles(g.xadj, n, g.S, s);
    fill_i32(cross.get(), 0, n, s);
    if (g.S > 0) {
        ProfScope ps("contract_count", (8.0 + 8.0) * static_cast<double>(g.S) + 8.0 * n, s);
        cross_count_kernel<<<static_cast<unsigned>(ntiles), kTileThreads, 0, s>>>(g.xadj, g.adj, n, g.S, C,
                                                                                   cross.get(), cvs.get(),
                                                                                   gtiles.trow.get());
        LAUNCHCHK();
        row_count_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, C, cross.get(), rowcnt.get());
        LAUNCHCHK();
    }
    exclusive_scan_i32_to_i64(rowcnt.get(), rowoff.get(), nc, mtot.get(), s);
    HIPCHK(hipMemcpyAsync(&m, mtot.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (m == 0) {
        coarse.S = 0;
        coarse.adj.alloc(1, s);
        coarse.ew.alloc(1, s);
        fill_i64(coarse.xadj.get(), 0, static_cast<int64_t>(nc) + 1, s);
        HIPCHK(hipStreamSynchronize(s));
        return;
    }
    fill_i64(rowoff.get() + nc, m, 1, s);
    DBuf<int32_t> tk(m, s), tw(m, s);
    {
        ProfScope ps("contract_emit", (4.0 + (g.ew ? 4.0 : 0.0)) * static_cast<double>(g.S) + 8.0 * n + 8.0 * m, s);
        DBuf<int32_t> fill(nc, s), nfill(n, s);
        DBuf<int64_t> nbase(n, s);
        fill_i32(fill.get(), 0, nc, s);
        fill_i32(nfill.get(), 0, n, s);
        node_base_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, C, cross.get(), rowoff.get(), fill.get(), nbase.get());
        LAUNCHCHK();
        row_scatter_kernel<<<static_cast<unsigned>(ntiles), kTileThreads, 0, s>>>(
            g.xadj, cvs.get(), g.ew, n, g.S, C, nbase.get(), nfill.get(), tk.get(), tw.get(), gtiles.trow.get());
        LAUNCHCHK();
    }
    cvs.release();

    // 3: merge (and order) every row
    DBuf<int32_t> dcnt(nc, s);
    merge_rows(nc, m, rowoff.get(), rowcnt.get(), tk.get(), tw.get(), dcnt.get(), sorted, s, bucket_mean);

    // 4: coarse offsets and the merged rows
    ProfScope ps_copy("contract_copy", 16.0 * static_cast<double>(m), s);
    DBuf<int64_t> stot(1, s);
    exclusive_scan_i32_to_i64(dcnt.get(), coarse.xadj.get(), nc, stot.get(), s);
    int64_t Sc = 0;
    HIPCHK(hipMemcpyAsync(&Sc, stot.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    fill_i64(coarse.xadj.get() + nc, Sc, 1, s);
    coarse.S = Sc;
    coarse.adj.alloc(std::max<int64_t>(Sc, 1), s);
    coarse.ew.alloc(std::max<int64_t>(Sc, 1), s);
    const int64_t mtiles = (m + kTile - 1) / kTile;
    TileRows ctiles(rowoff.get(), nc, m, s);
    row_copy_kernel<<<static_cast<unsigned>(mtiles), kTileThreads, 0, s>>>(rowoff.get(), nc, m, dcnt.get(),
                                                                           coarse.xadj.get(), tk.get(), tw.get(),
                                                                           coarse.adj.get(), coarse.ew.get(),
                                                                           ctiles.trow.get());
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
}

void sort_rows(OwnedDevGraph& g, hipStream_t s) {
    if (g.n == 0 || g.S == 0) return;
    ProfScope ps("contract_sort_rows", 16.0 * static_cast<double>(g.S), s);
    DBuf<int32_t> deg(g.n, s), dcnt(g.n, s);
    row_degrees_kernel<<<grid_for(g.n, 256), 256, 0, s>>>(g.n, g.xadj.get(), deg.get());
    LAUNCHCHK();
    merge_rows(g.n, g.S, g.xadj.get(), deg.get(), g.adj.get(), g.ew.get(), dcnt.get(), true, s);
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace sclap
