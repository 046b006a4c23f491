// Projection, cut / block weights, validation and the batch helpers on
// gfx950 (contraction is in contract.hip).  Slot-parallel kernels use the
// slot tiles of tiles.hpp.
#include <climits>
#include <mutex>
#include <string>

#include "graph_ops.hpp"
#include "sclap.h"
#include "profile.hpp"
#include "tiles.hpp"

namespace sclap {

namespace {

__global__ void project_kernel(int32_t n, const int32_t* __restrict__ C, const int32_t* __restrict__ cp,
                               int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) part[v] = cp[C[v]];
}

// ---------------------------------------------------------- cut and weights

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v) {
    __shared__ unsigned long long s[kTileThreads / kWave];
    v = wave_sum(v);
    if (lane_id() == 0) s[threadIdx.x / kWave] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < kTileThreads / kWave; ++w) t += s[w];
    __syncthreads();
    return t;
}

// Grid-stride over tiles; one atomic per workgroup.  P: the block type read
// for every neighbour (a byte copy when k <= 256: four times the neighbours
// per cache line of the random gather).
template <typename P>
__global__ void __launch_bounds__(kTileThreads) cut_kernel(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                                                           const int32_t* __restrict__ ew, int32_t n, int64_t S,
                                                           const P* __restrict__ part,
                                                           unsigned long long* __restrict__ cut, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    unsigned long long acc = 0;
    for (int64_t tile = blockIdx.x; tile * kTile < S; tile += gridDim.x) {
        const int64_t i0 = tile * kTile;
        const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
        tile_owners(xadj, trow, tile, i0, i1, owner);
        for (int r = 0; r < kTilePer; ++r) {
            const int64_t i = i0 + r * kTileThreads + threadIdx.x;
            if (i < i1 && part[owner[i - i0]] != part[adj[i]]) acc += ew ? static_cast<unsigned long long>(ew[i]) : 1ULL;
        }
        __syncthreads();
    }
    acc = block_sum_u64(acc);
    if (threadIdx.x == 0 && acc) atomicAdd(cut, acc);
}

__global__ void to_u8_kernel(int32_t n, const int32_t* __restrict__ part, uint8_t* __restrict__ out) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) out[v] = static_cast<uint8_t>(part[v]);
}

__global__ void __launch_bounds__(256) block_weight_kernel(int32_t n, const int32_t* __restrict__ part,
                                                           const int32_t* __restrict__ vw, int32_t k,
                                                           unsigned long long* __restrict__ bw) {
    __shared__ unsigned long long loc[1024];
    const bool use_lds = k <= 1024;
    if (use_lds)
        for (int j = threadIdx.x; j < k; j += 256) loc[j] = 0;
    __syncthreads();
    for (int32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const unsigned long long c = vw ? static_cast<unsigned long long>(vw[v]) : 1ULL;
        if (c) {
            if (use_lds) atomicAdd(&loc[part[v]], c);
            else atomicAdd(&bw[part[v]], c);
        }
    }
    __syncthreads();
    if (use_lds)
        for (int j = threadIdx.x; j < k; j += 256)
            if (loc[j]) atomicAdd(&bw[j], loc[j]);
}

// ------------------------------------------------------------- validation

struct VStats {
    unsigned long long cV;
    unsigned long long wsum;
    unsigned long long hfwd;
    unsigned long long hbwd;
    int32_t cmax;
    uint32_t bad;  // bit 0: structure / range, bit 1: negative node weight, bit 2: edge weight < 1
    uint32_t pad[2];
};

// Hash of a directed slot (u, v, w): sums over all slots and over all
// reversed slots agree for a symmetric graph.  One mix of the ordered pair,
// with the weight spread over all 64 bits by an odd multiplier.
__device__ __forceinline__ unsigned long long edge_hash(uint32_t u, uint32_t v, uint32_t w) {
    return mix64(((static_cast<uint64_t>(u) << 32) | v) ^ (static_cast<uint64_t>(w) * 0xD6E8FEB86659FD93ULL));
}

__global__ void __launch_bounds__(kTileThreads) validate_nodes_kernel(int32_t n, const int64_t* __restrict__ xadj,
                                                                      const int32_t* __restrict__ vw, VStats* st) {
    __shared__ int32_t s_max[kTileThreads / kWave];
    unsigned long long c = 0;
    int32_t cm = 0;
    uint32_t bad = 0;
    for (int32_t v = blockIdx.x * kTileThreads + threadIdx.x; v < n; v += gridDim.x * kTileThreads) {
        if (xadj[v + 1] < xadj[v]) bad |= 1u;
        const int32_t cv = vw ? vw[v] : 1;
        if (cv < 0) {
            bad |= 2u;
        } else {
            c += static_cast<unsigned long long>(cv);
            cm = cv > cm ? cv : cm;
        }
    }
    c = block_sum_u64(c);
    cm = wave_max(cm);
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = cm;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < kTileThreads / kWave; ++w) cm = s_max[w] > cm ? s_max[w] : cm;
        if (c) atomicAdd(&st->cV, c);
        atomicMax(&st->cmax, cm);
    }
    if (bad) atomicOr(&st->bad, bad);
}

__global__ void __launch_bounds__(kTileThreads) validate_slots_kernel(const int64_t* __restrict__ xadj,
                                                                      const int32_t* __restrict__ adj,
                                                                      const int32_t* __restrict__ ew, int32_t n,
                                                                      int64_t S, VStats* st, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    unsigned long long ws = 0, hf = 0, hb = 0;
    uint32_t bad = 0;
    for (int64_t tile = blockIdx.x; tile * kTile < S; tile += gridDim.x) {
        const int64_t i0 = tile * kTile;
        const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
        tile_owners(xadj, trow, tile, i0, i1, owner);
        for (int r = 0; r < kTilePer; ++r) {
            const int64_t i = i0 + r * kTileThreads + threadIdx.x;
            if (i >= i1) continue;
            const int32_t u = owner[i - i0];
            const int32_t x = adj[i];
            const int32_t w = ew ? ew[i] : 1;
            if (x < 0 || x >= n || x == u) bad |= 1u;
            if (w < 1) bad |= 4u;
            ws += static_cast<unsigned long long>(w > 0 ? w : 0);
            hf += edge_hash(static_cast<uint32_t>(u), static_cast<uint32_t>(x), static_cast<uint32_t>(w));
            hb += edge_hash(static_cast<uint32_t>(x), static_cast<uint32_t>(u), static_cast<uint32_t>(w));
        }
        __syncthreads();
    }
    ws = block_sum_u64(ws);
    hf = block_sum_u64(hf);
    hb = block_sum_u64(hb);
    if (threadIdx.x == 0) {
        if (ws) atomicAdd(&st->wsum, ws);
        atomicAdd(&st->hfwd, hf);
        atomicAdd(&st->hbwd, hb);
    }
    if (bad) atomicOr(&st->bad, bad);
}

// Flags any value outside [lo, hi) with at most one atomic per wave (a
// per-element atomic on the one flag serialises when most values are out,
// as in the unit-weight test of a weighted graph).
__global__ void range_kernel(const int32_t* __restrict__ a, int64_t count, int32_t lo, int32_t hi,
                             uint32_t* __restrict__ bad) {
    bool b = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const int32_t x = a[i];
        b |= x < lo || x >= hi;
    }
    if (__any(b) && lane_id() == 0) atomicOr(bad, 1u);
}

unsigned capped_tiles(int64_t S) {
    const int64_t t = (S + kTile - 1) / kTile;
    return static_cast<unsigned>(t < 1 ? 1 : (t > 2048 ? 2048 : t));
}

unsigned capped_nodes(int64_t n) {
    const int64_t t = (n + kTileThreads - 1) / kTileThreads;
    return static_cast<unsigned>(t < 1 ? 1 : (t > 2048 ? 2048 : t));
}

}  // namespace

void project(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part, hipStream_t s) {
    if (n <= 0) return;
    project_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, C, coarse_part, part);
    LAUNCHCHK();
}

void cut_and_weights(const DevGraph& g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw, hipStream_t s) {
    DBuf<unsigned long long> acc(1 + static_cast<size_t>(k), s);
    HIPCHK(hipMemsetAsync(acc.get(), 0, (1 + static_cast<size_t>(k)) * sizeof(unsigned long long), s));
    if (g.S > 0) {
        TileRows tr(g.xadj, g.n, g.S, s);
        if (k <= 256) {
            DBuf<uint8_t> p8(g.n, s);
            to_u8_kernel<<<grid_for(g.n, 256), 256, 0, s>>>(g.n, part, p8.get());
            LAUNCHCHK();
            cut_kernel<uint8_t><<<capped_tiles(g.S), kTileThreads, 0, s>>>(g.xadj, g.adj, g.ew, g.n, g.S, p8.get(),
                                                                          acc.get(), tr.trow.get());
        } else {
            cut_kernel<int32_t><<<capped_tiles(g.S), kTileThreads, 0, s>>>(g.xadj, g.adj, g.ew, g.n, g.S, part,
                                                                          acc.get(), tr.trow.get());
        }
        LAUNCHCHK();
    }
    if (g.n > 0) {
        block_weight_kernel<<<capped_nodes(g.n), 256, 0, s>>>(g.n, part, g.vw, k, acc.get() + 1);
        LAUNCHCHK();
    }
    std::vector<unsigned long long> h(1 + static_cast<size_t>(k));
    HIPCHK(hipMemcpyAsync(h.data(), acc.get(), h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *cut = static_cast<int64_t>(h[0] / 2);
    for (int32_t b = 0; b < k; ++b) bw[b] = static_cast<int64_t>(h[1 + b]);
}

// ------------------------------------------- cut without device allocation
//
// Workspace of cut_and_weights_noalloc: a fixed array in the library's
// device image (every device the library runs on holds its own copy until
// the process ends).  Layout: the cut and up to kNoAllocMaxK block weight
// accumulators (u64), the range flag, then from kNoAllocAccBytes the first
// row of every slot tile (int32).  Calls that overlap on one device share
// it and race; each call clears the accumulators and the flag itself.

namespace {

constexpr size_t kNoAllocBytes = size_t(16) << 20;
constexpr int32_t kNoAllocMaxK = 65536;
constexpr size_t kNoAllocAccBytes = size_t(1) << 20;  // 8 * (1 + kNoAllocMaxK) + 4 fits
constexpr int64_t kNoAllocMaxTiles = static_cast<int64_t>((kNoAllocBytes - kNoAllocAccBytes) / sizeof(int32_t)) - 1;
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device (the array's name is only a host-side handle).
unsigned char* noalloc_scratch() {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) fail(SCLAP_ERR_INVALID, "device index beyond the workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) fail(SCLAP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

}  // namespace

void cut_and_weights_noalloc(const DevGraph& g, const int32_t* part, int32_t k, int64_t* cut, int64_t* bw,
                             hipStream_t s) {
    const int64_t ntiles = g.S > 0 ? (g.S + kTile - 1) / kTile : 0;
    if (k > kNoAllocMaxK) fail(SCLAP_ERR_INVALID, "k exceeds the no-allocation workspace (at most 65536 blocks)");
    if (ntiles > kNoAllocMaxTiles)
        fail(SCLAP_ERR_INVALID, "graph exceeds the no-allocation workspace (at most 3,932,159 tiles of 2048 slots)");
    unsigned char* ws = noalloc_scratch();
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws);
    uint32_t* flag = reinterpret_cast<uint32_t*>(ws + sizeof(unsigned long long) * (1 + static_cast<size_t>(kNoAllocMaxK)));
    int32_t* trow = reinterpret_cast<int32_t*>(ws + kNoAllocAccBytes);
    // cleared by kernels (no memset node if a caller captures the call)
    fill_u32(reinterpret_cast<uint32_t*>(acc), 0, 2 * (1 + static_cast<int64_t>(k)), s);
    fill_u32(flag, 0, 1, s);
    if (g.n > 0) {
        range_kernel<<<grid_for(g.n, 256), 256, 0, s>>>(part, g.n, 0, k, flag);
        LAUNCHCHK();
        uint32_t bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad) fail(SCLAP_ERR_INVALID, "part value outside [0, k)");
    }
    if (ntiles > 0) {
        tile_rows_kernel<<<grid_for(ntiles + 1, 256), 256, 0, s>>>(g.xadj, g.n, g.S, ntiles, trow);
        LAUNCHCHK();
        cut_kernel<int32_t><<<capped_tiles(g.S), kTileThreads, 0, s>>>(g.xadj, g.adj, g.ew, g.n, g.S, part, acc, trow);
        LAUNCHCHK();
    }
    if (g.n > 0) {
        block_weight_kernel<<<capped_nodes(g.n), 256, 0, s>>>(g.n, part, g.vw, k, acc + 1);
        LAUNCHCHK();
    }
    unsigned long long c2 = 0;
    HIPCHK(hipMemcpyAsync(&c2, acc, sizeof(c2), hipMemcpyDeviceToHost, s));
    // block weights are non-negative and below 2^63: the u64 sums are the int64 values
    HIPCHK(hipMemcpyAsync(bw, acc + 1, sizeof(int64_t) * static_cast<size_t>(k), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *cut = static_cast<int64_t>(c2 / 2);
}

// ------------------------------------------------------ gather-rate probe
//
// The access that bounds node evaluation: for every adjacency slot, the
// label of the neighbour (a random 1- or 4-byte read).  The probe sums
// label[adj[e]] over all slots with several loads in flight per thread and
// writes one number, so its time is the rate at which this graph's neighbour
// labels can be gathered at all.

namespace {

template <typename T>
__global__ void __launch_bounds__(256) gather_probe_kernel(const int32_t* __restrict__ adj, const T* __restrict__ lab,
                                                           int64_t S, unsigned long long* __restrict__ out) {
    constexpr int U = 8;
    unsigned long long acc = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256 * U;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * 256 * U + threadIdx.x; b < S; b += stride) {
        int32_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = b + u * 256;
            x[u] = e < S ? adj[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += x[u] >= 0 ? static_cast<unsigned long long>(lab[x[u]]) : 0ULL;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) atomicAdd(out, acc);
}

}  // namespace

float gather_probe(const DevGraph& g, int32_t label_bytes, int32_t reps, hipStream_t s) {
    if (g.S == 0 || g.n == 0) return 0.0f;
    if (label_bytes != 1 && label_bytes != 4) fail(SCLAP_ERR_INVALID, "label_bytes must be 1 or 4");
    DBuf<int32_t> lab(g.n, s);
    iota_u32(reinterpret_cast<uint32_t*>(lab.get()), g.n, s);  // any values: only the addresses matter
    DBuf<unsigned long long> out(1, s);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const unsigned grid = 4096;
    auto launch = [&] {
        if (label_bytes == 1)
            gather_probe_kernel<uint8_t><<<grid, 256, 0, s>>>(g.adj, reinterpret_cast<const uint8_t*>(lab.get()),
                                                              g.S, out.get());
        else
            gather_probe_kernel<int32_t><<<grid, 256, 0, s>>>(g.adj, lab.get(), g.S, out.get());
        LAUNCHCHK();
    };
    launch();  // warm-up
    HIPCHK(hipEventRecord(e0, s));
    for (int32_t r = 0; r < reps; ++r) launch();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / static_cast<float>(reps > 0 ? reps : 1);
}

int validate_graph(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s) {
    const int32_t n = g.n;
    if (n < 0) return -1;
    if (n == 0) {
        *cV = 0;
        *cmax = 0;
        return 0;
    }
    if (!g.xadj) return -1;
    int64_t ends[2];
    HIPCHK(hipMemcpyAsync(&ends[0], g.xadj, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&ends[1], g.xadj + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != g.S || g.S < 0) return -1;
    if (g.S > 0 && !g.adj) return -1;
    DBuf<VStats> st(1, s);
    HIPCHK(hipMemsetAsync(st.get(), 0, sizeof(VStats), s));
    validate_nodes_kernel<<<capped_nodes(n), kTileThreads, 0, s>>>(n, g.xadj, g.vw, st.get());
    LAUNCHCHK();
    VStats h;
    HIPCHK(hipMemcpyAsync(&h, st.get(), sizeof(VStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h.bad) return -1;  // offsets not monotone or negative node weight
    if (g.S > 0) {
        TileRows tr(g.xadj, n, g.S, s);  // offsets checked monotone above
        validate_slots_kernel<<<capped_tiles(g.S), kTileThreads, 0, s>>>(g.xadj, g.adj, g.ew, n, g.S, st.get(),
                                                                          tr.trow.get());
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(&h, st.get(), sizeof(VStats), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (h.bad) return -1;
    if (h.cV > 2147483647ULL || h.wsum / 2 > 2147483647ULL) return -3;
    if (h.hfwd != h.hbwd) return -2;
    *cV = static_cast<int64_t>(h.cV);
    *cmax = h.cmax;
    return 0;
}

void node_weight_stats(const DevGraph& g, int64_t* cV, int64_t* cmax, hipStream_t s) {
    if (g.n == 0) {
        *cV = 0;
        *cmax = 0;
        return;
    }
    DBuf<VStats> st(1, s);
    HIPCHK(hipMemsetAsync(st.get(), 0, sizeof(VStats), s));
    validate_nodes_kernel<<<capped_nodes(g.n), kTileThreads, 0, s>>>(g.n, g.xadj, g.vw, st.get());
    LAUNCHCHK();
    VStats h;
    HIPCHK(hipMemcpyAsync(&h, st.get(), sizeof(VStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *cV = static_cast<int64_t>(h.cV);
    *cmax = h.cmax;
}

bool all_in_range(const int32_t* a, int64_t count, int32_t lo, int32_t hi, hipStream_t s) {
    if (count <= 0) return true;
    DBuf<uint32_t> bad(1, s);
    fill_u32(bad.get(), 0, 1, s);
    range_kernel<<<static_cast<unsigned>(std::min<int64_t>((count + 255) / 256, 8192)), 256, 0, s>>>(a, count, lo, hi,
                                                                                                    bad.get());
    LAUNCHCHK();
    uint32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, bad.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return h == 0;
}

// ---------------------------------------------- several graphs in one CSR
//
// Member m of a batch owns nodes [nb[m], nb[m+1]) and slots [sb[m], sb[m+1]);
// no edge leaves a member.  Empty members are allowed.

namespace {

// Largest m in [0, M) with base[m] <= x (base non-decreasing, base[0] <= x).
template <typename T>
__device__ __forceinline__ int32_t member_of(const T* __restrict__ base, int32_t M, int64_t x) {
    int32_t lo = 0, hi = M;
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (static_cast<int64_t>(base[mid]) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void member_ids_kernel(int32_t n, int32_t M, const int32_t* __restrict__ nb,
                                  const int32_t* __restrict__ ids, int32_t* __restrict__ gid) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) gid[v] = ids[member_of(nb, M, v)];
}

__global__ void members_closed_kernel(int64_t S, int32_t M, const int64_t* __restrict__ sb,
                                      const int32_t* __restrict__ nb, const int32_t* __restrict__ adj,
                                      uint32_t* __restrict__ bad) {
    uint32_t b = 0;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < S;
         j += static_cast<int64_t>(gridDim.x) * 256) {
        const int32_t m = member_of(sb, M, j);
        const int32_t u = adj[j];
        if (u < nb[m] || u >= nb[m + 1]) b = 1;
    }
    if (__any(b) && lane_id() == 0) atomicOr(bad, 1u);
}

// One atomic per wave when the wave's items belong to one graph (graphs are
// contiguous), else one per item.
__device__ __forceinline__ void add_by_graph(bool valid, int32_t g, unsigned long long val,
                                             unsigned long long* __restrict__ out) {
    const int32_t lo = wave_min(valid ? g : INT_MAX);
    const int32_t hi = wave_max(valid ? g : -1);
    if (lo == hi) {
        const unsigned long long t = wave_sum(valid ? val : 0ULL);
        if (lane_id() == 0 && t) atomicAdd(&out[lo], t);
    } else if (valid && val) {
        atomicAdd(&out[g], val);
    }
}

__global__ void graph_node_stats_kernel(int32_t n, const int32_t* __restrict__ gid, const int32_t* __restrict__ vw,
                                        unsigned long long* __restrict__ cV, unsigned long long* __restrict__ cmax) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    const bool valid = v < n;
    const int32_t g = valid ? gid[v] : 0;
    const int32_t c = valid ? (vw ? vw[v] : 1) : 0;
    add_by_graph(valid, g, static_cast<unsigned long long>(c < 0 ? 0 : c), cV);
    const int32_t lo = wave_min(valid ? g : INT_MAX);
    const int32_t hi = wave_max(valid ? g : -1);
    if (lo == hi) {
        const int32_t m = wave_max(valid ? c : 0);
        if (lane_id() == 0 && m > 0) atomicMax(&cmax[lo], static_cast<unsigned long long>(m));
    } else if (valid && c > 0) {
        atomicMax(&cmax[g], static_cast<unsigned long long>(c));
    }
}

__global__ void __launch_bounds__(kTileThreads) graph_cut_kernel(const int64_t* __restrict__ xadj,
                                                                 const int32_t* __restrict__ adj,
                                                                 const int32_t* __restrict__ ew, int32_t n, int64_t S,
                                                                 const int32_t* __restrict__ part,
                                                                 const int32_t* __restrict__ gid,
                                                                 unsigned long long* __restrict__ cut, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    for (int64_t tile = blockIdx.x; tile * kTile < S; tile += gridDim.x) {
        const int64_t i0 = tile * kTile;
        const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
        tile_owners(xadj, trow, tile, i0, i1, owner);
        // each lane sums its slots of the tile per graph (its graph changes
        // at most at a graph boundary), then one atomic per wave when the
        // wave's lanes ended in one graph
        int32_t gc = -1;
        unsigned long long acc = 0;
        for (int r = 0; r < kTilePer; ++r) {
            const int64_t i = i0 + r * kTileThreads + threadIdx.x;
            if (i >= i1) break;
            const int32_t u = owner[i - i0];
            const int32_t g = gid[u];
            if (g != gc) {
                if (acc) atomicAdd(&cut[gc], acc);
                gc = g;
                acc = 0;
            }
            if (part[u] != part[adj[i]]) acc += ew ? static_cast<unsigned long long>(ew[i]) : 1ULL;
        }
        add_by_graph(gc >= 0, gc, acc, cut);
        __syncthreads();
    }
}

__global__ void compact_nodes_kernel(int32_t n_new, int32_t Mk, const int32_t* __restrict__ nnb,
                                     const int32_t* __restrict__ onb, const int64_t* __restrict__ osb,
                                     const int64_t* __restrict__ nsb, const int64_t* __restrict__ oxadj,
                                     const int32_t* __restrict__ ovw, int64_t S_new, int64_t* __restrict__ nxadj,
                                     int32_t* __restrict__ nvw) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i == 0) nxadj[n_new] = S_new;
    if (i >= n_new) return;
    const int32_t m = member_of(nnb, Mk, i);
    const int32_t o = onb[m] + (i - nnb[m]);
    nxadj[i] = oxadj[o] - osb[m] + nsb[m];
    nvw[i] = ovw[o];
}

__global__ void compact_slots_kernel(int64_t S_new, int32_t Mk, const int64_t* __restrict__ nsb,
                                     const int64_t* __restrict__ osb, const int32_t* __restrict__ onb,
                                     const int32_t* __restrict__ nnb, const int32_t* __restrict__ oadj,
                                     const int32_t* __restrict__ oew, int32_t* __restrict__ nadj,
                                     int32_t* __restrict__ new_) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < S_new;
         j += static_cast<int64_t>(gridDim.x) * 256) {
        const int32_t m = member_of(nsb, Mk, j);
        const int64_t o = osb[m] + (j - nsb[m]);
        nadj[j] = oadj[o] - onb[m] + nnb[m];
        new_[j] = oew[o];
    }
}

__global__ void pack_nodes_kernel(int32_t n_new, int32_t Mk, const int32_t* __restrict__ nnb,
                                  const int32_t* __restrict__ onb, const int64_t* __restrict__ osb,
                                  const int64_t* __restrict__ oxadj, const int32_t* __restrict__ ovw,
                                  int64_t* __restrict__ nx, int32_t* __restrict__ nvw, int32_t* __restrict__ has_deg) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_new) return;
    const int32_t m = member_of(nnb, Mk, i);
    const int32_t o = onb[m] + (i - nnb[m]);
    nx[i + m] = oxadj[o] - osb[m];
    if (i + 1 == nnb[m + 1]) nx[i + m + 1] = oxadj[o + 1] - osb[m];
    if (nvw) nvw[i] = ovw[o];
    has_deg[i] = oxadj[o + 1] > oxadj[o] ? 1 : 0;
}

// rank: exclusive prefix count of has_deg over the packed nodes
__global__ void pack_slots_kernel(int64_t S_new, int32_t Mk, const int64_t* __restrict__ nsb,
                                  const int64_t* __restrict__ osb, const int32_t* __restrict__ onb,
                                  const int32_t* __restrict__ nnb, const int32_t* __restrict__ has_deg,
                                  const int32_t* __restrict__ rank, const int32_t* __restrict__ oadj,
                                  int32_t* __restrict__ nadj) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < S_new;
         j += static_cast<int64_t>(gridDim.x) * 256) {
        const int32_t m = member_of(nsb, Mk, j);
        const int32_t xp = nnb[m] + (oadj[osb[m] + (j - nsb[m])] - onb[m]);
        // a neighbour outside the member (an unchecked input with an edge
        // between graphs) reads as -1, which the host partitioner reports
        const bool inside = xp >= nnb[m] && xp < nnb[m + 1];
        nadj[j] = inside && has_deg[xp] ? rank[xp] - rank[nnb[m]] : -1;
    }
}

__global__ void unpack_members_kernel(int32_t n_new, int32_t Mk, const int32_t* __restrict__ nnb,
                                      const int32_t* __restrict__ onb, const int32_t* __restrict__ src,
                                      int32_t* __restrict__ dst) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_new) return;
    const int32_t m = member_of(nnb, Mk, i);
    dst[onb[m] + (i - nnb[m])] = src[i];
}

__global__ void remap_members_kernel(int32_t n, const int32_t* __restrict__ gid, const int32_t* __restrict__ delta,
                                     int32_t* __restrict__ C) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t d = delta[gid[v]];
    C[v] = d == INT_MIN ? -1 : C[v] + d;
}

__global__ void project_kept_kernel(int32_t n, const int32_t* __restrict__ C, const int32_t* __restrict__ cp,
                                    int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n && C[v] >= 0) part[v] = cp[C[v]];
}

__global__ void shift_by_graph_kernel(int32_t n, const int32_t* __restrict__ gid, const int32_t* __restrict__ add,
                                      int32_t sign, int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) part[v] += sign * add[gid[v]];
}

__global__ void gather_offsets_kernel(const int64_t* __restrict__ xadj, const int32_t* __restrict__ pos, int32_t M,
                                      int64_t* __restrict__ out) {
    const int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m < M) out[m] = xadj[pos[m]];
}

unsigned capped_grid_s(int64_t items) {
    const int64_t g = (items + 255) / 256;
    return static_cast<unsigned>(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

void member_ids(int32_t n, const std::vector<int32_t>& nb, const std::vector<int32_t>& ids, int32_t* gid,
                hipStream_t s) {
    if (n == 0) return;
    const int32_t M = static_cast<int32_t>(ids.size());
    DBuf<int32_t> d(2 * static_cast<size_t>(M) + 1, s);
    HIPCHK(hipMemcpyAsync(d.get(), nb.data(), (M + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.get() + M + 1, ids.data(), M * sizeof(int32_t), hipMemcpyHostToDevice, s));
    member_ids_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, M, d.get(), d.get() + M + 1, gid);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));  // host vectors may go away
}

std::vector<int64_t> member_slot_bases(const int64_t* xadj, const std::vector<int32_t>& nb, hipStream_t s) {
    const int32_t M1 = static_cast<int32_t>(nb.size());
    std::vector<int64_t> sb(M1);
    DBuf<int32_t> pos(M1, s);
    DBuf<int64_t> out(M1, s);
    HIPCHK(hipMemcpyAsync(pos.get(), nb.data(), M1 * sizeof(int32_t), hipMemcpyHostToDevice, s));
    gather_offsets_kernel<<<grid_for(M1, 256), 256, 0, s>>>(xadj, pos.get(), M1, out.get());
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(sb.data(), out.get(), M1 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return sb;
}

bool members_closed(const DevGraph& g, const std::vector<int32_t>& nb, const std::vector<int64_t>& sb,
                    hipStream_t s) {
    if (g.S == 0) return true;
    const int32_t M = static_cast<int32_t>(nb.size()) - 1;
    DBuf<int32_t> dnb(M + 1, s);
    DBuf<int64_t> dsb(M + 1, s);
    DBuf<uint32_t> bad(1, s);
    HIPCHK(hipMemcpyAsync(dnb.get(), nb.data(), (M + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dsb.get(), sb.data(), (M + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    fill_u32(bad.get(), 0, 1, s);
    members_closed_kernel<<<capped_grid_s(g.S), 256, 0, s>>>(g.S, M, dsb.get(), dnb.get(), g.adj, bad.get());
    LAUNCHCHK();
    uint32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, bad.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return h == 0;
}

void graph_node_stats(int32_t n, const int32_t* gid, const int32_t* vw, int32_t G, int64_t* cV, int64_t* cmax,
                      hipStream_t s) {
    DBuf<unsigned long long> d(2 * static_cast<size_t>(std::max(G, 1)), s);
    HIPCHK(hipMemsetAsync(d.get(), 0, 2 * std::max(G, 1) * sizeof(unsigned long long), s));
    if (n > 0) {
        graph_node_stats_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, vw, d.get(), d.get() + G);
        LAUNCHCHK();
    }
    std::vector<unsigned long long> h(2 * static_cast<size_t>(std::max(G, 1)));
    HIPCHK(hipMemcpyAsync(h.data(), d.get(), h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int32_t g = 0; g < G; ++g) {
        cV[g] = static_cast<int64_t>(h[g]);
        cmax[g] = static_cast<int64_t>(h[G + g]);
    }
}

void graph_cuts(const DevGraph& g, const int32_t* part, const int32_t* gid, int32_t G, int64_t* cut, hipStream_t s) {
    DBuf<unsigned long long> d(std::max(G, 1), s);
    HIPCHK(hipMemsetAsync(d.get(), 0, std::max(G, 1) * sizeof(unsigned long long), s));
    if (g.S > 0) {
        const int64_t ntiles = (g.S + kTile - 1) / kTile;
        const unsigned grid = static_cast<unsigned>(ntiles < 2048 ? ntiles : 2048);
        TileRows tr(g.xadj, g.n, g.S, s);
        graph_cut_kernel<<<grid, kTileThreads, 0, s>>>(g.xadj, g.adj, g.ew, g.n, g.S, part, gid, d.get(),
                                                       tr.trow.get());
        LAUNCHCHK();
    }
    std::vector<unsigned long long> h(std::max(G, 1));
    HIPCHK(hipMemcpyAsync(h.data(), d.get(), h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int32_t i = 0; i < G; ++i) cut[i] = static_cast<int64_t>(h[i] / 2);
}

void compact_members(const DevGraph& src, const std::vector<int32_t>& onb, const std::vector<int64_t>& osb,
                     const std::vector<int32_t>& nnb, const std::vector<int64_t>& nsb, OwnedDevGraph& dst,
                     hipStream_t s) {
    const int32_t Mk = static_cast<int32_t>(onb.size());
    const int32_t n_new = nnb[Mk];
    const int64_t S_new = nsb[Mk];
    dst.n = n_new;
    dst.S = S_new;
    dst.xadj.alloc(static_cast<size_t>(n_new) + 1, s);
    dst.vw.alloc(std::max(n_new, 1), s);
    dst.adj.alloc(std::max<int64_t>(S_new, 1), s);
    dst.ew.alloc(std::max<int64_t>(S_new, 1), s);
    DBuf<int32_t> i32(3 * static_cast<size_t>(Mk) + 2, s);  // nnb[Mk+1] | onb[Mk] | nnb copy for slots
    DBuf<int64_t> i64(3 * static_cast<size_t>(Mk) + 2, s);  // nsb[Mk+1] | osb[Mk] | nsb copy for nodes
    HIPCHK(hipMemcpyAsync(i32.get(), nnb.data(), (Mk + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i32.get() + Mk + 1, onb.data(), Mk * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i64.get(), nsb.data(), (Mk + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i64.get() + Mk + 1, osb.data(), Mk * sizeof(int64_t), hipMemcpyHostToDevice, s));
    compact_nodes_kernel<<<grid_for(std::max(n_new, 1), 256), 256, 0, s>>>(
        n_new, Mk, i32.get(), i32.get() + Mk + 1, i64.get() + Mk + 1, i64.get(), src.xadj, src.vw, S_new,
        dst.xadj.get(), dst.vw.get());
    LAUNCHCHK();
    if (S_new > 0) {
        compact_slots_kernel<<<capped_grid_s(S_new), 256, 0, s>>>(S_new, Mk, i64.get(), i64.get() + Mk + 1,
                                                                  i32.get() + Mk + 1, i32.get(), src.adj, src.ew,
                                                                  dst.adj.get(), dst.ew.get());
        LAUNCHCHK();
    }
    HIPCHK(hipStreamSynchronize(s));
}

void pack_members_for_host(const DevGraph& src, const std::vector<int32_t>& onb, const std::vector<int64_t>& osb,
                           const std::vector<int32_t>& nnb, const std::vector<int64_t>& nsb, int64_t* x,
                           int32_t* adj, int32_t* vw, hipStream_t s) {
    const int32_t Mk = static_cast<int32_t>(onb.size());
    const int32_t n_new = nnb[Mk];
    const int64_t S_new = nsb[Mk];
    if (Mk == 0 || n_new == 0) return;
    DBuf<int32_t> i32(2 * static_cast<size_t>(Mk) + 1, s);  // nnb[Mk+1] | onb[Mk]
    DBuf<int64_t> i64(2 * static_cast<size_t>(Mk) + 1, s);  // nsb[Mk+1] | osb[Mk]
    HIPCHK(hipMemcpyAsync(i32.get(), nnb.data(), (Mk + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i32.get() + Mk + 1, onb.data(), Mk * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i64.get(), nsb.data(), (Mk + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(i64.get() + Mk + 1, osb.data(), Mk * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DBuf<int32_t> flag(n_new, s), rank(n_new, s), tot(1, s);
    pack_nodes_kernel<<<grid_for(n_new, 256), 256, 0, s>>>(n_new, Mk, i32.get(), i32.get() + Mk + 1,
                                                           i64.get() + Mk + 1, src.xadj, src.vw, x,
                                                           src.vw ? vw : nullptr, flag.get());
    LAUNCHCHK();
    if (S_new > 0) {
        exclusive_scan_i32(flag.get(), rank.get(), n_new, tot.get(), s);
        pack_slots_kernel<<<capped_grid_s(S_new), 256, 0, s>>>(S_new, Mk, i64.get(), i64.get() + Mk + 1,
                                                               i32.get() + Mk + 1, i32.get(), flag.get(), rank.get(),
                                                               src.adj, adj);
        LAUNCHCHK();
    }
    HIPCHK(hipStreamSynchronize(s));  // the host index vectors are read by the copies above
}

void unpack_members(const int32_t* src, int32_t n_new, int32_t Mk, const int32_t* dnb, int32_t* dst, hipStream_t s) {
    if (n_new == 0 || Mk == 0) return;
    unpack_members_kernel<<<grid_for(n_new, 256), 256, 0, s>>>(n_new, Mk, dnb, dnb + Mk + 1, src, dst);
    LAUNCHCHK();
}

void remap_members(int32_t n, const int32_t* gid, const std::vector<int32_t>& delta, int32_t* C, hipStream_t s) {
    if (n == 0) return;
    DBuf<int32_t> d(std::max<size_t>(delta.size(), 1), s);
    HIPCHK(hipMemcpyAsync(d.get(), delta.data(), delta.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    remap_members_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, d.get(), C);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------- inside blocks
//
// Clustering inside the blocks of a partition (Section 4.4, Miscellanea: iterated
// V-cycles) runs on the subgraph of the slots u->v with blk[u] == blk[v]:
// every cluster then stays inside one block.  Kept slots keep their order.
// Pass 1 counts the kept slots of each slot tile, pass 2 scans inside the
// tile, scatters, and writes the new offset of every row starting in it.

namespace {

__global__ void __launch_bounds__(kTileThreads) within_count_kernel(const int64_t* __restrict__ xadj,
                                                                    const int32_t* __restrict__ adj, int32_t n,
                                                                    int64_t S, const int32_t* __restrict__ blk,
                                                                    int32_t* __restrict__ tcnt, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    __shared__ int32_t s_w[kTileThreads / kWave];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
    tile_owners(xadj, trow, static_cast<int64_t>(blockIdx.x), i0, i1, owner);
    int32_t c = 0;
    for (int r = 0; r < kTilePer; ++r) {
        const int64_t i = i0 + r * kTileThreads + threadIdx.x;
        if (i < i1) c += blk[owner[i - i0]] == blk[adj[i]];
    }
    c = wave_sum(c);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kTileThreads / kWave; ++w) t += s_w[w];
        tcnt[blockIdx.x] = t;
    }
}

// first u in [0, n] with xadj[u] >= slot
__device__ int32_t first_row_from(const int64_t* __restrict__ xadj, int32_t n, int64_t slot) {
    int32_t lo = 0, hi = n;  // answer in [lo, hi]; xadj[n] = S > slot
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (xadj[mid] >= slot) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kTileThreads) within_scatter_kernel(
    const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, const int32_t* __restrict__ ew, int32_t n,
    int64_t S, const int32_t* __restrict__ blk, const int64_t* __restrict__ tbase, int64_t* __restrict__ oxadj,
    int32_t* __restrict__ oadj, int32_t* __restrict__ oew, const int32_t* __restrict__ trow) {
    __shared__ int32_t owner[kTile];
    __shared__ int32_t pre[kTile];
    __shared__ int32_t s_w[kTileThreads / kWave];
    __shared__ int32_t s_u0;
    const int tid = threadIdx.x;
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const int64_t i1 = i0 + kTile < S ? i0 + kTile : S;
    if (tid == 0) s_u0 = first_row_from(xadj, n, i0);
    tile_owners(xadj, trow, static_cast<int64_t>(blockIdx.x), i0, i1, owner);  // synchronises
    // kTilePer consecutive slots per thread
    uint32_t keep = 0;
    int32_t c = 0;
#pragma unroll
    for (int j = 0; j < kTilePer; ++j) {
        const int idx = tid * kTilePer + j;
        const int64_t i = i0 + idx;
        if (i < i1 && blk[owner[idx]] == blk[adj[i]]) {
            keep |= 1u << j;
            ++c;
        }
    }
    // exclusive prefix of c over the workgroup
    int32_t incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= o) incl += t;
    }
    if (lane_id() == kWave - 1) s_w[tid / kWave] = incl;
    __syncthreads();
    int32_t run = incl - c;
    for (int w = 0; w < tid / kWave; ++w) run += s_w[w];
    const int64_t base = tbase[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kTilePer; ++j) {
        const int idx = tid * kTilePer + j;
        pre[idx] = run;
        if (keep >> j & 1u) {
            const int64_t i = i0 + idx;
            oadj[base + run] = adj[i];
            if (oew) oew[base + run] = ew[i];
            ++run;
        }
    }
    __syncthreads();
    for (int64_t u = static_cast<int64_t>(s_u0) + tid; u < n && xadj[u] < i1; u += kTileThreads)
        oxadj[u] = base + pre[xadj[u] - i0];
}

__global__ void inherit_blocks_kernel(int32_t n, const int32_t* __restrict__ C, const int32_t* __restrict__ blk,
                                      int32_t* __restrict__ cblk) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n && C[v] >= 0) cblk[C[v]] = blk[v];
}

// rows starting at S (empty tail rows, and the end offset)
__global__ void within_tail_kernel(const int64_t* __restrict__ xadj, int32_t n, int64_t S,
                                   const int64_t* __restrict__ total, int64_t* __restrict__ oxadj) {
    const int64_t u = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (u <= n && xadj[u] >= S) oxadj[u] = *total;
}

}  // namespace

void within_blocks(const DevGraph& g, const int32_t* blk, OwnedDevGraph& out, hipStream_t s) {
    ProfScope ps("within_blocks", 24.0 * static_cast<double>(g.S), s);
    out.n = g.n;
    out.xadj.alloc(static_cast<size_t>(g.n) + 1, s);
    DBuf<int64_t> total(1, s);
    int64_t St = 0;
    const int64_t tiles = (g.S + kTile - 1) / kTile;
    DBuf<int64_t> tbase;
    DBuf<int32_t> trow;
    if (g.S > 0) {
        TileRows tr(g.xadj, g.n, g.S, s);
        trow = std::move(tr.trow);
        DBuf<int32_t> tcnt(tiles, s);
        tbase.alloc(tiles, s);
        within_count_kernel<<<static_cast<unsigned>(tiles), kTileThreads, 0, s>>>(g.xadj, g.adj, g.n, g.S, blk,
                                                                                  tcnt.get(), trow.get());
        LAUNCHCHK();
        exclusive_scan_i32_to_i64(tcnt.get(), tbase.get(), tiles, total.get(), s);
        HIPCHK(hipMemcpyAsync(&St, total.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        fill_i64(total.get(), 0, 1, s);
    }
    out.S = St;
    out.adj.alloc(std::max<int64_t>(St, 1), s);
    if (g.ew) out.ew.alloc(std::max<int64_t>(St, 1), s);
    if (g.S > 0) {
        within_scatter_kernel<<<static_cast<unsigned>(tiles), kTileThreads, 0, s>>>(
            g.xadj, g.adj, g.ew, g.n, g.S, blk, tbase.get(), out.xadj.get(), out.adj.get(),
            g.ew ? out.ew.get() : nullptr, trow.get());
        LAUNCHCHK();
    }
    within_tail_kernel<<<grid_for(static_cast<int64_t>(g.n) + 1, 256), 256, 0, s>>>(g.xadj, g.n, g.S, total.get(),
                                                                                    out.xadj.get());
    LAUNCHCHK();
}

void inherit_blocks(int32_t n, const int32_t* C, const int32_t* blk, int32_t* cblk, hipStream_t s) {
    if (n == 0) return;
    inherit_blocks_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, C, blk, cblk);
    LAUNCHCHK();
}

// ------------------------------------------------- degree-ordered rounds
//
// Sub-rounds by increasing degree (Section 3.1; Section 4.1, while
// coarsening): per graph, the nodes with at least one neighbour ranked by
// (degree, id) and cut into nsub equal consecutive groups; degree-0 nodes
// never move and go to sub-round 0.  One radix sort of (degree, id) keys;
// in a batch a second, stable sort by graph groups each graph's nodes in its
// own node range, in (degree, id) order.

namespace {

__global__ void degree_keys_kernel(int32_t n, const int64_t* __restrict__ xadj, int bn,
                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const uint64_t d = static_cast<uint64_t>(xadj[v + 1] - xadj[v]);
    keys[v] = (d << bn) | static_cast<uint32_t>(v);
    vals[v] = static_cast<uint32_t>(v);
}

__global__ void graph_keys_kernel(int32_t n, const uint32_t* __restrict__ vals, const int32_t* __restrict__ gid,
                                  uint64_t* __restrict__ keys) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) keys[i] = static_cast<uint32_t>(gid[vals[i]]);
}

// n0[g] = number of degree-0 nodes of graph g (they lead its segment)
__global__ void zero_run_kernel(int32_t n, const uint32_t* __restrict__ vals, const int64_t* __restrict__ xadj,
                                const int32_t* __restrict__ gid, const int32_t* __restrict__ gbase,
                                const int32_t* __restrict__ gcount, int32_t* __restrict__ n0) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t v = static_cast<int32_t>(vals[i]);
    if (xadj[v + 1] != xadj[v]) return;
    const int32_t g = gid ? gid[v] : 0;
    const int32_t end = gbase[g] + gcount[g];
    bool last = i + 1 == end;
    if (!last) {
        const int32_t u = static_cast<int32_t>(vals[i + 1]);
        last = xadj[u + 1] != xadj[u];
    }
    if (last) n0[g] = i + 1 - gbase[g];
}

__global__ void degree_color_kernel(int32_t n, const uint32_t* __restrict__ vals, const int64_t* __restrict__ xadj,
                                    const int32_t* __restrict__ gid, const int32_t* __restrict__ gbase,
                                    const int32_t* __restrict__ gcount, const int32_t* __restrict__ n0,
                                    int32_t nsub, int32_t* __restrict__ color) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t v = static_cast<int32_t>(vals[i]);
    if (xadj[v + 1] == xadj[v]) {
        color[v] = 0;
        return;
    }
    const int32_t g = gid ? gid[v] : 0;
    const int64_t r = static_cast<int64_t>(i) - gbase[g] - n0[g];
    const int64_t cnt = static_cast<int64_t>(gcount[g]) - n0[g];
    color[v] = static_cast<int32_t>(r * nsub / cnt);
}

}  // namespace

void degree_colors(const DevGraph& g, int32_t G, const int32_t* gid, const int32_t* gbase, const int32_t* gcount,
                   int32_t nsub, int32_t* color, hipStream_t s) {
    const int32_t n = g.n;
    if (n == 0) return;
    ProfScope ps("degree_order", 0, s);
    const int bn = std::max(1, bits_for(static_cast<uint64_t>(n - 1)));
    const int bd = std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(g.S, 1))));
    if (bn + bd > 64) fail(-1, "graph too large for degree-ordered sub-rounds");
    DBuf<uint64_t> keys(n, s), ktmp(n, s);
    DBuf<uint32_t> vals(n, s), vtmp(n, s);
    degree_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g.xadj, bn, keys.get(), vals.get());
    LAUNCHCHK();
    RadixScratch rs;
    radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), n, 0, bn + bd, rs, s);
    DBuf<int32_t> one_base, one_count;
    if (gid) {
        graph_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, vals.get(), gid, keys.get());
        LAUNCHCHK();
        radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), n, 0,
                         std::max(1, bits_for(static_cast<uint64_t>(std::max(G - 1, 1)))), rs, s);
    } else {
        G = 1;
        one_base.alloc(1, s);
        one_count.alloc(1, s);
        fill_i32(one_base.get(), 0, 1, s);
        fill_i32(one_count.get(), n, 1, s);
        gbase = one_base.get();
        gcount = one_count.get();
    }
    DBuf<int32_t> n0(std::max(G, 1), s);
    fill_i32(n0.get(), 0, std::max(G, 1), s);
    zero_run_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, vals.get(), g.xadj, gid, gbase, gcount, n0.get());
    LAUNCHCHK();
    degree_color_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, vals.get(), g.xadj, gid, gbase, gcount, n0.get(), nsub,
                                                         color);
    LAUNCHCHK();
}

// ------------------------------------------------------- core renumbering

namespace {

__global__ void has_degree_kernel(int32_t n, const int64_t* __restrict__ xadj, int32_t* __restrict__ flag) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) flag[v] = xadj[v + 1] > xadj[v] ? 1 : 0;
}

__global__ void core_map_kernel(int64_t S, const int32_t* __restrict__ adj, const int32_t* __restrict__ flag,
                                const int32_t* __restrict__ rank, int32_t* __restrict__ out) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e < S) out[e] = flag[adj[e]] ? rank[adj[e]] : -1;  // -1: a neighbour without neighbours
}

}  // namespace

void core_ranks(const DevGraph& g, int32_t* out, hipStream_t s) {
    if (g.n == 0 || g.S == 0) return;
    DBuf<int32_t> flag(g.n, s), rank(g.n, s), tot(1, s);
    has_degree_kernel<<<grid_for(g.n, 256), 256, 0, s>>>(g.n, g.xadj, flag.get());
    LAUNCHCHK();
    exclusive_scan_i32(flag.get(), rank.get(), g.n, tot.get(), s);
    core_map_kernel<<<grid_for(g.S, 256), 256, 0, s>>>(g.S, g.adj, flag.get(), rank.get(), out);
    LAUNCHCHK();
}

// --------------------------------------------- device initial partition

namespace {

// positive-degree nodes: hash key and id at their rank
__global__ void seed_keys_kernel(int32_t n, const int64_t* __restrict__ xadj, const int32_t* __restrict__ rank,
                                 uint64_t prefix, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n || xadj[v + 1] == xadj[v]) return;
    keys[rank[v]] = mix64(prefix ^ static_cast<uint64_t>(static_cast<uint32_t>(v)));
    vals[rank[v]] = static_cast<uint32_t>(v);
}

__global__ void place_seeds_kernel(int32_t count, const uint32_t* __restrict__ vals, int32_t* __restrict__ part) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) part[vals[i]] = i;
}

__global__ void add_to_kernel(int32_t* __restrict__ w, int32_t add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) w[0] += add;
}

__global__ void pool_weight_kernel(int32_t n, const int32_t* __restrict__ part, int32_t pool,
                                   const int32_t* __restrict__ vw, int32_t* __restrict__ pw) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v < n) pw[v] = part[v] == pool ? (vw ? vw[v] : 1) : 0;
}

// pool node with exclusive prefix weight P: first block whose cumulative room exceeds P
__global__ void deal_pool_kernel(int32_t n, int32_t k, const int64_t* __restrict__ P,
                                 const int64_t* __restrict__ cum, int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n || part[v] != k) return;
    const int64_t p = P[v];
    int32_t lo = 0, hi = k;  // first b in [0, k) with cum[b] > p, k if none
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > p) hi = mid;
        else lo = mid + 1;
    }
    part[v] = lo < k ? lo : k - 1;
}

}  // namespace

LPResult device_initial_partition(const DevGraph& g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed, int32_t level,
                                  int32_t nsub, int32_t rounds, const LPTuning& tune, int32_t* part, hipStream_t s) {
    constexpr int64_t kBig = int64_t(1) << 30;  // pool weight offset: never eligible, always overloaded
    const int32_t n = g.n;
    LPResult res;
    if (n == 0) return res;
    int64_t cV = 0, cmax = 0;
    node_weight_stats(g, &cV, &cmax, s);
    if (Lmax >= kBig || cV >= kBig) fail(-1, "device initial partition needs Lmax and c(V) below 2^30");
    DBuf<int32_t> flag(n, s), rank(n, s), tot(1, s);
    has_degree_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g.xadj, flag.get());
    LAUNCHCHK();
    exclusive_scan_i32(flag.get(), rank.get(), n, tot.get(), s);
    int32_t npos = 0;
    HIPCHK(hipMemcpyAsync(&npos, tot.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    fill_i32(part, k, n, s);  // everything starts in the pool
    if (npos > 0) {
        ProfScope ps("initial_seeds", 0, s);
        DBuf<uint64_t> keys(npos, s), ktmp(npos, s);
        DBuf<uint32_t> vals(npos, s), vtmp(npos, s);
        const uint64_t prefix = hash_prefix({seed, 5, static_cast<uint64_t>(static_cast<uint32_t>(level))});
        seed_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g.xadj, rank.get(), prefix, keys.get(), vals.get());
        LAUNCHCHK();
        RadixScratch rs;
        radix_sort_pairs(keys.get(), vals.get(), ktmp.get(), vtmp.get(), npos, 0, 64, rs, s);
        const int32_t ns = std::min(k, npos);
        place_seeds_kernel<<<grid_for(ns, 256), 256, 0, s>>>(ns, vals.get(), part);
        LAUNCHCHK();
    }
    DBuf<int32_t> w(static_cast<size_t>(k) + 1, s);
    label_weights(g, part, w.get(), k + 1, s);
    add_to_kernel<<<1, 64, 0, s>>>(w.get() + k, static_cast<int32_t>(kBig));
    LAUNCHCHK();
    res = run_lp(g, kInitial, level, seed, nsub, rounds, Lmax, part, w.get(), k + 1, nullptr, tune, s);
    // the pool fills the blocks' remaining room in block order
    std::vector<int32_t> hw(static_cast<size_t>(k));
    HIPCHK(hipMemcpyAsync(hw.data(), w.get(), k * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int64_t> cum(static_cast<size_t>(k));
    int64_t run = 0;
    for (int32_t b = 0; b < k; ++b) {
        run += hw[b] < T ? T - hw[b] : 0;
        cum[b] = run;
    }
    DBuf<int64_t> dcum(k, s), P(n, s), ptot(1, s);
    HIPCHK(hipMemcpyAsync(dcum.get(), cum.data(), k * sizeof(int64_t), hipMemcpyHostToDevice, s));
    pool_weight_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, part, k, g.vw, flag.get());
    LAUNCHCHK();
    exclusive_scan_i32_to_i64(flag.get(), P.get(), n, ptot.get(), s);
    deal_pool_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, k, P.get(), dcum.get(), part);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));  // cum is read by the copy above
    return res;
}

void project_kept(int32_t n, const int32_t* C, const int32_t* coarse_part, int32_t* part, hipStream_t s) {
    if (n == 0) return;
    project_kept_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, C, coarse_part, part);
    LAUNCHCHK();
}

void shift_by_graph(int32_t n, const int32_t* gid, const int32_t* add, int32_t sign, int32_t* part, hipStream_t s) {
    if (n == 0) return;
    shift_by_graph_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, gid, add, sign, part);
    LAUNCHCHK();
}

}  // namespace sclap
