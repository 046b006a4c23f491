// Fills, prefix scans and a stable LSD radix sort for gfx950 (wave64).
#include "primitives.hpp"

namespace sclap {

// ------------------------------------------------------------------ fills

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, T value, int64_t count) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

__global__ void iota_kernel(uint32_t* __restrict__ p, int64_t count) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = static_cast<uint32_t>(i);
}

static unsigned fill_grid(int64_t count) {
    int64_t g = (count + 255) / 256;
    if (g > 8192) g = 8192;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

template <typename T>
static void fill_any(T* p, T value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    fill_kernel<T><<<fill_grid(count), 256, 0, s>>>(p, value, count);
    LAUNCHCHK();
}

void fill_i32(int32_t* p, int32_t v, int64_t c, hipStream_t s) { fill_any(p, v, c, s); }
void fill_i64(int64_t* p, int64_t v, int64_t c, hipStream_t s) { fill_any(p, v, c, s); }
void fill_u32(uint32_t* p, uint32_t v, int64_t c, hipStream_t s) { fill_any(p, v, c, s); }
void fill_u8(uint8_t* p, uint8_t v, int64_t c, hipStream_t s) { fill_any(p, v, c, s); }
void iota_u32(uint32_t* p, int64_t c, hipStream_t s) {
    if (c <= 0) return;
    iota_kernel<<<fill_grid(c), 256, 0, s>>>(p, c);
    LAUNCHCHK();
}

// ------------------------------------------------------------------ scans

struct OpAdd {
    template <typename T> __device__ static T identity() { return T(0); }
    template <typename T> __device__ static T apply(T a, T b) { return a + b; }
};
struct OpMax {
    template <typename T> __device__ static T identity() { return T(-2147483647 - 1); }
    template <typename T> __device__ static T apply(T a, T b) { return a > b ? a : b; }
};

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan across the 256 threads of a block; returns the inclusive
// prefix of this thread and sets block_total.
template <typename T, typename Op>
__device__ T block_scan_inclusive(T v, T& block_total) {
    __shared__ T wave_tot[kScanThreads / kWave];
    const int lane = lane_id();
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v = Op::apply(u, v);
    }
    if (lane == kWave - 1) wave_tot[wid] = v;
    __syncthreads();
    T pre = Op::template identity<T>();
    T tot = Op::template identity<T>();
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) pre = Op::apply(pre, wave_tot[w]);
        tot = Op::apply(tot, wave_tot[w]);
    }
    __syncthreads();
    block_total = tot;
    return Op::apply(pre, v);
}

template <typename Tin, typename Tout, typename Op>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const Tin* __restrict__ in, int64_t count,
                                                                   Tout* __restrict__ partial) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    Tout acc = Op::template identity<Tout>();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < count) acc = Op::apply(acc, static_cast<Tout>(in[base + j]));
    Tout tot;
    block_scan_inclusive<Tout, Op>(acc, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// carry: per-block exclusive offsets (null for a single block).
template <typename Tin, typename Tout, typename Op, bool kInclusive>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const Tin* in, Tout* out, int64_t count,
                                                                 const Tout* __restrict__ carry, Tout* total) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    Tout vals[kScanItems];
    Tout acc = Op::template identity<Tout>();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        vals[j] = (base + j < count) ? static_cast<Tout>(in[base + j]) : Op::template identity<Tout>();
        acc = Op::apply(acc, vals[j]);
    }
    Tout tot;
    const Tout incl = block_scan_inclusive<Tout, Op>(acc, tot);
    // exclusive prefix of this thread = inclusive prefix of the previous thread
    Tout a = carry ? carry[blockIdx.x] : Op::template identity<Tout>();
    {
        __shared__ Tout wave_last[kScanThreads / kWave];
        const Tout prev = __shfl_up(incl, 1, 64);
        const int lane = lane_id();
        const int wid = threadIdx.x / kWave;
        if (lane == kWave - 1) wave_last[wid] = incl;
        __syncthreads();
        if (lane > 0) a = Op::apply(a, prev);
        else if (wid > 0) a = Op::apply(a, wave_last[wid - 1]);
    }
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < count) {
            if (kInclusive) {
                a = Op::apply(a, vals[j]);
                out[base + j] = a;
            } else {
                out[base + j] = a;
                a = Op::apply(a, vals[j]);
            }
        }
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        Tout c = carry ? carry[blockIdx.x] : Op::template identity<Tout>();
        *total = Op::apply(c, tot);
    }
}

template <typename Tin, typename Tout, typename Op, bool kInclusive>
static void scan_impl(const Tin* in, Tout* out, int64_t count, Tout* total, hipStream_t s) {
    if (count <= 0) {
        if (total) {
            Tout zero = Tout(0);
            HIPCHK(hipMemcpyAsync(total, &zero, sizeof(Tout), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        return;
    }
    const int64_t nblocks = (count + kScanTile - 1) / kScanTile;
    if (nblocks == 1) {
        scan_down_kernel<Tin, Tout, Op, kInclusive><<<1, kScanThreads, 0, s>>>(in, out, count, nullptr, total);
        LAUNCHCHK();
        return;
    }
    DBuf<Tout> partial(static_cast<size_t>(nblocks), s);
    scan_reduce_kernel<Tin, Tout, Op><<<static_cast<unsigned>(nblocks), kScanThreads, 0, s>>>(in, count, partial.get());
    LAUNCHCHK();
    scan_impl<Tout, Tout, Op, false>(partial.get(), partial.get(), nblocks, nullptr, s);
    scan_down_kernel<Tin, Tout, Op, kInclusive><<<static_cast<unsigned>(nblocks), kScanThreads, 0, s>>>(
        in, out, count, partial.get(), total);
    LAUNCHCHK();
}

void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t count, int64_t* total, hipStream_t s) {
    scan_impl<int32_t, int64_t, OpAdd, false>(in, out, count, total, s);
}
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* total, hipStream_t s) {
    scan_impl<int32_t, int32_t, OpAdd, false>(in, out, count, total, s);
}
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total, hipStream_t s) {
    scan_impl<uint32_t, uint32_t, OpAdd, false>(in, out, count, total, s);
}
void inclusive_scan_i64(const int64_t* in, int64_t* out, int64_t count, hipStream_t s) {
    scan_impl<int64_t, int64_t, OpAdd, true>(in, out, count, nullptr, s);
}
void inclusive_max_i32(const int32_t* in, int32_t* out, int64_t count, hipStream_t s) {
    scan_impl<int32_t, int32_t, OpMax, true>(in, out, count, nullptr, s);
}

// ------------------------------------------------------------- radix sort

constexpr int kRadixBits = 8;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixWaves = kRadixThreads / kWave;
constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;

// counts[d * ntiles + tile] = number of keys of digit d in the tile.
__global__ void __launch_bounds__(kRadixThreads) radix_hist_kernel(const uint64_t* __restrict__ keys, int64_t count,
                                                                   int shift, int64_t ntiles,
                                                                   uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[kRadixDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kRadixTile;
#pragma unroll 4
    for (int r = 0; r < kRadixRounds; ++r) {
        int64_t i = base + r * kRadixThreads + threadIdx.x;
        if (i < count) atomicAdd(&h[(keys[i] >> shift) & (kRadixDigits - 1)], 1u);
    }
    __syncthreads();
    counts[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items keep their input order inside each digit.
__global__ void __launch_bounds__(kRadixThreads) radix_scatter_kernel(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint64_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t count, int shift, int64_t ntiles, const uint32_t* __restrict__ offsets) {
    __shared__ uint32_t base_off[kRadixDigits];
    __shared__ uint32_t wave_cnt[kRadixWaves][kRadixDigits];
    __shared__ uint32_t wave_off[kRadixWaves][kRadixDigits];
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    base_off[tid] = offsets[static_cast<int64_t>(tid) * ntiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kRadixWaves; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();
    const int64_t tile_base = static_cast<int64_t>(blockIdx.x) * kRadixTile;
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = tile_base + r * kRadixThreads + tid;
        const bool valid = i < count;
        uint64_t key = valid ? keys_in[i] : 0;
        uint32_t val = (valid && vals_in) ? vals_in[i] : 0;
        const uint32_t d = static_cast<uint32_t>((key >> shift) & (kRadixDigits - 1));
        // lanes of this wave with the same digit
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            match &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = static_cast<uint32_t>(__popcll(match & lt));
        if (valid && rank == 0) wave_cnt[wid][d] = static_cast<uint32_t>(__popcll(match));
        __syncthreads();
        {
            // thread tid owns digit tid: prefix over waves
            uint32_t run = base_off[tid];
#pragma unroll
            for (int w = 0; w < kRadixWaves; ++w) {
                wave_off[w][tid] = run;
                run += wave_cnt[w][tid];
                wave_cnt[w][tid] = 0;
            }
            base_off[tid] = run;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = wave_off[wid][d] + rank;
            keys_out[pos] = key;
            if (vals_in) vals_out[pos] = val;
        }
    }
}

void radix_sort_pairs(uint64_t* keys, uint32_t* values, uint64_t* keys_tmp, uint32_t* values_tmp, int64_t count,
                      int begin_bit, int end_bit, RadixScratch& scratch, hipStream_t s) {
    if (count <= 1 || end_bit <= begin_bit) return;
    if (count > 0xFFFFFFFELL) fail(-1, "radix sort: too many items");
    const int64_t ntiles = (count + kRadixTile - 1) / kRadixTile;
    scratch.counts.reserve(static_cast<size_t>(ntiles) * kRadixDigits, s);
    uint64_t* kin = keys;
    uint32_t* vin = values;
    uint64_t* kout = keys_tmp;
    uint32_t* vout = values_tmp;
    for (int shift = begin_bit; shift < end_bit; shift += kRadixBits) {
        radix_hist_kernel<<<static_cast<unsigned>(ntiles), kRadixThreads, 0, s>>>(kin, count, shift, ntiles,
                                                                                   scratch.counts.get());
        LAUNCHCHK();
        exclusive_scan_u32(scratch.counts.get(), scratch.counts.get(), ntiles * kRadixDigits, nullptr, s);
        radix_scatter_kernel<<<static_cast<unsigned>(ntiles), kRadixThreads, 0, s>>>(
            kin, vin, kout, vout, count, shift, ntiles, scratch.counts.get());
        LAUNCHCHK();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (kin != keys) {
        HIPCHK(hipMemcpyAsync(keys, kin, static_cast<size_t>(count) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        if (values)
            HIPCHK(hipMemcpyAsync(values, vin, static_cast<size_t>(count) * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                  s));
    }
}

}  // namespace sclap
