// Internal runtime pieces shared by the gfx950 kernels and the host driver:
// error handling, stream-ordered device buffers, the colour / tie-break hash,
// and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace sclap {

// ---------------------------------------------------------------- errors

struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

[[noreturn]] void fail(int status, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHK(x) ::sclap::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCHCHK() ::sclap::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ------------------------------------------------------------ device memory

// Stream-ordered device memory through a block cache (alloc.hip): a freed
// block is reused by later allocations of its size class on the same stream.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, size_t bytes, hipStream_t s);
// Returns the cached blocks of stream s (or of every stream of the current
// device) to the device's memory pool.
void release_cached(hipStream_t s, bool all_streams);

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t count = 0;
    hipStream_t s = nullptr;
    DBuf() = default;
    DBuf(size_t n, hipStream_t st) { alloc(n, st); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), count(o.count), s(o.s) { o.p = nullptr; o.count = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; count = o.count; s = o.s; o.p = nullptr; o.count = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t n, hipStream_t st) {
        release();
        s = st;
        count = n;
        p = n ? static_cast<T*>(dev_alloc(n * sizeof(T), st)) : nullptr;
    }
    // grow-only reallocation (contents not preserved)
    void reserve(size_t n, hipStream_t st) {
        if (n > count || p == nullptr) alloc(n > 0 ? n : 1, st);
    }
    void release() {
        if (p) dev_free(p, count * sizeof(T), s);
        p = nullptr;
        count = 0;
    }
    T* get() const { return p; }
};

// ------------------------------------------------------------------ hash

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

// SplitMix64 output function of z + gamma (Steele, Lea, Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Chained hash H(w0..wj) = mix(...mix(mix(w0) ^ w1)... ^ wj).  The library
// hashes a fixed prefix on the host and finishes on the device with one mix:
//   colour(v) = mix(H(seed, 1, level, phase) ^ v) mod nsub
//   tie(x)    = mix(H(seed, 2, level, phase, round) ^ x)
inline uint64_t hash_prefix(std::initializer_list<uint64_t> words) {
    uint64_t h = 0;
    bool first = true;
    for (uint64_t w : words) {
        h = first ? mix64(w) : mix64(h ^ w);
        first = false;
    }
    return h;
}

// 32-bit slot hash for LDS / global open-addressing tables (not semantic).
__device__ __forceinline__ uint32_t slot_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// --------------------------------------------------------------- wave64

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ULL : (~0ULL >> (64 - l));
}

// Orders LDS accesses of the lanes of one wave (wave-private LDS regions).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl(static_cast<uint32_t>(v), src, 64);
    uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src, 64);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), o, 64);
        uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), o, 64);
        uint64_t u = (static_cast<uint64_t>(hi) << 32) | lo;
        v = u < v ? u : v;
    }
    return v;
}

inline int bits_for(uint64_t maxval) {  // bits needed to hold values 0..maxval
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

inline unsigned grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

// Block-wide append for 256-thread workgroups with one atomic per workgroup:
// c items per thread; returns the position of this thread's first item in
// *counter's sequence (the thread's items are consecutive, the order across
// workgroups unspecified).
__device__ __forceinline__ uint32_t block_append_count(uint32_t c, uint32_t* counter) {
    __shared__ uint32_t s_cnt[4];
    __shared__ uint32_t s_base;
    const int wid = threadIdx.x >> 6;
    const int lane = lane_id();
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_cnt[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < 4; ++w) {
            const uint32_t t = s_cnt[w];
            s_cnt[w] = run;
            run += t;
        }
        s_base = run ? atomicAdd(counter, run) : 0;
    }
    __syncthreads();
    const uint32_t idx = s_base + s_cnt[wid] + incl - c;
    __syncthreads();
    return idx;
}

}  // namespace sclap
