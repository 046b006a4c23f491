// Device primitives written for gfx950 (wave64): fills, prefix scans and a
// stable LSD radix sort.  Host-side launchers enqueue on the given stream.
#pragma once

#include "common.hpp"

namespace sclap {

void fill_i32(int32_t* p, int32_t value, int64_t count, hipStream_t s);
void fill_i64(int64_t* p, int64_t value, int64_t count, hipStream_t s);
void fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
void fill_u8(uint8_t* p, uint8_t value, int64_t count, hipStream_t s);
void iota_u32(uint32_t* p, int64_t count, hipStream_t s);

// Exclusive prefix sum of in[0..count) into out[0..count); when total is not
// null, *total (device) receives the sum of all inputs.  in and out may alias.
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t count, int64_t* total, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* total, hipStream_t s);
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total, hipStream_t s);
// Inclusive prefix sum of int64 values.
void inclusive_scan_i64(const int64_t* in, int64_t* out, int64_t count, hipStream_t s);
// Inclusive prefix max of int32 values.
void inclusive_max_i32(const int32_t* in, int32_t* out, int64_t count, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key bits [begin_bit,
// end_bit).  values may be null.  The sorted result ends in keys/values
// (the *_tmp buffers, of the same size, are scratch).  count <= 2^32 - 2.
struct RadixScratch {
    DBuf<uint32_t> counts;  // per (digit, tile)
};
void radix_sort_pairs(uint64_t* keys, uint32_t* values, uint64_t* keys_tmp, uint32_t* values_tmp, int64_t count,
                      int begin_bit, int end_bit, RadixScratch& scratch, hipStream_t s);

}  // namespace sclap
