// Device primitives (see prim.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pastis {

template <typename T>
hipError_t fill(T *p, int64_t n, T v, hipStream_t s);
hipError_t iota(uint32_t *p, int64_t n, hipStream_t s);

// Temporary bytes for exclusive_scan over n elements.
size_t scan_temp_bytes(int64_t n);
// out[i] = sum of in[0..i-1]; *total (device, may be null) = sum of all.
template <typename TIn, typename TOut>
hipError_t exclusive_scan(const TIn *in, int64_t n, TOut *out, TOut *total, void *temp, hipStream_t s);

// Temporary bytes for radix_sort over n elements.
size_t radix_temp_bytes(int64_t n);
// Stable LSD radix sort by the low `bits` bits of keys (8 bits per pass),
// carrying vals.  Buffers ping-pong; *result_in_alt tells where the sorted
// data ended up.
hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, int64_t n, int bits,
                      void *temp, hipStream_t s, bool *result_in_alt);

}  // namespace pastis
