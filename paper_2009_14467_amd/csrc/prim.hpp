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

// Workgroups go to the chip's eight XCDs round-robin by id, and each XCD has
// its own L2.  Items [0, n) are split into eight contiguous segments, one per
// XCD, and a unit (a block, or one of `per` waves of a block) walks its XCD's
// segment with the stride of that XCD's units: items processed at the same
// time on one XCD are then neighbours in the caller's order, so where that
// order groups related rows (sequences sorted or clustered by similarity),
// the posting lists they share are served by one L2.  A grid of fewer than
// eight blocks uses one segment per block, so any grid covers every item
// exactly once.
struct XcdWalk {
    int64_t first, end, step;
};
__device__ __forceinline__ XcdWalk xcd_walk(int64_t n, int per = 1, int sub = 0) {
    const int segs = gridDim.x < 8u ? (int)gridDim.x : 8;
    const int x = (int)(blockIdx.x % segs);
    const int64_t blocks_x = ((int64_t)gridDim.x - x + segs - 1) / segs;
    const int64_t seg = (n + segs - 1) / segs;
    const int64_t b = x * seg, e = b + seg < n ? b + seg : n;
    return {b + (int64_t)(blockIdx.x / segs) * per + sub, e, blocks_x * per};
}

}  // namespace pastis
