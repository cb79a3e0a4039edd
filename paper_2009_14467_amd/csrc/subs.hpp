// Substitute k-mer rows (see subs.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pastis {

constexpr int kMaxK = 8;

int s_rows_threads();
// S rows of the nu (device count) distinct k-mers (ids ascending in uk_id):
// (m + 1) slots per row of posting-group heads s_u (uk_start[v] + v for
// k-mer v) / distances s_d; s_cnt = used slots.  A substitute's head comes
// from kmap (dense, k <= 6) or, when kmap is null, from a binary search of
// uk_id.  tmp_ids / tmp_d hold m entries for each of s_rows_threads() threads.
hipError_t launch_s_rows(const uint64_t *uk_id, const uint32_t *nu, const uint32_t *uk_start, const int32_t *kmap,
                         const int8_t *blosum25, int k, int m, int alpha, uint32_t *s_u, int8_t *s_d, uint32_t *s_cnt,
                         uint64_t *tmp_ids, int8_t *tmp_d, hipStream_t s);
// m nearest substitutes of n given k-mer ids: out_ids / out_d [n][m], out_n[n].
hipError_t launch_nearest_ids(const uint64_t *kid, int64_t n, const int8_t *blosum25, int k, int m, int alpha,
                              uint64_t *out_ids, int8_t *out_d, int32_t *out_n, hipStream_t s);

}  // namespace pastis
