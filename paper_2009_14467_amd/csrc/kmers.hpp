// k-mer tables of a sequence set (see kmers.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pastis {

constexpr uint64_t kInvalidKmer = 0xFFFFFFFFull;

// Device arrays; capacities: n_res entries for postings/rows and distinct
// k-mers, n + 1 for row bounds, 24^k for kmap.  counts[0] = nnz,
// counts[1] = number of distinct k-mers, counts[2] = nnz again (row scan).
struct KmerTables {
    uint32_t *counts;  // 4 entries
    uint32_t *post_seq;
    uint16_t *post_pos;
    uint32_t *post_u;
    uint32_t *uk_id;
    uint32_t *uk_start;  // nu + 1
    uint32_t *row_cnt;   // n + 1
    uint32_t *row_start; // n + 1
    uint32_t *row_u;
    uint16_t *row_pos;
    int32_t *kmap;
};

size_t kmers_temp_bytes(int64_t n_res, int64_t n);
int64_t kmap_entries(int k);
hipError_t build_kmers(const uint8_t *codes, const int64_t *offsets, int64_t n, int64_t n_res, int k, bool want_kmap,
                       KmerTables &kt, void *temp, hipStream_t s);

}  // namespace pastis
