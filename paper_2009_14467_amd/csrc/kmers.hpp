// k-mer tables of a sequence set (see kmers.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pastis {

// k-mers of up to this length index the dense id -> distinct-k-mer map
// (24^6 entries, 764 MB); longer ones are found by binary search over the
// sorted distinct ids (the map would need 24^7 = 4.6e9 entries and more)
constexpr int kDenseMapMaxK = 6;

// Device arrays; capacities: n_res entries for postings/rows and distinct
// k-mers, n + 1 for row bounds, 24^k for kmap.  The product stage reads the
// postings as headed records: group u occupies records head(u) ..
// head(u) + len(u), a header (len(u), u) followed by its (sequence,
// position) records, with head(u) = uk_start[u] + u; a row entry or a
// substitute then names its posting list by head(u), and one line holds both
// the list's length and its first records.  counts[0] = nnz,
// counts[1] = number of distinct k-mers.
// Distinct ids are ascending in uk_id.
struct KmerTables {
    uint32_t *counts;  // 4 entries
    uint32_t *post_seq;
    uint16_t *post_pos;
    uint32_t *post_u;
    uint64_t *uk_id;     // radix-24 ids, up to 24^8 for k = 8
    uint32_t *uk_start;  // nu + 1
    uint32_t *row_start; // n + 1
    uint32_t *row_u;
    uint16_t *row_pos;
    // optional (may be null): per row entry, the index of its k-mer's group
    // header in the headed posting records, head(u) = uk_start[u] + u
    uint32_t *row_h;
    // optional, set with row_h: per row entry, the length of that group
    // (uk_start[u + 1] - uk_start[u]), so the row scan and the product read
    // it in row order instead of from the scattered group header
    uint32_t *row_len;
    int32_t *kmap;  // id -> head(u) of the distinct k-mer u, or -1
};

size_t kmers_temp_bytes(int64_t n_res, int64_t n);
int64_t kmap_entries(int k);
hipError_t build_kmers(const uint8_t *codes, const int64_t *offsets, int64_t n, int64_t n_res, int k, bool want_kmap,
                       KmerTables &kt, void *temp, hipStream_t s);

}  // namespace pastis
