// Candidate discovery stage (see spgemm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kmers.hpp"

namespace pastis {

// Candidate pairs lo < hi sorted by (lo, hi), SoA on the device.
struct Candidates {
    uint32_t *lo, *hi, *count, *seed1, *seed2;
};

struct BinBufs {
    int *counts, *starts, *cursor, *idx;
};

int key_bits(int64_t n);

// (A S) rows: ub = per-row upper bound, as_start = its exclusive scan
// (n + 1 entries), as_len = actual row lengths.
struct AsArgs {
    const KmerTables *kt;
    const uint32_t *s_u;
    const int8_t *s_d;
    const uint32_t *s_cnt;
    int W;
    int64_t n;
    uint32_t *ub;
    uint64_t *as_start;
    uint32_t *as_len;
    uint32_t *as_s, *as_dp;
    int8_t *bin_of;
    BinBufs bins;
    unsigned long long *max_ub;
    void *scan_temp;
    uint32_t *gtables;
    int global_blocks;
};
hipError_t as_stage(const AsArgs &a, hipStream_t s);         // bounds, offsets, bins
hipError_t as_run(const AsArgs &a, uint32_t gcap, hipStream_t s);  // fill the rows

struct SpgemmArgs {
    const KmerTables *kt;
    int exact;
    const uint32_t *row_start32;
    const uint64_t *row_start64;
    const uint32_t *row_len;
    const uint32_t *ent_s;
    const uint32_t *ent_len;  // posting length of each entry, or null (read from its header)
    const uint16_t *ent_pos16;
    const uint32_t *ent_dp;
    int64_t n;
    // row block: the pairs (lo, hi) with blk_lo <= lo < blk_hi ([0, n) for all)
    uint32_t blk_lo, blk_hi;
    int ck;
    uint64_t *work;
    int8_t *bin_of;
    BinBufs bins;
    unsigned long long *max_big;
    unsigned long long *products;  // postings visited by one pass over the rows
    uint32_t *big_rows, *n_big;  // n_big: 2 counters
    // the postings of A^T as headed records (nnz + distinct k-mers of them);
    // ent_s holds the header index of each entry's posting group
    uint2 *post_rec;
    int64_t nnz;
    // directional entries
    unsigned long long *d_count;  // directional entries requested (may exceed cap)
    uint32_t *d_overflow;
    uint64_t *d_key;
    uint32_t *d_cnt, *d_s1, *d_s2, *d_dir;
    uint32_t cap;
    int nbits;
    unsigned long long *gtables;
    uint32_t *gcand;
    int global_blocks;
    // per-block product stages of the LDS kernels (spgemm_stage_entries())
    uint2 *stage;
};
size_t spgemm_stage_entries();
hipError_t spgemm_plan(const SpgemmArgs &a, hipStream_t s);
hipError_t spgemm_run(const SpgemmArgs &a, uint32_t gcap, hipStream_t s);

struct SymArgs {
    int64_t n_dir;
    const uint32_t *d_ndir;
    uint64_t *key, *key_alt;
    uint32_t *perm, *perm_alt;
    const uint32_t *cnt, *s1, *s2, *dir;
    uint8_t *flag;
    uint32_t *pick, *opos;
    uint32_t *d_ncand;
    int nbits;
    void *sort_temp;
    Candidates out;
};
hipError_t symmetrise(const SymArgs &a, hipStream_t s);

}  // namespace pastis
