// Internal declarations of the gfx950 library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pastis.h"
#include "mlp.hpp"

namespace pastis {

// Residue codes 0..23 follow the paper's numbering (Section V-B):
// A R N D C Q E G H I L K M F P S T W Y V B Z X *.
constexpr int kAlpha = 24;
// Column code used for DP cells outside the target sequence: every score
// against it is kPadScore, so such cells never raise a running maximum.
constexpr int kPadCode = 24;
constexpr int kPadScore = -10000;
constexpr uint32_t kNoSeed = 0xFFFFFFFFu;
constexpr int kMaxLen = 65535;

// BLOSUM62 in the residue order above (host copy; uploaded at context creation).
extern const int8_t kBlosum62[kAlpha * kAlpha];

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Scoring {
    int gap_open, gap_extend, xdrop, id_pct, cov_pct;
    // pairs with 100 * score >= direct_pct * la skip the start-bound pass
    // (likely to pass the cut); exact either way, only the cost moves
    int direct_pct = 50;
};

// Oriented pair descriptor: rows a = shorter sequence (first on a tie).
struct PairDesc {
    int64_t a_off, b_off;
    int32_t la, lb;
    int32_t pa1, pb1, pa2, pb2;  // oriented seeds (-1 when absent)
    int32_t swapped;
    int32_t a_seq;  // index of sequence a
};

// Stage timer: HIP events recorded on the call's stream, read after a sync.
enum Stage { kStEncode = 0, kStKmers, kStSubs, kStSpgemm, kStSched, kStAlign1, kStAlign2, kStFilter, kStLearned, kNumStages };

#define PASTIS_TRY(expr)                \
    do {                                \
        pastis_status _s = (expr);      \
        if (_s != PASTIS_OK) return _s; \
    } while (0)

#define HIP_TRY(ctx, expr, what)                                        \
    do {                                                                \
        hipError_t _e = (expr);                                         \
        if (_e != hipSuccess) return pastis::hip_error(ctx, _e, what);  \
    } while (0)

struct SwWork;

// Host copy of the offsets plus the device residues/offsets of a call.
struct Staged {
    const uint8_t *d_res = nullptr;
    const int64_t *d_off = nullptr;
    std::vector<int64_t> h_off;
    int64_t n_res = 0;
    int max_len = 0;
};

pastis_status stage_sequences(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int on_device, hipStream_t s, Staged &st);
pastis_status encode_into(pastis_ctx *ctx, const uint8_t *d_res, int64_t n_res, uint8_t **codes_out,
                          unsigned long long *flag, hipStream_t s);
pastis_status read_flags(pastis_ctx *ctx, unsigned long long *d_flags, unsigned long long *h_flags, int count,
                         hipStream_t s);
pastis_status reset_flags(pastis_ctx *ctx, unsigned long long **d_flags, hipStream_t s);
pastis_status make_sw_work(pastis_ctx *ctx, int64_t npairs, int max_len, SwWork &wk);
pastis_status align_core(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, const uint32_t *pi,
                         const uint32_t *pj, const uint32_t *seed1, const uint32_t *seed2, int64_t npairs,
                         pastis_pair_record *out, hipStream_t s);
// Append the features and pass/fail labels (records rec of the exact
// alignment) of the ctx's current candidates to the training pool.
pastis_status mlp_pool_append(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n,
                              const pastis_pair_record *rec, hipStream_t s, int64_t *added);
// Read `count` device words into host memory (synchronises the stream).
pastis_status read_device(pastis_ctx *ctx, const void *d, void *h, size_t bytes, hipStream_t s);

}  // namespace pastis

struct pastis_ctx {
    pastis_params params;
    int device = 0;
    std::string last_error;
    int64_t bad_residue = -1;
    pastis_run_stats stats{};
    int8_t *d_blosum = nullptr;  // 24 x 24 int8 + pad row (25 x 25 when padded)
    // grow-only device buffers, reused across calls
    pastis::DeviceBuffer buf[128];
    // discovery results kept for the align stage / candidate copies
    int64_t n_candidates = 0;
    int64_t n_seqs_last = 0;
    bool have_candidates = false;
    bool records_internal = false;  // the current alignment's records feed edges only
    int last_max16 = 0;             // the last SW call ran 16-bit pass-1 bins up to this R
    uint64_t last_n_dir = 0;        // directional entries of the last candidate discovery
    pastis_tuning tune{16, 50, 1, 1, 0, 4, 4, {0}};
    // learned filter
    pastis::MlpState mlp{};
    bool mlp_alloc = false, mlp_set = false;
    float mlp_tau = 0.f;
    int mlp_step = 0;
    void *h_pinned = nullptr;
    size_t h_pinned_bytes = 0;
    hipEvent_t ev[2 * 9] = {};
    hipEvent_t bin_ev[2 * 32] = {};  // around each SW pass-1 bin launch
    // the multi-strip (long) SW bins run on a second stream, concurrently with
    // the one-strip bins: fork / join events of pass 1, start bound, statistics
    hipStream_t long_stream = nullptr;
    hipEvent_t long_fork[3] = {}, long_join[3] = {};
    // graph mode: the SW stage captured on a stream of the context
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_join[2] = {};
    hipGraphExec_t sw_exec = nullptr;
    uint64_t sw_key = 0;
    bool ev_used[9] = {};
    // no-allocation calls: while arena is set, every buffer of the call is
    // carved from it (the per-device static workspace) instead of allocated
    char *arena = nullptr;
    char *noalloc_ws = nullptr;  // this device's workspace (pastis_align_pairs_noalloc)
    size_t arena_cap = 0, arena_used = 0;
    size_t arena_off[128] = {}, arena_len[128] = {};
};

namespace pastis {

enum BufId {
    kBufResidues = 0,
    kBufOffsets,
    kBufCodes,
    kBufFlag,
    kBufPairs,
    kBufPass1,
    kBufScratch,
    kBufBinOf,
    kBufBinMeta,
    kBufIdx,
    kBufIdx2,
    kBufCandLo,
    kBufCandHi,
    kBufCandCnt,
    kBufCandS1,
    kBufCandS2,
    kBufRecords,
    kBufXdRedo,
    kBufXdRing,
    kBufMlpComp,
    kBufMlpFeat,
    kBufMlpLogit,
    kBufMlpKeep,
    kBufMlpPos,
    kBufMlpTmp,
    kBufMlpOrder,
    kBufSortKeys,
    kBufSortKeysAlt,
    kBufSortValsAlt,
    kBufSortTemp,
    kBufCount  // first id used by the discovery stage
};
constexpr int kNumBufs = 128;

pastis_status set_error(pastis_ctx *ctx, pastis_status s, const std::string &msg);
pastis_status hip_error(pastis_ctx *ctx, hipError_t e, const char *what);
// Make buffer `id` at least `bytes` long (contents not preserved on growth).
pastis_status ensure(pastis_ctx *ctx, int id, size_t bytes, void **out);
pastis_status ensure_pinned(pastis_ctx *ctx, size_t bytes, void **out);
// Record the start / end of a stage on stream s; collect() adds elapsed times
// of every recorded stage into ctx->stats.ms_stage (after synchronising s).
hipError_t stage_begin(pastis_ctx *ctx, int stage, hipStream_t s);
hipError_t stage_end(pastis_ctx *ctx, int stage, hipStream_t s);
hipError_t stage_collect(pastis_ctx *ctx, hipStream_t s);

// ---- kernels' host launchers (each returns hipGetLastError()) ----
hipError_t launch_encode(const uint8_t *ascii, int64_t n, uint8_t *codes, unsigned long long *bad, hipStream_t s);
hipError_t launch_orient_pairs(const int64_t *offsets, int64_t n, const uint32_t *pi, const uint32_t *pj,
                               const uint32_t *seed1, const uint32_t *seed2, int64_t npairs, int k, PairDesc *out,
                               unsigned long long *bad, hipStream_t s);

struct SwPass1Out {
    int32_t score;
    int32_t end_a, end_b;
    int32_t pad;
};

// Work buffers of an alignment stage (device): per-pair bin ids, bin counts,
// bin starts for the two passes, a cursor, the two binned index lists, and
// boundary-row scratch for pairs taller than one strip (6 planes of max_len
// ints per wave, for sw_scratch_waves() waves).
// counters: [0] cells, [1] statistics-pass pairs, [2] their cells, [3]
// start-bound pairs, [4] their cells, [kCounterXdQueue] the x-drop kernel's
// work queue, [kCounterBinCells + b] pass-1 cells of SW bin b
constexpr int kCounterXdQueue = 5;
constexpr int kCounterIntraFlag = 6;  // an intra-pair wait ran out of its bound
constexpr int kCounterBinCells = 8;
constexpr int kNumCounters = kCounterBinCells + 32;

struct SwWork {
    unsigned long long *counters;
    int8_t *bin_of;
    int *counts, *starts, *starts2, *cursor;
    int *idx, *idx2;
    int *scratch;
    int64_t scratch_per_wave;
    int *queue;  // work-queue counters: pass 1, start bound, statistics, pass 1 of the taller half (32 bins each)
    // per bin: the first pass-1 item of its taller half (16-bit strip bins of
    // up to 8 rows per lane split their pairs by rows: up to 64 R - 32 rows,
    // and more)
    int *split;
    // pairing of the 16-bit pass (pairs sorted by bin, then longer b first)
    uint64_t *sort_keys = nullptr, *sort_keys_alt = nullptr;
    uint32_t *sort_vals_alt = nullptr;
    void *sort_temp = nullptr;
};
int sw_num_bins();
void sw_bin_shape(int bin, int32_t *rows_per_lane, int32_t *multi);
int64_t xd_global_waves();
size_t xd_ring_bytes_per_wave();
// XD alignment of every pair; bands wider than the LDS ring are redone from
// redo[] (device list, count in *n_redo, which must start at 0) with rings in
// gring (xd_global_waves() * xd_ring_bytes_per_wave() bytes).
hipError_t launch_xd(pastis_ctx *ctx, const uint8_t *codes, const PairDesc *pairs, int64_t npairs,
                     const int8_t *blosum, const Scoring &sc, int k, pastis_pair_record *out, uint32_t *redo,
                     uint32_t *n_redo, int *gring, unsigned long long *counters, hipStream_t s);
int64_t sw_scratch_waves();
// Queries the resident blocks of the SW kernels whose grids follow their
// occupancy (once per process, before any launch is captured).
void sw_init_occupancy();
// Sequences a of at most this many rows run in one strip (no boundary rows).
int sw_one_strip_max_rows();

// max16 > 0: pass 1 of one-strip pairs with at most max16 rows per lane in
// 16-bit lanes, two pairs per wave; its records leave end_b = -1 for pairs
// that skip the statistics pass.  grid_scale multiplies the pass-1 grids;
// intra = 1 runs pass 1 of the 32-bit multi-strip bins one workgroup per pair;
// 16-bit bins of at most narrow16 (<= 4) rows per lane run strips of 16 lanes
// (eight pairs per wave), the other bins up to 8 rows per lane strips of 32;
// multi-strip launches take at most long_blocks (1..4) blocks per CU.
hipError_t launch_sw(pastis_ctx *ctx, const uint8_t *codes, const PairDesc *pairs, int64_t npairs,
                     const int8_t *blosum, const Scoring &sc, SwPass1Out *p1, pastis_pair_record *out,
                     const SwWork &wk, int stats_mode, int max16, int grid_scale, int grid_scale_wide, int intra,
                     int narrow16, int long_blocks, bool timed, hipStream_t s);
// 16-bit pass 1 needs o + e >= 4 (biased scores stay non-negative).
bool sw16_supported(const Scoring &sc);
bool sw_bin_is16(int bin, int max16);

}  // namespace pastis
