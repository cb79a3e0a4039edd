// C ABI entry points: context, staging, error handling, and the align stage.
#include <algorithm>
#include <chrono>
#include <mutex>

#include "internal.hpp"
#include "prim.hpp"

using namespace pastis;

namespace pastis {

pastis_status set_error(pastis_ctx *ctx, pastis_status s, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return s;
}

pastis_status hip_error(pastis_ctx *ctx, hipError_t e, const char *what) {
    return set_error(ctx, PASTIS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

pastis_status ensure(pastis_ctx *ctx, int id, size_t bytes, void **out) {
    if (bytes == 0) bytes = 256;
    if (ctx->arena) {
        // a no-allocation call: carve the buffer from the device workspace
        // (once per id and call, as the cached buffers are grow-only)
        if (ctx->arena_len[id] >= bytes) {
            *out = ctx->arena + ctx->arena_off[id];
            return PASTIS_OK;
        }
        const size_t off = (ctx->arena_used + 255) & ~(size_t)255;
        if (off + bytes > ctx->arena_cap)
            return set_error(ctx, PASTIS_E_CAPACITY,
                             "the call needs more than the " + std::to_string(ctx->arena_cap) +
                                 " bytes of the no-allocation workspace");
        ctx->arena_off[id] = off;
        ctx->arena_len[id] = bytes;
        ctx->arena_used = off + bytes;
        *out = ctx->arena + off;
        return PASTIS_OK;
    }
    DeviceBuffer &b = ctx->buf[id];
    if (b.bytes < bytes) {
        if (b.ptr) {
            hipError_t e = hipFree(b.ptr);
            if (e != hipSuccess) return hip_error(ctx, e, "hipFree");
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = bytes + bytes / 4;  // some headroom against regrowth
        hipError_t e = hipMalloc(&b.ptr, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ctx, PASTIS_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
        }
        b.bytes = want;
    }
    *out = b.ptr;
    return PASTIS_OK;
}

pastis_status ensure_pinned(pastis_ctx *ctx, size_t bytes, void **out) {
    if (ctx->arena && ctx->h_pinned_bytes < bytes)
        return set_error(ctx, PASTIS_E_INVAL, "a no-allocation call takes device inputs and outputs only");
    if (ctx->h_pinned_bytes < bytes) {
        if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
        ctx->h_pinned = nullptr;
        ctx->h_pinned_bytes = 0;
        hipError_t e = hipHostMalloc(&ctx->h_pinned, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return set_error(ctx, PASTIS_E_NOMEM, "pinned host allocation failed");
        ctx->h_pinned_bytes = bytes;
    }
    *out = ctx->h_pinned;
    return PASTIS_OK;
}

hipError_t stage_begin(pastis_ctx *ctx, int stage, hipStream_t s) {
    ctx->ev_used[stage] = true;
    return hipEventRecord(ctx->ev[2 * stage], s);
}

hipError_t stage_end(pastis_ctx *ctx, int stage, hipStream_t s) { return hipEventRecord(ctx->ev[2 * stage + 1], s); }

hipError_t stage_collect(pastis_ctx *ctx, hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int st = 0; st < kNumStages; ++st) {
        if (!ctx->ev_used[st]) continue;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ctx->ev[2 * st], ctx->ev[2 * st + 1]);
        if (e != hipSuccess) return e;
        ctx->stats.ms_stage[st] += ms;
        ctx->ev_used[st] = false;
    }
    return hipSuccess;
}

}  // namespace pastis

namespace {

// Workspace of pastis_align_pairs_noalloc: every buffer such a call uses is
// carved from it.  Each GPU holds its own copy until the process ends; all
// calls on one GPU share it.  Host code reaches it only through the address
// hipGetSymbolAddress gives for the current device (the array's name is a
// host-side stand-in there).
static __device__ __align__(256) unsigned char scratch[PASTIS_NOALLOC_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// This device's address of the workspace, looked up once per device with
// the device current (context creation).
hipError_t bind_scratch(int device, char **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (char *)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

pastis_status validate(const pastis_params *p, std::string &why) {
    if (p->k < 1 || p->k > 8) return why = "k must be in 1..8", PASTIS_E_INVAL;
    if (p->n_subs < 0 || p->n_subs > 64) return why = "n_subs must be in 0..64", PASTIS_E_INVAL;
    if (p->sub_alphabet != 20 && p->sub_alphabet != 24) return why = "sub_alphabet must be 20 or 24", PASTIS_E_INVAL;
    if (p->ck_min < 1) return why = "ck_min must be >= 1", PASTIS_E_INVAL;
    if (p->align_mode != PASTIS_ALIGN_SW && p->align_mode != PASTIS_ALIGN_XD)
        return why = "align_mode must be SW or XD", PASTIS_E_INVAL;
    if (p->gap_open < 0 || p->gap_open > 1000 || p->gap_extend < 0 || p->gap_extend > 1000)
        return why = "gap costs must be in 0..1000", PASTIS_E_INVAL;
    if (p->xdrop < 0 || p->xdrop > 1000000) return why = "xdrop must be in 0..1e6", PASTIS_E_INVAL;
    if (p->min_identity_pct < 0 || p->min_identity_pct > 100 || p->min_coverage_pct < 0 ||
        p->min_coverage_pct > 100)
        return why = "identity/coverage percentages must be in 0..100", PASTIS_E_INVAL;
    if (p->weight_mode != PASTIS_WEIGHT_ANI && p->weight_mode != PASTIS_WEIGHT_NS)
        return why = "weight_mode must be ANI or NS", PASTIS_E_INVAL;
    if (p->score_width != 0 && p->score_width != 16 && p->score_width != 32)
        return why = "score_width must be 0, 16 or 32", PASTIS_E_INVAL;
    if (p->full_records != 0 && p->full_records != 1) return why = "full_records must be 0 or 1", PASTIS_E_INVAL;
    if (p->filter_mode != 0 && p->filter_mode != 1) return why = "filter_mode must be 0 or 1", PASTIS_E_INVAL;
    if (p->graph_mode != 0 && p->graph_mode != 1) return why = "graph_mode must be 0 or 1", PASTIS_E_INVAL;
    if (p->candidate_room < 0) return why = "candidate_room must be >= 0", PASTIS_E_INVAL;
    if (p->block_entries < 0) return why = "block_entries must be >= 0", PASTIS_E_INVAL;
    for (int t = 0; t < 3; ++t)
        if (p->reserved[t] != 0) return why = "reserved fields must be zero", PASTIS_E_INVAL;
    return PASTIS_OK;
}

}  // namespace

namespace pastis {

pastis_status stage_sequences(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int on_device, hipStream_t s, Staged &st) {
    if (n < 0) return set_error(ctx, PASTIS_E_INVAL, "n must be >= 0");
    if (!offsets) return set_error(ctx, PASTIS_E_INVAL, "offsets is NULL");
    st.h_off.resize((size_t)n + 1);
    if (on_device) {
        HIP_TRY(ctx, hipMemcpyAsync(st.h_off.data(), offsets, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s),
                "copy offsets");
        HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    } else {
        memcpy(st.h_off.data(), offsets, sizeof(int64_t) * (n + 1));
    }
    if (st.h_off[0] != 0) return set_error(ctx, PASTIS_E_INVAL, "offsets[0] must be 0");
    int64_t mx = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = st.h_off[i + 1] - st.h_off[i];
        if (len < 0) return set_error(ctx, PASTIS_E_INVAL, "offsets must be non-decreasing");
        if (len > kMaxLen)
            return set_error(ctx, PASTIS_E_INVAL,
                             "sequence " + std::to_string(i) + " is longer than 65535 residues");
        mx = std::max(mx, len);
    }
    st.n_res = st.h_off[n];
    st.max_len = (int)mx;
    if (on_device) {
        st.d_res = residues;
        st.d_off = offsets;
    } else {
        void *dr = nullptr, *doff = nullptr;
        PASTIS_TRY(ensure(ctx, kBufResidues, (size_t)std::max<int64_t>(st.n_res, 1), &dr));
        PASTIS_TRY(ensure(ctx, kBufOffsets, sizeof(int64_t) * (n + 1), &doff));
        if (st.n_res > 0)
            HIP_TRY(ctx, hipMemcpyAsync(dr, residues, (size_t)st.n_res, hipMemcpyHostToDevice, s), "copy residues");
        HIP_TRY(ctx, hipMemcpyAsync(doff, st.h_off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s),
                "copy offsets");
        st.d_res = (const uint8_t *)dr;
        st.d_off = (const int64_t *)doff;
    }
    return PASTIS_OK;
}

// Encodes into kBufCodes; the bad-residue flag lives in kBufFlag[0].
pastis_status encode_into(pastis_ctx *ctx, const uint8_t *d_res, int64_t n_res, uint8_t **codes_out,
                          unsigned long long *flag, hipStream_t s) {
    void *codes = nullptr;
    PASTIS_TRY(ensure(ctx, kBufCodes, (size_t)std::max<int64_t>(n_res, 1), &codes));
    HIP_TRY(ctx, launch_encode(d_res, n_res, (uint8_t *)codes, flag, s), "encode kernel");
    *codes_out = (uint8_t *)codes;
    return PASTIS_OK;
}

pastis_status read_device(pastis_ctx *ctx, const void *d, void *h, size_t bytes, hipStream_t s) {
    HIP_TRY(ctx, hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s), "read device");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status read_flags(pastis_ctx *ctx, unsigned long long *d_flags, unsigned long long *h_flags, int count,
                         hipStream_t s) {
    HIP_TRY(ctx, hipMemcpyAsync(h_flags, d_flags, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, s),
            "read flags");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

// flags[0]: smallest bad residue index (init ~0), flags[1]: pair errors
pastis_status reset_flags(pastis_ctx *ctx, unsigned long long **d_flags, hipStream_t s) {
    void *f = nullptr;
    PASTIS_TRY(ensure(ctx, kBufFlag, 4 * sizeof(unsigned long long), &f));
    const unsigned long long init[4] = {~0ull, 0ull, 0ull, 0ull};
    HIP_TRY(ctx, hipMemcpyAsync(f, init, sizeof(init), hipMemcpyHostToDevice, s), "reset flags");
    *d_flags = (unsigned long long *)f;
    return PASTIS_OK;
}

pastis_status make_sw_work(pastis_ctx *ctx, int64_t npairs, int max_len, SwWork &wk) {
    sw_init_occupancy();
    void *p = nullptr;
    PASTIS_TRY(ensure(ctx, kBufBinOf, (size_t)std::max<int64_t>(npairs, 1), &p));
    wk.bin_of = (int8_t *)p;
    PASTIS_TRY(ensure(ctx, kBufBinMeta, sizeof(int) * 384 + sizeof(unsigned long long) * kNumCounters, &p));
    wk.counts = (int *)p;
    wk.counters = (unsigned long long *)((int *)p + 384);
    // counts: 32 bins; starts, starts2: 33 bounds each; cursor, split: 32;
    // four work queues of 32 bins
    wk.starts = wk.counts + 32;
    wk.starts2 = wk.counts + 72;
    wk.cursor = wk.counts + 112;
    wk.split = wk.counts + 144;
    wk.queue = wk.counts + 176;
    PASTIS_TRY(ensure(ctx, kBufIdx, sizeof(int) * (size_t)std::max<int64_t>(npairs, 1), &p));
    wk.idx = (int *)p;
    PASTIS_TRY(ensure(ctx, kBufIdx2, sizeof(int) * (size_t)std::max<int64_t>(npairs, 1), &p));
    wk.idx2 = (int *)p;
    wk.scratch_per_wave = 6 * (int64_t)std::max(max_len, 1);
    // only multi-strip pairs (a sequence a longer than one strip) touch the
    // boundary rows; without such a sequence the buffer is never read
    const size_t scratch_bytes = max_len > sw_one_strip_max_rows()
                                     ? sizeof(int) * (size_t)wk.scratch_per_wave * (size_t)sw_scratch_waves()
                                     : 256;
    PASTIS_TRY(ensure(ctx, kBufScratch, scratch_bytes, &p));
    wk.scratch = (int *)p;
    return PASTIS_OK;
}

static pastis_status make_sort_work(pastis_ctx *ctx, int64_t npairs, SwWork &wk) {
    const size_t n = (size_t)std::max<int64_t>(npairs, 1);
    void *p = nullptr;
    PASTIS_TRY(ensure(ctx, kBufSortKeys, sizeof(uint64_t) * n, &p));
    wk.sort_keys = (uint64_t *)p;
    PASTIS_TRY(ensure(ctx, kBufSortKeysAlt, sizeof(uint64_t) * n, &p));
    wk.sort_keys_alt = (uint64_t *)p;
    PASTIS_TRY(ensure(ctx, kBufSortValsAlt, sizeof(uint32_t) * n, &p));
    wk.sort_vals_alt = (uint32_t *)p;
    PASTIS_TRY(ensure(ctx, kBufSortTemp, radix_temp_bytes(npairs) + 256, &p));
    wk.sort_temp = p;
    return PASTIS_OK;
}

// Orient the pairs, then run the context's alignment mode; `out` gets one
// record per pair.  Validates pair indices (PASTIS_E_INVAL).
void mlp_free(pastis_ctx *ctx);

// The SW stage as a HIP graph on the context's stream: captured when its
// shape (pair count, buffers, scoring, schedule) differs from the cached one,
// else replayed.  The caller's stream waits for it through events; the stage
// time goes to the pass-1 slot.
static uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

static pastis_status sw_graph(pastis_ctx *ctx, const uint8_t *codes, const PairDesc *pairs, int64_t npairs,
                              const Scoring &sc, SwPass1Out *p1, pastis_pair_record *out, const SwWork &wk,
                              int stats_mode, int max16, hipStream_t s) {
    const int grid = ctx->tune.sw_grid_scale, grid_wide = ctx->tune.sw_grid_scale_wide, intra = ctx->tune.sw_intra_pair;
    const int narrow = ctx->tune.sw16_narrow_rows, long_blocks = ctx->tune.sw_long_blocks;
    uint64_t key = 0;
    const uint64_t parts[] = {(uint64_t)npairs, (uint64_t)codes, (uint64_t)pairs, (uint64_t)p1, (uint64_t)out,
                              (uint64_t)wk.counters, (uint64_t)wk.bin_of, (uint64_t)wk.counts, (uint64_t)wk.idx,
                              (uint64_t)wk.idx2, (uint64_t)wk.scratch, (uint64_t)wk.scratch_per_wave,
                              (uint64_t)wk.sort_keys, (uint64_t)wk.sort_keys_alt, (uint64_t)wk.sort_vals_alt,
                              (uint64_t)wk.sort_temp, (uint64_t)sc.gap_open, (uint64_t)sc.gap_extend,
                              (uint64_t)sc.id_pct, (uint64_t)sc.cov_pct, (uint64_t)sc.direct_pct,
                              (uint64_t)stats_mode, (uint64_t)max16, (uint64_t)grid, (uint64_t)grid_wide, (uint64_t)intra,
                              (uint64_t)narrow, (uint64_t)long_blocks,
                              (uint64_t)ctx->d_blosum};
    for (uint64_t v : parts) key = mix(key, v);
    hipStream_t gs = ctx->graph_stream;
    if (!ctx->sw_exec || key != ctx->sw_key) {
        if (ctx->sw_exec) {
            (void)hipGraphExecDestroy(ctx->sw_exec);
            ctx->sw_exec = nullptr;
        }
        HIP_TRY(ctx, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal), "graph capture");
        const hipError_t le = launch_sw(ctx, codes, pairs, npairs, ctx->d_blosum, sc, p1, out, wk, stats_mode, max16,
                                        grid, grid_wide, intra, narrow, long_blocks, false, gs);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(gs, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_error(ctx, le != hipSuccess ? le : ce, "graph capture");
        }
        const hipError_t ie = hipGraphInstantiate(&ctx->sw_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            ctx->sw_exec = nullptr;
            return hip_error(ctx, ie, "graph instantiate");
        }
        ctx->sw_key = key;
        ctx->stats.sw_graph = 1;
    } else {
        ctx->stats.sw_graph = 2;
    }
    HIP_TRY(ctx, hipEventRecord(ctx->graph_join[0], s), "event");
    HIP_TRY(ctx, hipStreamWaitEvent(gs, ctx->graph_join[0], 0), "event");
    HIP_TRY(ctx, stage_begin(ctx, kStAlign1, gs), "event");
    HIP_TRY(ctx, hipGraphLaunch(ctx->sw_exec, gs), "graph launch");
    HIP_TRY(ctx, stage_end(ctx, kStAlign1, gs), "event");
    HIP_TRY(ctx, hipEventRecord(ctx->graph_join[1], gs), "event");
    HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->graph_join[1], 0), "event");
    return PASTIS_OK;
}

pastis_status align_core(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, const uint32_t *pi,
                         const uint32_t *pj, const uint32_t *seed1, const uint32_t *seed2, int64_t npairs,
                         pastis_pair_record *out, hipStream_t s) {
    ctx->stats.n_aligned = npairs;
    if (npairs == 0) return PASTIS_OK;
    unsigned long long *d_flags = nullptr, h_flags[4];
    PASTIS_TRY(reset_flags(ctx, &d_flags, s));
    void *pairs = nullptr;
    PASTIS_TRY(ensure(ctx, kBufPairs, sizeof(PairDesc) * (size_t)npairs, &pairs));
    HIP_TRY(ctx,
            launch_orient_pairs(st.d_off, n, pi, pj, seed1, seed2, npairs, ctx->params.k, (PairDesc *)pairs,
                                d_flags + 1, s),
            "orient kernel");
    PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 2, s));
    if (h_flags[1] & 1ull) return set_error(ctx, PASTIS_E_INVAL, "pair index out of range or pi == pj");
    const pastis_params &P = ctx->params;
    Scoring sc{P.gap_open, P.gap_extend, P.xdrop, P.min_identity_pct, P.min_coverage_pct, ctx->tune.sw_direct_pct};
    void *p1 = nullptr;
    PASTIS_TRY(ensure(ctx, kBufPass1, sizeof(SwPass1Out) * (size_t)npairs, &p1));
    SwWork wk;
    PASTIS_TRY(make_sw_work(ctx, npairs, st.max_len, wk));
    HIP_TRY(ctx, fill<unsigned long long>(wk.counters, kNumCounters, 0ull, s), "reset");
    ctx->stats.sw_bins = 0;
    ctx->stats.int32_pairs = 0;
    ctx->last_max16 = 0;
    // traceback statistics: every pair on request; none for the normalised
    // score weight; otherwise only where the coverage cut can still hold
    const int stats_mode = P.full_records ? 1 : (P.weight_mode == PASTIS_WEIGHT_NS ? 2 : 0);
    if (P.align_mode == PASTIS_ALIGN_SW) {
        // 16-bit pass 1 on request, or by default where its records stay
        // inside the search (they omit end_b of pairs without statistics,
        // which no edge then reports)
        const bool use16 = sw16_supported(sc) && stats_mode != 1 &&
                           (P.score_width == 16 || (P.score_width == 0 && ctx->records_internal));
        const int max16 = !use16 ? 0 : P.score_width == 16 ? 16 : ctx->tune.sw16_max_rows;
        if (max16 > 0) PASTIS_TRY(make_sort_work(ctx, npairs, wk));
        ctx->last_max16 = max16;
        if (P.graph_mode) {
            PASTIS_TRY(sw_graph(ctx, codes, (const PairDesc *)pairs, npairs, sc, (SwPass1Out *)p1, out, wk, stats_mode,
                                max16, s));
        } else {
            HIP_TRY(ctx,
                    launch_sw(ctx, codes, (const PairDesc *)pairs, npairs, ctx->d_blosum, sc, (SwPass1Out *)p1, out,
                              wk, stats_mode, max16, ctx->tune.sw_grid_scale, ctx->tune.sw_grid_scale_wide,
                              ctx->tune.sw_intra_pair, ctx->tune.sw16_narrow_rows, ctx->tune.sw_long_blocks, true, s),
                    "sw kernels");
        }
    } else {
        void *redo = nullptr, *ring = nullptr;
        PASTIS_TRY(ensure(ctx, kBufXdRedo, sizeof(uint32_t) * (size_t)(npairs + 4), &redo));
        PASTIS_TRY(ensure(ctx, kBufXdRing, (size_t)xd_global_waves() * xd_ring_bytes_per_wave(), &ring));
        uint32_t *n_redo = (uint32_t *)redo + npairs;
        HIP_TRY(ctx, fill<uint32_t>(n_redo, 1, 0u, s), "reset");
        HIP_TRY(ctx,
                launch_xd(ctx, codes, (const PairDesc *)pairs, npairs, ctx->d_blosum, sc, P.k, out, (uint32_t *)redo,
                          n_redo, (int *)ring, wk.counters, s),
                "xd kernels");
    }
    unsigned long long c[kNumCounters];
    PASTIS_TRY(read_device(ctx, wk.counters, c, sizeof(c), s));
    if (c[kCounterIntraFlag]) return set_error(ctx, PASTIS_E_DEVICE, "intra-pair pass 1: a strip hand-off wait ran out");
    ctx->stats.cells = (int64_t)c[0];
    ctx->stats.stats_pass_pairs = (int64_t)c[1];
    ctx->stats.stats_pass_cells = (int64_t)c[2];
    ctx->stats.bound_pass_pairs = (int64_t)c[3];
    ctx->stats.bound_pass_cells = (int64_t)c[4];
    if (P.align_mode == PASTIS_ALIGN_SW && !P.graph_mode) {
        int starts[33];  // pass-1 bin bounds (the pass-2 binning reuses the counts)
        PASTIS_TRY(read_device(ctx, wk.starts, starts, sizeof(starts), s));
        const int nb = sw_num_bins();
        ctx->stats.sw_bins = nb;
        for (int b = 0; b < nb; ++b) {
            sw_bin_shape(b, &ctx->stats.sw_bin_rows[b], &ctx->stats.sw_bin_multi[b]);
            const bool b16 = sw_bin_is16(b, ctx->last_max16);
            ctx->stats.sw_bin_bits[b] = b16 ? 16 : 32;
            if (!b16) ctx->stats.int32_pairs += starts[b + 1] - starts[b];
            ctx->stats.sw_bin_pairs[b] = starts[b + 1] - starts[b];
            ctx->stats.sw_bin_cells[b] = (int64_t)c[kCounterBinCells + b];
            float ms = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->bin_ev[2 * b], ctx->bin_ev[2 * b + 1]), "event time");
            ctx->stats.sw_bin_ms[b] = ms;
        }
    }
    return PASTIS_OK;
}

pastis_status align_candidates(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, hipStream_t s,
                               pastis_pair_record **rec_out) {
    const int64_t nc = ctx->n_candidates;
    void *rec = nullptr;
    PASTIS_TRY(ensure(ctx, kBufRecords, sizeof(pastis_pair_record) * (size_t)std::max<int64_t>(nc, 1), &rec));
    *rec_out = (pastis_pair_record *)rec;
    ctx->records_internal = true;
    struct Reset {
        pastis_ctx *c;
        ~Reset() { c->records_internal = false; }
    } reset{ctx};
    return align_core(ctx, st, codes, n, (const uint32_t *)ctx->buf[kBufCandLo].ptr,
                      (const uint32_t *)ctx->buf[kBufCandHi].ptr, (const uint32_t *)ctx->buf[kBufCandS1].ptr,
                      (const uint32_t *)ctx->buf[kBufCandS2].ptr, nc, (pastis_pair_record *)rec, s);
}

}  // namespace pastis

extern "C" {

void pastis_default_params(pastis_params *p) {
    memset(p, 0, sizeof(*p));
    p->k = 6;
    p->n_subs = 0;
    p->sub_alphabet = 20;
    p->ck_min = 1;
    p->align_mode = PASTIS_ALIGN_SW;
    p->gap_open = 11;
    p->gap_extend = 1;
    p->xdrop = 49;
    p->min_identity_pct = 30;
    p->min_coverage_pct = 70;
    p->weight_mode = PASTIS_WEIGHT_ANI;
    p->score_width = 0;
    p->full_records = 0;
}

const char *pastis_status_string(pastis_status s) {
    switch (s) {
        case PASTIS_OK: return "ok";
        case PASTIS_E_INVAL: return "invalid argument";
        case PASTIS_E_BAD_RESIDUE: return "residue outside the 24-letter alphabet";
        case PASTIS_E_NOMEM: return "out of memory";
        case PASTIS_E_DEVICE: return "HIP device error";
        case PASTIS_E_CAPACITY: return "destination too small";
        case PASTIS_E_STATE: return "call out of order";
    }
    return "unknown status";
}

pastis_status pastis_create(const pastis_params *p, int device, pastis_ctx **out) {
    if (!p || !out) return PASTIS_E_INVAL;
    *out = nullptr;
    std::string why;
    if (validate(p, why) != PASTIS_OK) return PASTIS_E_INVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return PASTIS_E_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return PASTIS_E_DEVICE;
    pastis_ctx *ctx = new pastis_ctx();
    ctx->params = *p;
    ctx->device = device;
    if (bind_scratch(device, &ctx->noalloc_ws) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return PASTIS_E_DEVICE;
    }
    // 25 x 25 scoring table: residues 0..23 plus the pad code, whose scores
    // are the most negative int8 so padded cells never raise a maximum.
    int8_t table[25 * 25];
    for (int a = 0; a < 25; ++a)
        for (int b = 0; b < 25; ++b)
            table[a * 25 + b] = (a < kAlpha && b < kAlpha) ? kBlosum62[a * kAlpha + b] : (int8_t)-128;
    if (hipMalloc(&ctx->d_blosum, sizeof(table)) != hipSuccess ||
        hipMemcpy(ctx->d_blosum, table, sizeof(table), hipMemcpyHostToDevice) != hipSuccess) {
        delete ctx;
        return PASTIS_E_DEVICE;
    }
    for (auto &ev : ctx->ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            pastis_destroy(ctx);
            return PASTIS_E_DEVICE;
        }
    }
    for (auto &ev : ctx->bin_ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            pastis_destroy(ctx);
            return PASTIS_E_DEVICE;
        }
    }
    // default priority; non-blocking so it never waits on the null stream
    if (hipStreamCreateWithFlags(&ctx->long_stream, hipStreamNonBlocking) != hipSuccess) {
        pastis_destroy(ctx);
        return PASTIS_E_DEVICE;
    }
    for (int i = 0; i < 3; ++i) {
        if (hipEventCreateWithFlags(&ctx->long_fork[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->long_join[i], hipEventDisableTiming) != hipSuccess) {
            pastis_destroy(ctx);
            return PASTIS_E_DEVICE;
        }
    }
    if (p->graph_mode) {
        // default priority; non-blocking so it never waits on the null stream
        if (hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->graph_join[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->graph_join[1], hipEventDisableTiming) != hipSuccess) {
            pastis_destroy(ctx);
            return PASTIS_E_DEVICE;
        }
    }
    *out = ctx;
    return PASTIS_OK;
}

void pastis_destroy(pastis_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    mlp_free(ctx);
    for (auto &b : ctx->buf)
        if (b.ptr) (void)hipFree(b.ptr);
    if (ctx->d_blosum) (void)hipFree(ctx->d_blosum);
    if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
    for (auto &ev : ctx->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : ctx->bin_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->sw_exec) (void)hipGraphExecDestroy(ctx->sw_exec);
    if (ctx->long_stream) {
        (void)hipStreamSynchronize(ctx->long_stream);
        (void)hipStreamDestroy(ctx->long_stream);
    }
    for (int i = 0; i < 3; ++i) {
        if (ctx->long_fork[i]) (void)hipEventDestroy(ctx->long_fork[i]);
        if (ctx->long_join[i]) (void)hipEventDestroy(ctx->long_join[i]);
    }
    if (ctx->graph_stream) {
        (void)hipStreamSynchronize(ctx->graph_stream);
        (void)hipStreamDestroy(ctx->graph_stream);
    }
    for (auto &ev : ctx->graph_join)
        if (ev) (void)hipEventDestroy(ev);
    delete ctx;
}

const char *pastis_last_error(const pastis_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int64_t pastis_bad_residue_index(const pastis_ctx *ctx) { return ctx ? ctx->bad_residue : -1; }

pastis_status pastis_stats(const pastis_ctx *ctx, pastis_run_stats *out) {
    if (!ctx || !out) return PASTIS_E_INVAL;
    *out = ctx->stats;
    return PASTIS_OK;
}

pastis_status pastis_encode(pastis_ctx *ctx, const uint8_t *residues, int64_t n_residues, int input_on_device,
                            uint8_t *codes, void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    if (n_residues < 0 || (n_residues > 0 && (!residues || !codes)))
        return set_error(ctx, PASTIS_E_INVAL, "bad encode arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->bad_residue = -1;
    const uint8_t *d_res = residues;
    if (!input_on_device && n_residues > 0) {
        void *dr = nullptr;
        PASTIS_TRY(ensure(ctx, kBufResidues, (size_t)n_residues, &dr));
        HIP_TRY(ctx, hipMemcpyAsync(dr, residues, (size_t)n_residues, hipMemcpyHostToDevice, s), "copy residues");
        d_res = (const uint8_t *)dr;
    }
    unsigned long long *d_flags = nullptr, h_flags[4];
    PASTIS_TRY(reset_flags(ctx, &d_flags, s));
    HIP_TRY(ctx, launch_encode(d_res, n_residues, codes, d_flags, s), "encode kernel");
    PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
    if (h_flags[0] != ~0ull) {
        ctx->bad_residue = (int64_t)h_flags[0];
        return set_error(ctx, PASTIS_E_BAD_RESIDUE, "bad residue at index " + std::to_string(h_flags[0]));
    }
    return PASTIS_OK;
}

}  // extern "C"

namespace {

pastis_status align_pairs_impl(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                               int input_on_device, const uint32_t *pi, const uint32_t *pj, const uint32_t *seed1,
                               const uint32_t *seed2, int64_t npairs, pastis_pair_record *out, void *stream) {
    if (npairs < 0 || (npairs > 0 && (!pi || !pj || !out)))
        return set_error(ctx, PASTIS_E_INVAL, "bad pair arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    auto t0 = std::chrono::steady_clock::now();
    ctx->bad_residue = -1;
    ctx->stats = pastis_run_stats{};
    Staged st;
    PASTIS_TRY(stage_sequences(ctx, residues, offsets, n, input_on_device, s, st));
    unsigned long long *d_flags = nullptr, h_flags[4];
    PASTIS_TRY(reset_flags(ctx, &d_flags, s));
    uint8_t *codes = nullptr;
    HIP_TRY(ctx, stage_begin(ctx, kStEncode, s), "event");
    PASTIS_TRY(encode_into(ctx, st.d_res, st.n_res, &codes, d_flags, s));
    HIP_TRY(ctx, stage_end(ctx, kStEncode, s), "event");
    PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
    if (h_flags[0] != ~0ull) {
        ctx->bad_residue = (int64_t)h_flags[0];
        return set_error(ctx, PASTIS_E_BAD_RESIDUE, "bad residue at index " + std::to_string(h_flags[0]));
    }
    PASTIS_TRY(align_core(ctx, st, codes, n, pi, pj, seed1, seed2, npairs, out, s));
    HIP_TRY(ctx, stage_collect(ctx, s), "sync");
    auto t1 = std::chrono::steady_clock::now();
    ctx->stats.n_sequences = n;
    ctx->stats.n_residues = st.n_res;
    ctx->stats.ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return PASTIS_OK;
}

}  // namespace

extern "C" {

pastis_status pastis_align_pairs(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                 int input_on_device, const uint32_t *pi, const uint32_t *pj, const uint32_t *seed1,
                                 const uint32_t *seed2, int64_t npairs, pastis_pair_record *out, void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    return align_pairs_impl(ctx, residues, offsets, n, input_on_device, pi, pj, seed1, seed2, npairs, out, stream);
}

pastis_status pastis_align_pairs_noalloc(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                         const uint32_t *pi, const uint32_t *pj, const uint32_t *seed1,
                                         const uint32_t *seed2, int64_t npairs, pastis_pair_record *out,
                                         void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    if (ctx->params.align_mode != PASTIS_ALIGN_SW)
        return set_error(ctx, PASTIS_E_INVAL, "the no-allocation entry point runs Smith-Waterman only");
    if (!ctx->noalloc_ws) return set_error(ctx, PASTIS_E_STATE, "no workspace bound to this context");
    // every buffer of this call comes from the device's workspace; graph
    // mode (whose instantiation allocates) is off for the call
    struct Guard {
        pastis_ctx *c;
        int32_t graph;
        ~Guard() {
            c->arena = nullptr;
            c->params.graph_mode = graph;
        }
    } guard{ctx, ctx->params.graph_mode};
    ctx->params.graph_mode = 0;
    ctx->arena = ctx->noalloc_ws;
    ctx->arena_cap = PASTIS_NOALLOC_BYTES;
    ctx->arena_used = 0;
    memset(ctx->arena_len, 0, sizeof(ctx->arena_len));
    return align_pairs_impl(ctx, residues, offsets, n, 1, pi, pj, seed1, seed2, npairs, out, stream);
}

}  // extern "C"
