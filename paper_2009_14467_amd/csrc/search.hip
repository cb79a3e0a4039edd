// The whole pipeline (Section IV): encode -> k-mers -> [S, A S] -> sparse
// product + threshold + symmetrisation -> candidates -> alignment -> filter
// -> edges.  Host orchestration of the stage kernels, plus the C ABI calls of
// the discovery stage and the result handle.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "kmers.hpp"
#include "prim.hpp"
#include "spgemm.hpp"
#include "subs.hpp"

struct pastis_result {
    pastis_edge *d_edges = nullptr;
    int64_t n = 0;
    int device = 0;
};

namespace pastis {
namespace {

enum DiscBuf {
    kDKCounts = kBufCount,
    kDPostSeq,
    kDPostPos,
    kDPostU,
    kDUkId,
    kDUkStart,
    kDRowStart,
    kDRowU,
    kDRowPos,
    kDKmap,
    kDTemp,
    kDSu,
    kDSd,
    kDScnt,
    kDStmpIds,
    kDStmpD,
    kDAsUb,
    kDAsStart,
    kDAsLen,
    kDAsS,
    kDAsDp,
    kDAsGtab,
    kDMisc,
    kDWork,
    kDBigRows,
    kDDirKey,
    kDDirCnt,
    kDDirS1,
    kDDirS2,
    kDDirDir,
    kDDirKeyAlt,
    kDPerm,
    kDPermAlt,
    kDFlag,
    kDPick,
    kDOpos,
    kDGtab,
    kDGcand,
    kDEdgeFlag,
    kDEdgePos,
    kDSubIn,
    kDSubIds,
    kDSubD,
    kDSubN,
    kDTuneLo,
    kDTuneHi,
    kDTuneS1,
    kDTuneS2,
    kDTuneRec,
    kDPostRec,
    kDRowH,
    kDRowLen,
    kDStage,
    kDEnd
};
static_assert(kDEnd <= kNumBufs, "buffer ids");

template <typename T>
pastis_status get(pastis_ctx *ctx, int id, size_t count, T **out) {
    void *p = nullptr;
    PASTIS_TRY(ensure(ctx, id, sizeof(T) * (count > 0 ? count : 1), &p));
    *out = (T *)p;
    return PASTIS_OK;
}

inline uint32_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return (uint32_t)p;
}

// Misc device words: [0..3] k-mer counts (in KmerTables), the rest below.
struct Misc {
    unsigned long long *max_ub;   // 1
    unsigned long long *max_big;  // 1
    uint32_t *n_big;              // 2
    unsigned long long *d_count;  // 1 (its own 64-bit word)
    uint32_t *d_overflow;         // 1
    uint32_t *n_cand;             // 1
    uint32_t *n_edges;            // 1
    unsigned long long *products; // 1
    int *bin_meta;                // 160 (80 words)
    unsigned long long *nnz_s;    // 1, after bin_meta
};

pastis_status misc(pastis_ctx *ctx, Misc &m) {
    unsigned long long *base = nullptr;
    PASTIS_TRY(get(ctx, kDMisc, 128, &base));
    m.max_ub = base;
    m.max_big = base + 1;
    uint32_t *w = (uint32_t *)(base + 2);
    m.n_big = w;
    m.d_count = base + 7;
    m.d_overflow = w + 3;
    m.n_cand = w + 4;
    m.n_edges = w + 5;
    m.products = base + 6;
    m.bin_meta = (int *)(base + 8);
    m.nnz_s = base + 88;
    return PASTIS_OK;
}

// Edges of aligned candidates (sorted by (lo, hi) since the candidates are).
__global__ void edge_flag_kernel(const pastis_pair_record *__restrict__ rec, int64_t n, int ns_mode,
                                 uint8_t *__restrict__ flag) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        flag[q] = ns_mode ? (rec[q].score > 0) : (rec[q].passed != 0);
}

__global__ void edge_write_kernel(const pastis_pair_record *__restrict__ rec, const uint8_t *__restrict__ flag,
                                  const uint32_t *__restrict__ pos, int64_t n, const uint32_t *__restrict__ lo,
                                  const uint32_t *__restrict__ hi, const uint32_t *__restrict__ count,
                                  const int64_t *__restrict__ offsets, int ns_mode, pastis_edge *__restrict__ out) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[q]) continue;
        const pastis_pair_record r = rec[q];
        pastis_edge e;
        const uint32_t i = lo[q], j = hi[q];
        // rows a are sequence i unless the pair was swapped (then a = j)
        const bool a_is_i = r.swapped == 0;
        e.i = i;
        e.j = j;
        e.score = r.score;
        e.matches = (uint32_t)r.matches;
        e.columns = (uint32_t)r.columns;
        e.beg_i = (uint32_t)(a_is_i ? r.beg_a : r.beg_b);
        e.end_i = (uint32_t)(a_is_i ? r.end_a : r.end_b);
        e.beg_j = (uint32_t)(a_is_i ? r.beg_b : r.beg_a);
        e.end_j = (uint32_t)(a_is_i ? r.end_b : r.end_a);
        e.shared_kmers = (uint16_t)(count[q] > 65535u ? 65535u : count[q]);
        e.seed_used = r.seed_used < 0 ? (uint8_t)255 : (uint8_t)r.seed_used;
        e.flags = (uint8_t)(r.swapped & 1);
        e.identity = __fdiv_rn((float)r.matches, (float)(r.columns > 0 ? r.columns : 1));
        const int64_t li = offsets[i + 1] - offsets[i], lj = offsets[j + 1] - offsets[j];
        e.ns_weight = __fdiv_rn((float)r.score, (float)(li < lj ? li : lj));
        if (ns_mode) {
            // the normalised score needs only the score: the traceback
            // statistics and the alignment's extent are not computed (16-bit
            // pass 1 finds no end column)
            e.beg_i = e.beg_j = e.end_i = e.end_j = 0xFFFFFFFFu;
            e.matches = e.columns = 0;
            e.identity = 0.0f;
        }
        out[pos[q]] = e;
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

// *out += sum of a[0..n) (out cleared by the caller)
__global__ void sum_u32_kernel(const uint32_t *__restrict__ a, int64_t n, unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        acc += a[x];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// Directional entries are indexed with 32 bits downstream.
constexpr uint64_t kMaxDir = 0xFFFFFFF0ull;

// What the sparse product of every row block reads: the k-mer tables and,
// with substitutes, the rows of A S.  Built once per call; sp.kt points at kt.
struct DiscTables {
    KmerTables kt;
    SpgemmArgs sp{};
    int64_t nnz = 0, nu = 0;
    size_t temp_bytes = 0;  // the k-mer stage's temporary buffer (kDTemp)
    DiscTables() = default;
    DiscTables(const DiscTables &) = delete;
    DiscTables &operator=(const DiscTables &) = delete;
};

// Discovery, first part: k-mers, and S and A S with substitutes.
pastis_status discover_tables(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, hipStream_t s,
                              DiscTables &dt) {
    const pastis_params &P = ctx->params;
    const int64_t m = st.n_res;
    const bool subs = P.n_subs > 0;
    // k-mer entries and posting-group heads (entries + groups <= 2 * residues)
    // are 31-bit indices
    if (m >= (1ll << 30)) return set_error(ctx, PASTIS_E_INVAL, "a discovery takes fewer than 2^30 residues");
    Misc M;
    PASTIS_TRY(misc(ctx, M));

    // ---- k-mers
    HIP_TRY(ctx, stage_begin(ctx, kStKmers, s), "event");
    KmerTables &kt = dt.kt;
    PASTIS_TRY(get(ctx, kDKCounts, 4, &kt.counts));
    PASTIS_TRY(get(ctx, kDPostSeq, m, &kt.post_seq));
    PASTIS_TRY(get(ctx, kDPostPos, m, &kt.post_pos));
    PASTIS_TRY(get(ctx, kDPostU, m, &kt.post_u));
    PASTIS_TRY(get(ctx, kDUkId, m, &kt.uk_id));
    PASTIS_TRY(get(ctx, kDUkStart, m + 1, &kt.uk_start));
    PASTIS_TRY(get(ctx, kDRowStart, n + 1, &kt.row_start));
    PASTIS_TRY(get(ctx, kDRowU, m, &kt.row_u));
    PASTIS_TRY(get(ctx, kDRowPos, m, &kt.row_pos));
    kt.row_h = nullptr;
    kt.row_len = nullptr;
    if (!subs) {  // the exact product's entries
        PASTIS_TRY(get(ctx, kDRowH, m, &kt.row_h));
        PASTIS_TRY(get(ctx, kDRowLen, m, &kt.row_len));
    }
    kt.kmap = nullptr;
    const bool dense_map = subs && P.k <= kDenseMapMaxK;  // longer k-mers: binary search of the distinct ids
    if (dense_map) PASTIS_TRY(get(ctx, kDKmap, (size_t)kmap_entries(P.k), &kt.kmap));
    char *temp = nullptr;
    dt.temp_bytes = kmers_temp_bytes(m, n);
    PASTIS_TRY(get(ctx, kDTemp, dt.temp_bytes, &temp));
    HIP_TRY(ctx, build_kmers(codes, st.d_off, n, m, P.k, dense_map, kt, temp, s), "k-mer kernels");
    HIP_TRY(ctx, stage_end(ctx, kStKmers, s), "event");
    uint32_t kc[4];
    PASTIS_TRY(read_device(ctx, kt.counts, kc, sizeof(kc), s));
    const int64_t nnz = kc[0], nu = kc[1];
    dt.nnz = nnz;
    dt.nu = nu;
    ctx->stats.n_kmers = nnz;

    // ---- substitute rows and A S
    SpgemmArgs &sp = dt.sp;
    sp.kt = &kt;
    sp.n = n;
    sp.ck = P.ck_min;
    sp.exact = subs ? 0 : 1;
    if (subs) {
        HIP_TRY(ctx, stage_begin(ctx, kStSubs, s), "event");
        const int W = P.n_subs + 1;
        uint32_t *s_u, *s_cnt;
        uint64_t *tmp_ids;
        int8_t *s_d, *tmp_d;
        PASTIS_TRY(get(ctx, kDSu, (size_t)nu * W, &s_u));
        PASTIS_TRY(get(ctx, kDSd, (size_t)nu * W, &s_d));
        PASTIS_TRY(get(ctx, kDScnt, (size_t)nu, &s_cnt));
        PASTIS_TRY(get(ctx, kDStmpIds, (size_t)s_rows_threads() * P.n_subs, &tmp_ids));
        PASTIS_TRY(get(ctx, kDStmpD, (size_t)s_rows_threads() * P.n_subs, &tmp_d));
        HIP_TRY(ctx,
                launch_s_rows(kt.uk_id, kt.counts + 1, kt.uk_start, kt.kmap, ctx->d_blosum, P.k, P.n_subs,
                              P.sub_alphabet, s_u, s_d, s_cnt, tmp_ids, tmp_d, s),
                "S kernel");
        AsArgs as{};
        as.kt = &kt;
        as.s_u = s_u;
        as.s_d = s_d;
        as.s_cnt = s_cnt;
        as.W = W;
        as.n = n;
        PASTIS_TRY(get(ctx, kDAsUb, n, &as.ub));
        PASTIS_TRY(get(ctx, kDAsStart, n + 1, &as.as_start));
        PASTIS_TRY(get(ctx, kDAsLen, n, &as.as_len));
        PASTIS_TRY(get(ctx, kBufBinOf, n, &as.bin_of));
        as.bins = BinBufs{M.bin_meta, M.bin_meta + 32, M.bin_meta + 64, nullptr};
        PASTIS_TRY(get(ctx, kBufIdx, n, &as.bins.idx));
        as.max_ub = M.max_ub;
        as.scan_temp = temp;
        HIP_TRY(ctx, as_stage(as, s), "A S plan");
        // nnz(S): the kept slots of every row (the k-mer itself and its
        // present substitutes), for the discovery's traffic accounting
        HIP_TRY(ctx, fill<unsigned long long>(M.nnz_s, 1, 0ull, s), "reset");
        if (nu > 0) {
            sum_u32_kernel<<<grid_for(nu), 256, 0, s>>>(s_cnt, nu, M.nnz_s);
            HIP_TRY(ctx, hipGetLastError(), "sum kernel");
        }
        unsigned long long nnz_s = 0;
        PASTIS_TRY(read_device(ctx, M.nnz_s, &nnz_s, sizeof(nnz_s), s));
        ctx->stats.n_subs_entries = (int64_t)nnz_s;
        uint64_t tot = 0;
        unsigned long long mx = 0;
        PASTIS_TRY(read_device(ctx, as.as_start + n, &tot, sizeof(tot), s));
        PASTIS_TRY(read_device(ctx, M.max_ub, &mx, sizeof(mx), s));
        PASTIS_TRY(get(ctx, kDAsS, tot, &as.as_s));
        PASTIS_TRY(get(ctx, kDAsDp, tot, &as.as_dp));
        uint32_t gcap = 0;
        as.global_blocks = 256;
        if (mx > 0) {
            gcap = next_pow2(2 * mx);
            as.global_blocks = (int)std::max<int64_t>(8, std::min<int64_t>(256, (int64_t)(2ll << 30) / (8ll * gcap)));
            PASTIS_TRY(get(ctx, kDAsGtab, (size_t)as.global_blocks * 2 * gcap, &as.gtables));
        }
        HIP_TRY(ctx, as_run(as, gcap, s), "A S kernels");
        HIP_TRY(ctx, stage_end(ctx, kStSubs, s), "event");
        sp.row_start64 = as.as_start;
        sp.row_len = as.as_len;
        sp.ent_s = as.as_s;
        sp.ent_dp = as.as_dp;
    } else {
        sp.row_start32 = kt.row_start;
        sp.ent_s = kt.row_h;
        sp.ent_len = kt.row_len;
        sp.ent_pos16 = kt.row_pos;
    }
    return PASTIS_OK;
}

// Discovery, second part: the candidate pairs (lo, hi) with r0 <= lo < r1
// into kBufCand*, sorted by (lo, hi); their count in *n_cand_out.  A block
// whose directional entries would exceed `limit` sets *split_need to the
// entries it asked for (when it may be split and holds more than one
// sequence) and produces nothing; otherwise such a block fails with
// PASTIS_E_CAPACITY.
pastis_status discover_block(pastis_ctx *ctx, DiscTables &dt, int64_t n, int64_t r0, int64_t r1, uint64_t limit,
                             bool may_split, hipStream_t s, int64_t *n_cand_out, uint64_t *split_need) {
    const pastis_params &P = ctx->params;
    Misc M;
    PASTIS_TRY(misc(ctx, M));
    const int64_t nnz = dt.nnz, nu = dt.nu;
    SpgemmArgs sp = dt.sp;
    sp.kt = &dt.kt;
    sp.blk_lo = (uint32_t)r0;
    sp.blk_hi = (uint32_t)r1;
    if (split_need) *split_need = 0;

    // ---- sparse product
    HIP_TRY(ctx, stage_begin(ctx, kStSpgemm, s), "event");
    PASTIS_TRY(get(ctx, kDWork, n, &sp.work));
    PASTIS_TRY(get(ctx, kBufBinOf, n, &sp.bin_of));
    sp.bins = BinBufs{M.bin_meta, M.bin_meta + 32, M.bin_meta + 64, nullptr};
    PASTIS_TRY(get(ctx, kBufIdx, n, &sp.bins.idx));
    sp.max_big = M.max_big;
    sp.products = M.products;
    PASTIS_TRY(get(ctx, kDBigRows, n, &sp.big_rows));
    PASTIS_TRY(get(ctx, kDPostRec, nnz + nu, &sp.post_rec));
    PASTIS_TRY(get(ctx, kDStage, spgemm_stage_entries(), &sp.stage));
    sp.nnz = nnz;
    sp.n_big = M.n_big;
    sp.d_count = M.d_count;
    sp.d_overflow = M.d_overflow;
    sp.nbits = key_bits(n);
    HIP_TRY(ctx, spgemm_plan(sp, s), "product plan");
    unsigned long long mxw = 0, prods = 0;
    PASTIS_TRY(read_device(ctx, M.max_big, &mxw, sizeof(mxw), s));
    PASTIS_TRY(read_device(ctx, M.products, &prods, sizeof(prods), s));
    ctx->stats.spgemm_products = (int64_t)prods;
    const uint32_t gcap = next_pow2(2 * std::max<unsigned long long>(mxw, 12288ull));
    // tables of the big rows: up to 8 GiB, at most 512 blocks
    sp.global_blocks = (int)std::max<int64_t>(8, std::min<int64_t>(512, (int64_t)(8ll << 30) / (24ll * gcap)));
    PASTIS_TRY(get(ctx, kDGtab, (size_t)sp.global_blocks * gcap, &sp.gtables));
    PASTIS_TRY(get(ctx, kDGcand, (size_t)sp.global_blocks * 2 * gcap, &sp.gcand));
    // Room for the directional entries: every entry takes at least ck_min
    // products, so products / ck_min bounds them; that bound is used when its
    // buffers stay within 6 GiB (24 bytes an entry), else the last call's
    // count plus a quarter.  A run that still overflows is redone with room
    // for all of its entries.
    const uint64_t dir_ub = prods / (uint64_t)std::max(1, sp.ck) + 1024;
    uint64_t want = std::max<uint64_t>({(uint64_t)4 * n, 1ull << 20, ctx->last_n_dir + ctx->last_n_dir / 4});
    if (dir_ub <= (1ull << 28)) want = std::max(want, dir_ub);
    if (P.candidate_room > 0) want = (uint64_t)P.candidate_room;  // the caller's setting
    limit = std::min(limit, kMaxDir);
    uint32_t cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>({want, dir_ub, limit}));
    for (int attempt = 0;; ++attempt) {
        sp.cap = cap;
        PASTIS_TRY(get(ctx, kDDirKey, cap, &sp.d_key));
        PASTIS_TRY(get(ctx, kDDirCnt, cap, &sp.d_cnt));
        PASTIS_TRY(get(ctx, kDDirS1, cap, &sp.d_s1));
        PASTIS_TRY(get(ctx, kDDirS2, cap, &sp.d_s2));
        PASTIS_TRY(get(ctx, kDDirDir, cap, &sp.d_dir));
        // the spill counter (second word) is reset so each attempt starts clean
        HIP_TRY(ctx, fill<uint32_t>(sp.n_big + 1, 1, 0u, s), "reset");
        uint32_t nb0 = 0;
        PASTIS_TRY(read_device(ctx, sp.n_big, &nb0, sizeof(nb0), s));
        HIP_TRY(ctx, spgemm_run(sp, gcap, s), "product kernels");
        uint32_t ovf = 0;
        PASTIS_TRY(read_device(ctx, M.d_overflow, &ovf, sizeof(ovf), s));
        if (!ovf) break;
        // the 64-bit counter holds every entry the run asked for, so one redo
        // with that much room succeeds; a count beyond the limit cannot
        unsigned long long need = 0;
        PASTIS_TRY(read_device(ctx, M.d_count, &need, sizeof(need), s));
        if (need > limit && may_split && r1 - r0 > 1) {
            HIP_TRY(ctx, stage_end(ctx, kStSpgemm, s), "event");
            *split_need = need;
            *n_cand_out = 0;
            return PASTIS_OK;
        }
        if (need > limit || attempt >= 2)
            return set_error(ctx, PASTIS_E_CAPACITY,
                             "candidate discovery produced " + std::to_string(need) +
                                 " directional entries; at most " + std::to_string(limit) +
                                 " fit one block (raise block_entries or ck_min, or split the sequences)");
        cap = (uint32_t)std::min<uint64_t>(need + need / 4 + 1024, limit);
        // redo from the planned state: restore the big-row count of the plan
        HIP_TRY(ctx, fill<uint32_t>(sp.n_big, 1, nb0, s), "reset");
    }
    unsigned long long n_dir64 = 0;
    PASTIS_TRY(read_device(ctx, M.d_count, &n_dir64, sizeof(n_dir64), s));
    const uint32_t n_dir = (uint32_t)n_dir64;  // <= cap <= kMaxDir after a run without overflow
    ctx->last_n_dir = n_dir;

    // ---- symmetrise, sort, threshold already applied
    SymArgs sy{};
    sy.n_dir = n_dir;
    sy.d_ndir = (const uint32_t *)M.d_count;  // low word (little-endian), below 2^32 here
    sy.key = sp.d_key;
    PASTIS_TRY(get(ctx, kDDirKeyAlt, n_dir, &sy.key_alt));
    PASTIS_TRY(get(ctx, kDPerm, n_dir, &sy.perm));
    PASTIS_TRY(get(ctx, kDPermAlt, n_dir, &sy.perm_alt));
    sy.cnt = sp.d_cnt;
    sy.s1 = sp.d_s1;
    sy.s2 = sp.d_s2;
    sy.dir = sp.d_dir;
    PASTIS_TRY(get(ctx, kDFlag, n_dir, &sy.flag));
    PASTIS_TRY(get(ctx, kDPick, n_dir, &sy.pick));
    PASTIS_TRY(get(ctx, kDOpos, n_dir, &sy.opos));
    sy.d_ncand = M.n_cand;
    sy.nbits = sp.nbits;
    PASTIS_TRY(get(ctx, kDTemp, std::max(dt.temp_bytes, radix_temp_bytes(n_dir) + scan_temp_bytes(n_dir)),
                   (char **)&sy.sort_temp));
    PASTIS_TRY(get(ctx, kBufCandLo, n_dir, &sy.out.lo));
    PASTIS_TRY(get(ctx, kBufCandHi, n_dir, &sy.out.hi));
    PASTIS_TRY(get(ctx, kBufCandCnt, n_dir, &sy.out.count));
    PASTIS_TRY(get(ctx, kBufCandS1, n_dir, &sy.out.seed1));
    PASTIS_TRY(get(ctx, kBufCandS2, n_dir, &sy.out.seed2));
    if (n_dir > 0) {
        HIP_TRY(ctx, symmetrise(sy, s), "symmetrise");
    } else {
        HIP_TRY(ctx, fill<uint32_t>(M.n_cand, 1, 0u, s), "reset");
    }
    HIP_TRY(ctx, stage_end(ctx, kStSpgemm, s), "event");
    uint32_t nc = 0;
    PASTIS_TRY(read_device(ctx, M.n_cand, &nc, sizeof(nc), s));
    *n_cand_out = nc;
    ctx->stats.n_candidates = nc;
    ctx->n_candidates = nc;
    ctx->n_seqs_last = n;
    ctx->have_candidates = true;
    return PASTIS_OK;
}

// Discovery of every candidate pair at once.
pastis_status discover(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, hipStream_t s,
                       int64_t *n_cand_out) {
    DiscTables dt;
    PASTIS_TRY(discover_tables(ctx, st, codes, n, s, dt));
    return discover_block(ctx, dt, n, 0, n, kMaxDir, false, s, n_cand_out, nullptr);
}

// Counts of one row block that a search in several blocks adds up (stage
// times add up in ms_stage by themselves; per-bin shapes are the same in
// every block).
using StatCount = int64_t pastis_run_stats::*;
constexpr StatCount kBlockCounts[] = {
    &pastis_run_stats::n_candidates,     &pastis_run_stats::n_aligned,        &pastis_run_stats::n_edges,
    &pastis_run_stats::cells,            &pastis_run_stats::stats_pass_pairs, &pastis_run_stats::int32_pairs,
    &pastis_run_stats::bound_pass_pairs, &pastis_run_stats::bound_pass_cells, &pastis_run_stats::stats_pass_cells,
    &pastis_run_stats::spgemm_products};

void clear_block_stats(pastis_run_stats &b) {
    for (StatCount m : kBlockCounts) b.*m = 0;
    for (int i = 0; i < 32; ++i) {
        b.sw_bin_pairs[i] = 0;
        b.sw_bin_cells[i] = 0;
        b.sw_bin_ms[i] = 0.0;
    }
}

void add_block_stats(pastis_run_stats &acc, const pastis_run_stats &b) {
    for (StatCount m : kBlockCounts) acc.*m += b.*m;
    acc.sw_bins = b.sw_bins;
    acc.sw_graph = b.sw_graph;
    for (int i = 0; i < 32; ++i) {
        acc.sw_bin_rows[i] = b.sw_bin_rows[i];
        acc.sw_bin_multi[i] = b.sw_bin_multi[i];
        acc.sw_bin_bits[i] = b.sw_bin_bits[i];
        acc.sw_bin_pairs[i] += b.sw_bin_pairs[i];
        acc.sw_bin_cells[i] += b.sw_bin_cells[i];
        acc.sw_bin_ms[i] += b.sw_bin_ms[i];
    }
}

void set_block_stats(pastis_run_stats &dst, const pastis_run_stats &acc) {
    for (StatCount m : kBlockCounts) dst.*m = acc.*m;
    dst.sw_bins = acc.sw_bins;
    dst.sw_graph = acc.sw_graph;
    for (int i = 0; i < 32; ++i) {
        dst.sw_bin_rows[i] = acc.sw_bin_rows[i];
        dst.sw_bin_multi[i] = acc.sw_bin_multi[i];
        dst.sw_bin_bits[i] = acc.sw_bin_bits[i];
        dst.sw_bin_pairs[i] = acc.sw_bin_pairs[i];
        dst.sw_bin_cells[i] = acc.sw_bin_cells[i];
        dst.sw_bin_ms[i] = acc.sw_bin_ms[i];
    }
}

pastis_status begin_call(pastis_ctx *ctx) {
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->bad_residue = -1;
    ctx->stats = pastis_run_stats{};
    ctx->last_error.clear();
    return PASTIS_OK;
}

pastis_status stage_and_encode(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                               int on_device, hipStream_t s, Staged &st, uint8_t **codes) {
    PASTIS_TRY(stage_sequences(ctx, residues, offsets, n, on_device, s, st));
    unsigned long long *d_flags = nullptr, h_flags[4];
    PASTIS_TRY(reset_flags(ctx, &d_flags, s));
    HIP_TRY(ctx, stage_begin(ctx, kStEncode, s), "event");
    PASTIS_TRY(encode_into(ctx, st.d_res, st.n_res, codes, d_flags, s));
    HIP_TRY(ctx, stage_end(ctx, kStEncode, s), "event");
    PASTIS_TRY(read_flags(ctx, d_flags, h_flags, 1, s));
    if (h_flags[0] != ~0ull) {
        ctx->bad_residue = (int64_t)h_flags[0];
        return set_error(ctx, PASTIS_E_BAD_RESIDUE, "bad residue at index " + std::to_string(h_flags[0]));
    }
    ctx->stats.n_sequences = n;
    ctx->stats.n_residues = st.n_res;
    return PASTIS_OK;
}

}  // namespace

pastis_status mlp_filter_candidates(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n,
                                   hipStream_t s);

// The tuner's sample keeps every candidate whose shorter sequence (the
// alignment's rows) falls in a hashed subset of the sequences: the 16-bit
// pass groups pairs that share that sequence, and an even stride through
// the candidates would thin those groups out and misjudge the grouping.
__device__ __forceinline__ uint32_t seq_hash(uint32_t v) {
    uint32_t h = v * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    return h ^ (h >> 13);
}

__global__ void tune_flag_kernel(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                 const int64_t *__restrict__ offsets, int64_t nc, uint64_t thr,
                                 uint8_t *__restrict__ flag) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = lo[c], j = hi[c];  // i < j
        const int64_t li = offsets[i + 1] - offsets[i], lj = offsets[j + 1] - offsets[j];
        const uint32_t a = lj < li ? j : i;  // rows: the shorter, the lower index on a tie
        flag[c] = (uint64_t)seq_hash(a) < thr ? 1 : 0;
    }
}

__global__ void tune_sample_kernel(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                   const uint32_t *__restrict__ s1, const uint32_t *__restrict__ s2,
                                   const uint8_t *__restrict__ flag, const uint32_t *__restrict__ pos, int64_t nc,
                                   int64_t m, uint32_t *__restrict__ olo, uint32_t *__restrict__ ohi,
                                   uint32_t *__restrict__ os1, uint32_t *__restrict__ os2) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[c]) continue;
        const uint32_t q = pos[c];
        if (q >= (uint64_t)m) continue;
        olo[q] = lo[c];
        ohi[q] = hi[c];
        os1[q] = s1[c];
        os2[q] = s2[c];
    }
}

// Align the ctx's current candidates; records into kDRecords.
pastis_status align_candidates(pastis_ctx *ctx, const Staged &st, const uint8_t *codes, int64_t n, hipStream_t s,
                               pastis_pair_record **rec_out);

}  // namespace pastis

using namespace pastis;

extern "C" {

pastis_status pastis_discover(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int input_on_device, void *stream, int64_t *n_candidates) {
    if (!ctx || !n_candidates) return PASTIS_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    PASTIS_TRY(begin_call(ctx));
    ctx->have_candidates = false;
    Staged st;
    uint8_t *codes = nullptr;
    PASTIS_TRY(stage_and_encode(ctx, residues, offsets, n, input_on_device, s, st, &codes));
    PASTIS_TRY(discover(ctx, st, codes, n, s, n_candidates));
    HIP_TRY(ctx, stage_collect(ctx, s), "sync");
    ctx->stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PASTIS_OK;
}

pastis_status pastis_candidates_copy(pastis_ctx *ctx, uint32_t *lo, uint32_t *hi, uint32_t *count, uint32_t *seed1,
                                     uint32_t *seed2, int64_t cap, int dst_on_device, void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    if (!ctx->have_candidates) return set_error(ctx, PASTIS_E_STATE, "no candidates: call pastis_discover first");
    const int64_t nc = ctx->n_candidates;
    if (cap < nc) return set_error(ctx, PASTIS_E_CAPACITY, "candidate buffers too small");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int ids[5] = {kBufCandLo, kBufCandHi, kBufCandCnt, kBufCandS1, kBufCandS2};
    uint32_t *dst[5] = {lo, hi, count, seed1, seed2};
    for (int f = 0; f < 5; ++f) {
        if (!dst[f] || nc == 0) continue;
        HIP_TRY(ctx, hipMemcpyAsync(dst[f], ctx->buf[ids[f]].ptr, sizeof(uint32_t) * nc, kind, s), "copy");
    }
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status pastis_subkmers(pastis_ctx *ctx, const uint64_t *kmer_ids, int64_t n, uint64_t *out_ids,
                              int32_t *out_dist, int32_t *out_count, void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!kmer_ids || !out_ids || !out_dist || !out_count))) return PASTIS_E_INVAL;
    const pastis_params &P = ctx->params;
    if (P.n_subs <= 0) return set_error(ctx, PASTIS_E_INVAL, "n_subs must be > 0");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (n == 0) return PASTIS_OK;
    int8_t *d8 = nullptr;
    PASTIS_TRY(get(ctx, kDSubD, (size_t)n * P.n_subs, &d8));
    HIP_TRY(ctx, launch_nearest_ids(kmer_ids, n, ctx->d_blosum, P.k, P.n_subs, P.sub_alphabet, out_ids, d8, out_count, s),
            "neighbourhood kernel");
    // widen distances to int32 on the host side of the copy
    std::vector<int8_t> h8((size_t)n * P.n_subs);
    PASTIS_TRY(read_device(ctx, d8, h8.data(), h8.size(), s));
    std::vector<int32_t> h32(h8.begin(), h8.end());
    HIP_TRY(ctx, hipMemcpyAsync(out_dist, h32.data(), sizeof(int32_t) * h32.size(), hipMemcpyHostToDevice, s), "copy");
    HIP_TRY(ctx, hipStreamSynchronize(s), "sync");
    return PASTIS_OK;
}

pastis_status pastis_search(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                            int input_on_device, void *stream, pastis_result **out) {
    if (!ctx || !out) return PASTIS_E_INVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    PASTIS_TRY(begin_call(ctx));
    ctx->have_candidates = false;
    Staged st;
    uint8_t *codes = nullptr;
    PASTIS_TRY(stage_and_encode(ctx, residues, offsets, n, input_on_device, s, st, &codes));
    DiscTables dt;
    PASTIS_TRY(discover_tables(ctx, st, codes, n, s, dt));
    Misc M;
    PASTIS_TRY(misc(ctx, M));
    const int ns = ctx->params.weight_mode == PASTIS_WEIGHT_NS;
    const uint64_t limit = ctx->params.block_entries > 0 ? (uint64_t)ctx->params.block_entries : kMaxDir;
    // Row blocks (the pairs whose lower index falls in [r0, r1)), the next
    // one last.  A block whose discovery would exceed the limit is split;
    // blocks run in order of r0, so their edges, each sorted, concatenate
    // into the sorted edge list.
    std::vector<std::pair<int64_t, int64_t>> todo{{0, n}};
    struct Parts {
        std::vector<std::pair<pastis_edge *, int64_t>> v;
        ~Parts() {
            for (auto &p : v)
                if (p.first) (void)hipFree(p.first);
        }
    } parts;
    pastis_run_stats acc{};
    int64_t n_edges = 0, n_blocks = 0;
    while (!todo.empty()) {
        const std::pair<int64_t, int64_t> blk = todo.back();
        todo.pop_back();
        clear_block_stats(ctx->stats);
        int64_t nc = 0;
        uint64_t need = 0;
        PASTIS_TRY(discover_block(ctx, dt, n, blk.first, blk.second, limit, true, s, &nc, &need));
        if (need) {
            // split into enough parts for the entries it asked for, with a
            // quarter to spare, at rows that give each part an equal share of
            // pairs if those spread evenly (row x is the lower index of about
            // n - 1 - x pairs); a part that still overflows is split again
            const int64_t r0 = blk.first, r1 = blk.second;
            const int64_t k = std::max<int64_t>(
                2, std::min<int64_t>(r1 - r0, (int64_t)std::ceil(1.25 * (double)need / (double)limit)));
            auto area = [&](int64_t x) { return 0.5 * (double)(x - r0) * (double)(2 * n - r0 - x + 1); };
            std::vector<int64_t> cut{r0};
            for (int64_t i = 1; i < k; ++i) {
                const double target = area(r1) * (double)i / (double)k;
                int64_t lo_x = cut.back() + 1, hi_x = r1 - (k - i);  // leave a row for each later part
                while (lo_x < hi_x) {
                    const int64_t mid = lo_x + (hi_x - lo_x) / 2;
                    if (area(mid) >= target)
                        hi_x = mid;
                    else
                        lo_x = mid + 1;
                }
                cut.push_back(lo_x);
            }
            cut.push_back(r1);
            for (size_t i = cut.size() - 1; i > 0; --i) todo.push_back({cut[i - 1], cut[i]});
            continue;
        }
        ++n_blocks;
        if (ctx->params.filter_mode == 1) {
            PASTIS_TRY(mlp_filter_candidates(ctx, st, codes, n, s));
            nc = ctx->n_candidates;
        }
        pastis_pair_record *rec = nullptr;
        PASTIS_TRY(align_candidates(ctx, st, codes, n, s, &rec));
        // edges
        HIP_TRY(ctx, stage_begin(ctx, kStFilter, s), "event");
        uint8_t *flag = nullptr;
        uint32_t *pos = nullptr;
        PASTIS_TRY(get(ctx, kDEdgeFlag, nc, &flag));
        PASTIS_TRY(get(ctx, kDEdgePos, nc, &pos));
        char *temp = nullptr;
        PASTIS_TRY(get(ctx, kDTemp, std::max(dt.temp_bytes, scan_temp_bytes(nc) + 4096), &temp));
        if (nc > 0) {
            edge_flag_kernel<<<grid_for(nc), 256, 0, s>>>(rec, nc, ns, flag);
            HIP_TRY(ctx, hipGetLastError(), "edge kernel");
        }
        HIP_TRY(ctx, (exclusive_scan<uint8_t, uint32_t>(flag, nc, pos, M.n_edges, temp, s)), "scan");
        uint32_t ne = 0;
        PASTIS_TRY(read_device(ctx, M.n_edges, &ne, sizeof(ne), s));
        pastis_edge *d = nullptr;
        if (ne > 0) {
            if (hipMalloc(&d, sizeof(pastis_edge) * ne) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(ctx, PASTIS_E_NOMEM, "edge allocation failed");
            }
            parts.v.push_back({d, (int64_t)ne});
            edge_write_kernel<<<grid_for(nc), 256, 0, s>>>(
                rec, flag, pos, nc, (const uint32_t *)ctx->buf[kBufCandLo].ptr,
                (const uint32_t *)ctx->buf[kBufCandHi].ptr, (const uint32_t *)ctx->buf[kBufCandCnt].ptr, st.d_off, ns,
                d);
            HIP_TRY(ctx, hipGetLastError(), "edge kernel");
        }
        HIP_TRY(ctx, stage_end(ctx, kStFilter, s), "event");
        HIP_TRY(ctx, stage_collect(ctx, s), "sync");
        ctx->stats.n_edges = ne;
        n_edges += ne;
        add_block_stats(acc, ctx->stats);
        // the candidate buffers keep only the last block's pairs
        if (blk.first > 0 || blk.second < n) ctx->have_candidates = false;
    }
    set_block_stats(ctx->stats, acc);
    ctx->stats.n_row_blocks = n_blocks;
    pastis_result *res = new pastis_result();
    res->device = ctx->device;
    res->n = n_edges;
    if (parts.v.size() == 1) {
        res->d_edges = parts.v[0].first;
        parts.v[0].first = nullptr;
    } else if (n_edges > 0) {
        if (hipMalloc(&res->d_edges, sizeof(pastis_edge) * n_edges) != hipSuccess) {
            (void)hipGetLastError();
            delete res;
            return set_error(ctx, PASTIS_E_NOMEM, "edge allocation failed");
        }
        int64_t at = 0;
        for (auto &p : parts.v) {
            const hipError_t e = hipMemcpyAsync(res->d_edges + at, p.first, sizeof(pastis_edge) * p.second,
                                                hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) {
                (void)hipFree(res->d_edges);
                delete res;
                return hip_error(ctx, e, "copy");
            }
            at += p.second;
        }
        const hipError_t e = hipStreamSynchronize(s);  // before the parts are freed
        if (e != hipSuccess) {
            (void)hipFree(res->d_edges);
            delete res;
            return hip_error(ctx, e, "sync");
        }
    }
    ctx->stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = res;
    return PASTIS_OK;
}

pastis_status pastis_mlp_collect(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                 int input_on_device, const pastis_params *discovery, void *stream,
                                 int64_t *n_added) {
    if (!ctx) return PASTIS_E_INVAL;
    if (n_added) *n_added = 0;
    hipStream_t s = (hipStream_t)stream;
    // this collection's discovery parameters, and an alignment that only
    // decides the cut (no filter, no graph, records kept inside)
    struct Restore {
        pastis_ctx *c;
        pastis_params p;
        ~Restore() { c->params = p; }
    } restore{ctx, ctx->params};
    pastis_params &P = ctx->params;
    if (discovery) {
        if (discovery->k < 1 || discovery->k > kMaxK) return set_error(ctx, PASTIS_E_INVAL, "discovery k out of range");
        if (discovery->n_subs < 0 || discovery->n_subs > 64)
            return set_error(ctx, PASTIS_E_INVAL, "discovery n_subs must be in 0..64");
        if (discovery->sub_alphabet != 20 && discovery->sub_alphabet != 24)
            return set_error(ctx, PASTIS_E_INVAL, "discovery sub_alphabet must be 20 or 24");
        if (discovery->ck_min < 1) return set_error(ctx, PASTIS_E_INVAL, "discovery ck_min must be >= 1");
        P.k = discovery->k;
        P.n_subs = discovery->n_subs;
        P.sub_alphabet = discovery->sub_alphabet;
        P.ck_min = discovery->ck_min;
    }
    P.weight_mode = PASTIS_WEIGHT_ANI;
    P.filter_mode = 0;
    P.full_records = 0;
    P.graph_mode = 0;
    auto t0 = std::chrono::steady_clock::now();
    PASTIS_TRY(begin_call(ctx));
    ctx->have_candidates = false;
    Staged st;
    uint8_t *codes = nullptr;
    PASTIS_TRY(stage_and_encode(ctx, residues, offsets, n, input_on_device, s, st, &codes));
    int64_t nc = 0;
    PASTIS_TRY(discover(ctx, st, codes, n, s, &nc));
    pastis_pair_record *rec = nullptr;
    PASTIS_TRY(align_candidates(ctx, st, codes, n, s, &rec));
    int64_t added = 0;
    PASTIS_TRY(mlp_pool_append(ctx, st, codes, n, rec, s, &added));
    HIP_TRY(ctx, stage_collect(ctx, s), "sync");
    ctx->stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (n_added) *n_added = added;
    return PASTIS_OK;
}

pastis_status pastis_result_count(const pastis_result *r, int64_t *n_edges) {
    if (!r || !n_edges) return PASTIS_E_INVAL;
    *n_edges = r->n;
    return PASTIS_OK;
}

const pastis_edge *pastis_result_device_ptr(const pastis_result *r) { return r ? r->d_edges : nullptr; }

pastis_status pastis_result_copy(const pastis_result *r, pastis_edge *dst, int64_t cap, int dst_on_device,
                                 void *stream) {
    if (!r || (r->n > 0 && !dst)) return PASTIS_E_INVAL;
    if (cap < r->n) return PASTIS_E_CAPACITY;
    if (r->n == 0) return PASTIS_OK;
    if (hipSetDevice(r->device) != hipSuccess) return PASTIS_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(dst, r->d_edges, sizeof(pastis_edge) * r->n,
                       dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s) != hipSuccess)
        return PASTIS_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PASTIS_E_DEVICE;
    return PASTIS_OK;
}

void pastis_result_free(pastis_result *r) {
    if (!r) return;
    if (r->d_edges) {
        (void)hipSetDevice(r->device);
        (void)hipFree(r->d_edges);
    }
    delete r;
}

}  // extern "C"

extern "C" {

pastis_status pastis_get_tuning(const pastis_ctx *ctx, pastis_tuning *out) {
    if (!ctx || !out) return PASTIS_E_INVAL;
    *out = ctx->tune;
    return PASTIS_OK;
}

pastis_status pastis_set_tuning(pastis_ctx *ctx, const pastis_tuning *t) {
    if (!ctx || !t) return PASTIS_E_INVAL;
    if (t->sw16_max_rows < 0 || t->sw16_max_rows > 16 || t->sw_direct_pct < 0 || t->sw_grid_scale < 1 ||
        t->sw_grid_scale > 64 || t->sw_grid_scale_wide < 1 || t->sw_grid_scale_wide > 64 || t->sw_intra_pair < 0 ||
        t->sw_intra_pair > 1 || t->sw16_narrow_rows < 0 || t->sw16_narrow_rows > 4 || t->sw_long_blocks < 1 ||
        t->sw_long_blocks > 4)
        return set_error(ctx, PASTIS_E_INVAL, "tuning value out of range");
    for (int i = 0; i < 1; ++i)
        if (t->reserved[i] != 0) return set_error(ctx, PASTIS_E_INVAL, "reserved fields must be zero");
    ctx->tune = *t;
    return PASTIS_OK;
}

pastis_status pastis_autotune(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int input_on_device, int64_t max_pairs, void *stream, pastis_tuning *out) {
    if (!ctx || max_pairs < 1) return PASTIS_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    PASTIS_TRY(begin_call(ctx));
    Staged st;
    uint8_t *codes = nullptr;
    PASTIS_TRY(stage_and_encode(ctx, residues, offsets, n, input_on_device, s, st, &codes));
    int64_t nc = 0;
    PASTIS_TRY(discover(ctx, st, codes, n, s, &nc));
    if (nc > 0 && ctx->params.align_mode == PASTIS_ALIGN_SW) {
        const int64_t cap = std::min<int64_t>(nc, max_pairs);
        uint32_t *lo, *hi, *s1, *s2, *pos;
        uint8_t *flag;
        char *temp;
        pastis_pair_record *rec;
        PASTIS_TRY(get(ctx, kDTuneLo, cap, &lo));
        PASTIS_TRY(get(ctx, kDTuneHi, cap, &hi));
        PASTIS_TRY(get(ctx, kDTuneS1, cap, &s1));
        PASTIS_TRY(get(ctx, kDTuneS2, cap, &s2));
        PASTIS_TRY(get(ctx, kDTuneRec, cap, &rec));
        PASTIS_TRY(get(ctx, kDEdgeFlag, nc, &flag));
        PASTIS_TRY(get(ctx, kDEdgePos, nc + 1, &pos));
        PASTIS_TRY(get(ctx, kDTemp, scan_temp_bytes(nc) + 4096, &temp));
        // sequences kept with probability cap / nc (all of them when cap >= nc)
        const uint64_t thr = cap >= nc ? (1ull << 32) : (uint64_t)(4294967296.0 * (double)cap / (double)nc);
        const uint32_t *clo = (const uint32_t *)ctx->buf[kBufCandLo].ptr, *chi = (const uint32_t *)ctx->buf[kBufCandHi].ptr;
        tune_flag_kernel<<<grid_for(nc), 256, 0, s>>>(clo, chi, st.d_off, nc, thr, flag);
        HIP_TRY(ctx, hipGetLastError(), "sample kernel");
        HIP_TRY(ctx, (exclusive_scan<uint8_t, uint32_t>(flag, nc, pos, pos + nc, temp, s)), "scan");
        tune_sample_kernel<<<grid_for(nc), 256, 0, s>>>(clo, chi, (const uint32_t *)ctx->buf[kBufCandS1].ptr,
                                                       (const uint32_t *)ctx->buf[kBufCandS2].ptr, flag, pos, nc, cap,
                                                       lo, hi, s1, s2);
        HIP_TRY(ctx, hipGetLastError(), "sample kernel");
        uint32_t total = 0;
        PASTIS_TRY(read_device(ctx, pos + nc, &total, sizeof(total), s));
        const int64_t m = std::min<int64_t>(cap, total);
        if (m == 0) {
            if (out) *out = ctx->tune;
            return PASTIS_OK;
        }
        // time one alignment of the sample under the current ctx->tune
        auto time_once = [&](double *ms) -> pastis_status {
            ctx->stats = pastis_run_stats{};
            ctx->records_internal = true;
            const pastis_status r = align_core(ctx, st, codes, n, lo, hi, s1, s2, m, rec, s);
            ctx->records_internal = false;
            PASTIS_TRY(r);
            HIP_TRY(ctx, stage_collect(ctx, s), "sync");
            *ms = ctx->stats.ms_stage[kStSched] + ctx->stats.ms_stage[kStAlign1] + ctx->stats.ms_stage[kStAlign2];
            return PASTIS_OK;
        };
        auto measure = [&](double *best) -> pastis_status {
            double a = 0, b = 0;
            PASTIS_TRY(time_once(&a));
            PASTIS_TRY(time_once(&b));
            *best = std::min(a, b);
            return PASTIS_OK;
        };
        double cur = 0;
        PASTIS_TRY(measure(&cur));  // warms the buffers up
        const int rows16[] = {16, 12, 8, 0};
        const int direct[] = {0, 25, 50, 75, 100, 200, 1 << 20};
        const int grid[] = {1, 2, 4};
        // a value replaces the one in force only when it is at least 1%
        // faster on the sample: smaller differences are within timing noise
        // and need not carry over to the whole candidate set.  The value in
        // force is timed again first, so each knob's values are compared
        // under the same conditions (clocks, caches) rather than against a
        // figure taken several sweeps earlier.
        auto sweep = [&](int32_t *knob, const int *vals, int nv) -> pastis_status {
            const int32_t keep = *knob;
            int32_t best_v = keep;
            PASTIS_TRY(measure(&cur));
            double best_ms = cur;
            for (int i = 0; i < nv; ++i) {
                if (vals[i] == keep) continue;
                *knob = vals[i];
                double ms = 0;
                PASTIS_TRY(measure(&ms));
                if (ms < 0.99 * best_ms) {
                    best_ms = ms;
                    best_v = vals[i];
                }
            }
            *knob = best_v;
            cur = best_ms;
            return PASTIS_OK;
        };
        PASTIS_TRY(sweep(&ctx->tune.sw16_max_rows, rows16, 4));
        PASTIS_TRY(sweep(&ctx->tune.sw_direct_pct, direct, 7));
        PASTIS_TRY(sweep(&ctx->tune.sw_grid_scale, grid, 3));
        PASTIS_TRY(sweep(&ctx->tune.sw_grid_scale_wide, grid, 3));
        const int intra[] = {0, 1};
        PASTIS_TRY(sweep(&ctx->tune.sw_intra_pair, intra, 2));
        const int narrow[] = {4, 2, 0};
        PASTIS_TRY(sweep(&ctx->tune.sw16_narrow_rows, narrow, 3));
        const int longb[] = {4, 2, 1};
        PASTIS_TRY(sweep(&ctx->tune.sw_long_blocks, longb, 3));
        // The knobs whose best value depends on the tails of the launches
        // (the start-bound routing, and inter- vs intra-pair mode and the grid
        // of the multi-strip bins, whose few long pairs set those tails) are
        // refined on the whole candidate set, since a sample shortens the
        // tails: on the large workload a 2M-pair sample chose 25% routing,
        // and all 8.9M candidates run 1% faster at 75%.  One warm-up run at
        // the full size, then one run per value; a value replaces the one in
        // force when at least 0.5% faster (whole-set runs vary less than
        // sample runs).  Sets of over 2^26 candidates (3 GB of records) are
        // not refined.
        if (m < nc && nc <= ((int64_t)1 << 26)) {
            pastis_pair_record *rec_all = nullptr;
            PASTIS_TRY(get(ctx, kDTuneRec, nc, &rec_all));
            const uint32_t *cs1 = (const uint32_t *)ctx->buf[kBufCandS1].ptr;
            const uint32_t *cs2 = (const uint32_t *)ctx->buf[kBufCandS2].ptr;
            auto time_all = [&](double *ms) -> pastis_status {
                ctx->stats = pastis_run_stats{};
                ctx->records_internal = true;
                const pastis_status r = align_core(ctx, st, codes, n, clo, chi, cs1, cs2, nc, rec_all, s);
                ctx->records_internal = false;
                PASTIS_TRY(r);
                HIP_TRY(ctx, stage_collect(ctx, s), "sync");
                *ms = ctx->stats.ms_stage[kStSched] + ctx->stats.ms_stage[kStAlign1] + ctx->stats.ms_stage[kStAlign2];
                return PASTIS_OK;
            };
            double all_ms = 0;
            PASTIS_TRY(time_all(&all_ms));
            // at most about 12 more runs: skipped where one takes over 2 s
            if (all_ms > 2000.0) {
                if (out) *out = ctx->tune;
                return PASTIS_OK;
            }
            PASTIS_TRY(time_all(&all_ms));
            auto refine = [&](int32_t *knob, const int *vals, int nv) -> pastis_status {
                const int32_t keep = *knob;
                int32_t best_v = keep;
                double best_ms = all_ms;
                for (int i = 0; i < nv; ++i) {
                    if (vals[i] == keep) continue;
                    *knob = vals[i];
                    double ms = 0;
                    PASTIS_TRY(time_all(&ms));
                    if (ms < 0.995 * best_ms) {
                        best_ms = ms;
                        best_v = vals[i];
                    }
                }
                *knob = best_v;
                all_ms = best_ms;
                return PASTIS_OK;
            };
            const int route[] = {25, 50, 75, 100};
            PASTIS_TRY(refine(&ctx->tune.sw_direct_pct, route, 4));
            PASTIS_TRY(refine(&ctx->tune.sw_intra_pair, intra, 2));
            PASTIS_TRY(refine(&ctx->tune.sw_long_blocks, longb, 3));
            // the grids of the one-strip bins, whose ends also shorten with
            // the sample (about 1% of large's step between their values)
            PASTIS_TRY(refine(&ctx->tune.sw_grid_scale_wide, grid, 3));
            PASTIS_TRY(refine(&ctx->tune.sw_grid_scale, grid, 3));
        }
    }
    if (out) *out = ctx->tune;
    return PASTIS_OK;
}

}  // extern "C"
