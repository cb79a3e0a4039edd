// Smith-Waterman alignment of candidate pairs (Section IV-E): one 64-lane
// wavefront per pair, 32-bit DP words, pairs binned by the length of the
// shorter sequence.
//
// Layout.  The rows of the shorter sequence a are split into strips of 64*R
// rows; lane l owns rows [l*R, l*R + R) of a strip and sweeps the columns of b
// one column behind lane l-1 (lane l is at column t - l in step t).  All DP
// state stays in registers; the bottom row of a lane's block moves to the next
// lane once per step with a DPP wavefront shift, and the column residue moves
// with it (lane 0 takes it from a register chunk of b via readlane).  Pairs
// whose shorter side needs more than one strip pass the strip's bottom row
// through a per-wave global buffer.  R is chosen per pair (one-strip bins
// R = 1..16; multi-strip bins R = 9..16 with the fewest strips of at most
// 1024 rows), so few lanes hold padding rows.
//
// Scores.  A per-lane profile in LDS holds, for every column residue code, the
// R int8 scores of the lane's rows; one LDS load per step serves R cells and
// the byte selects fold into the adds (SDWA).
//
// Pass 1 computes the score and the canonical end: the smallest row, then the
// smallest column, holding the maximum.  Each row keeps max((h << 16) |
// (0xFFFF - column)), which orders by score and then by the earlier column.
//
// Pass 2 recomputes the rectangle [0, end_a] x [0, end_b] carrying, for every
// cell and state (H, E, F), the start cell, identical pairs and diagonal
// columns of the canonical path ending there.  Each cell takes the predecessor
// a traceback would take (diagonal before horizontal before vertical gap,
// extension before opening; a zero diagonal predecessor starts a new path), so
// by induction the end cell holds the traceback's statistics.  The strip rows
// are padded at the top so the end cell is always row R-1 of lane 63.
#include <algorithm>
#include <type_traits>

#include <utility>

#include "internal.hpp"
#include "prim.hpp"

namespace pastis {

hipError_t launch_bins(const int8_t *bin_of, int64_t n, int nbins, int *counts, int *starts, int *cursor, int *idx,
                       hipStream_t s);

namespace {

constexpr int kWave = 64;
constexpr int kNeg = -(1 << 28);
// waves per block of the 32-bit kernels: one int8 profile of 25 x 64 x R
// bytes per wave, blocks of at most ~51 KB of LDS (three per CU)
__host__ __device__ constexpr int wpb32(int R) { return R <= 8 ? 4 : 2; }
constexpr int kProfCodes = kAlpha + 1;  // 24 residues + the pad code
constexpr int kMaxR = 16;               // rows per lane
constexpr int kSingleBins = kMaxR;      // bins 0..15: one strip of 64 * (bin + 1) rows
constexpr int kMultiBin = kSingleBins;  // bins 16..23: several strips of 64 * R rows, R = bin - 7
constexpr int kMultiMinR = kMaxR / 2 + 1;
// bins 24..31: as 16..23 for sequences a of at most kMax16Rows rows, whose
// scores (at most 11 per row with BLOSUM62) stay below 2^15
constexpr int kMulti16Bin = kMultiBin + kMaxR - kMultiMinR + 1;
constexpr int kNumBins = kMulti16Bin + kMaxR - kMultiMinR + 1;
constexpr int kMax16Rows = 32767 / 11;
static_assert(kNumBins <= 32, "bin tables hold 32 entries");

__host__ __device__ constexpr int rows_of_bin(int bin) {
    return bin >= kMulti16Bin ? bin - kMulti16Bin + kMultiMinR : bin >= kMultiBin ? bin - kMultiBin + kMultiMinR
                                                                                   : bin + 1;
}
constexpr int kDppWaveShr1 = 0x138;

// lane l receives lane l-1's value; lane 0 receives `lane0`
__device__ __forceinline__ int shr1(int lane0, int v) {
    return __builtin_amdgcn_update_dpp(lane0, v, kDppWaveShr1, 0xF, 0xF, false);
}

// lane l receives lane l-1's value; lane 0 receives 0 (the move's bound
// control zero-fills, so no separate write of lane 0's value is needed)
__device__ __forceinline__ int shr1z(int v) { return __builtin_amdgcn_update_dpp(0, v, kDppWaveShr1, 0xF, 0xF, true); }

// R int8 scores per lane and residue code, in ceil(R / 4) words
template <int R>
using ProfWord = typename std::conditional<
    (R <= 4), uint32_t,
    typename std::conditional<(R <= 8), uint2, typename std::conditional<(R <= 12), uint3, uint4>::type>::type>::type;

template <int R>
__device__ __forceinline__ uint32_t word_of(const ProfWord<R> &w, int k) {
    if constexpr (R <= 4) {
        return w;
    } else if constexpr (R <= 8) {
        return k == 0 ? w.x : w.y;
    } else if constexpr (R <= 12) {
        return k == 0 ? w.x : k == 1 ? w.y : w.z;
    } else {
        return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
    }
}

template <int R>
__device__ __forceinline__ ProfWord<R> make_word(const uint32_t (&w)[4]) {
    if constexpr (R <= 4) {
        return w[0];
    } else if constexpr (R <= 8) {
        return make_uint2(w[0], w[1]);
    } else if constexpr (R <= 12) {
        return make_uint3(w[0], w[1], w[2]);
    } else {
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
}

template <int R>
__device__ __forceinline__ int sigma_at(const ProfWord<R> &w, int r) {
    return (int)(int8_t)(word_of<R>(w, r >> 2) >> (8 * (r & 3)));
}

template <int R>
__device__ __forceinline__ void build_profile(ProfWord<R> (*prof)[kWave], const int8_t *sblosum, const uint8_t *a,
                                              int la, int base, int lane) {
    int ar[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ar[r] = (base + r >= 0 && base + r < la) ? a[base + r] : kPadCode;
    for (int c = 0; c < kProfCodes; ++c) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < R; ++r) w[r >> 2] |= (uint32_t)(uint8_t)sblosum[ar[r] * kProfCodes + c] << (8 * (r & 3));
        prof[c][lane] = make_word<R>(w);
    }
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
        unsigned olo = __shfl_xor(lo, off, kWave), ohi = __shfl_xor(hi, off, kWave);
        unsigned long long o = ((unsigned long long)ohi << 32) | olo;
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ void load_blosum(int8_t *sblosum, const int8_t *blosum) {
    for (int t = threadIdx.x; t < kProfCodes * kProfCodes; t += blockDim.x) sblosum[t] = blosum[t];
    __syncthreads();
}

// A load the compiler must issue per lane through the vector memory path (the
// data was written by another lane of the same wave earlier in the kernel).
template <typename T>
__device__ __forceinline__ T vload(const T *p) {
    return __builtin_nontemporal_load(p);
}

// A wave's next window of `count` consecutive items of its bin: lane 0 claims
// it from the bin's queue counter (zeroed before the launch), so that a
// resident grid stays busy until the bin is empty, waves that finish early
// taking more work.  The counter is claimed by a vector atomic.
__device__ __forceinline__ int64_t take(int *queue, const int *starts, int bin, int count) {
    int v = 0;
    if ((threadIdx.x & (kWave - 1)) == 0) v = atomicAdd(queue + bin, count);
    return starts[bin] + (int64_t)__builtin_amdgcn_readfirstlane(v);
}

// the same from a counter of its own over items [begin, ...)
__device__ __forceinline__ int64_t take_from(int *counter, int begin, int count) {
    int v = 0;
    if ((threadIdx.x & (kWave - 1)) == 0) v = atomicAdd(counter, count);
    return begin + (int64_t)__builtin_amdgcn_readfirstlane(v);
}

// ---------------------------------------------------------------- pass 1

// max(x - y, 0) for x >= 0, y >= 0 (one clamped subtract)
__device__ __forceinline__ int subs(int x, int y) {
    return (int)__builtin_elementwise_sub_sat((unsigned)x, (unsigned)y);
}

// Pass 1, 32-bit lanes.  The gap states are kept floored at zero, E' =
// max(E, 0) and F' = max(F, 0) (max(E' - e, 0) = max(E - e, 0) for e >= 0,
// one clamped subtract); max(d, E', F') then already holds the local
// alignment's zero.  The strip boundary carries F'.
template <int R, bool MULTI>
__global__ __launch_bounds__(64 * wpb32(R)) void sw_pass1_kernel(const uint8_t *__restrict__ codes,
                                                       const PairDesc *__restrict__ pairs,
                                                       const int *__restrict__ idx, const int *__restrict__ starts,
                                                       int bin, const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                       SwPass1Out *__restrict__ out, int *__restrict__ scratch,
                                                       int64_t scratch_per_wave, int *queue) {
    constexpr int WPB = wpb32(R);
    __shared__ ProfWord<R> prof_all[WPB][kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    ProfWord<R>(*prof)[kWave] = prof_all[wave];
    const int64_t gwave = (int64_t)blockIdx.x * WPB + wave;
    int *bnd_h = scratch + gwave * scratch_per_wave;  // bottom row H / F of the strip above
    int *bnd_f = bnd_h + scratch_per_wave / 2;
    const int item_end = starts[bin + 1];
    constexpr int RS = kWave * R;

    for (int64_t w = take(queue, starts, bin, 1); w < item_end; w = take(queue, starts, bin, 1)) {
        const int q = idx[w];
        const PairDesc pd = pairs[q];
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int la = pd.la, lb = pd.lb;
        unsigned long long best = 0;  // (score << 32) | ~(row << 16 | col)
        const int nstrips = (la > 0 && lb > 0) ? (MULTI ? (la + RS - 1) / RS : 1) : 0;
        for (int s = 0; s < nstrips; ++s) {
            const int base = s * RS + lane * R;
            build_profile<R>(prof, sblosum, a, la, base, lane);
            const bool from_above = s > 0;
            const bool to_below = s + 1 < nstrips;
            int H[R], G[R], E[R];
            unsigned key[R];  // single strip: (h << 16) | (0xFFFF - col)
            int rmax[R], rcol[R];  // multi strip: scores may exceed 16 bits
#pragma unroll
            for (int r = 0; r < R; ++r) {
                H[r] = 0;
                G[r] = -go_ge;
                E[r] = 0;
                key[r] = 0;
                rmax[r] = 0;
                rcol[r] = 0;
            }
            int hlast = 0, flast = 0, hprev = 0, cres = kPadCode;
            // column residues and the strip boundary row arrive in coalesced
            // chunks of 64 columns, fetched one chunk ahead; lane 0 reads its
            // value for step t with readlane
            int chunk = kPadCode, ch_h = 0, ch_f = 0;
            int nx = (lane < lb) ? (int)b[lane] : kPadCode;
            int nx_h = 0, nx_f = 0;
            if (MULTI && from_above && lane < lb) {
                nx_h = vload(bnd_h + lane);
                nx_f = vload(bnd_f + lane);
            }
            // one DP step; in the tail (t >= lb) lanes past the last column
            // must not touch their running maxima
            auto step = [&](const int t, auto tail_tag) {
                constexpr bool kTail = decltype(tail_tag)::value;
                if ((t & (kWave - 1)) == 0) {
                    chunk = nx;
                    const int c = t + kWave + lane;
                    nx = (c < lb) ? (int)b[c] : kPadCode;
                    if (MULTI && from_above) {
                        ch_h = nx_h;
                        ch_f = nx_f;
                        if (c < lb) {
                            nx_h = vload(bnd_h + c);
                            nx_f = vload(bnd_f + c);
                        }
                    }
                }
                const int bt = __builtin_amdgcn_readlane(chunk, t & (kWave - 1));
                int in_h = 0, in_f = 0;
                if (MULTI && !kTail && from_above) {
                    in_h = __builtin_amdgcn_readlane(ch_h, t & (kWave - 1));
                    in_f = __builtin_amdgcn_readlane(ch_f, t & (kWave - 1));
                }
                const int rh = shr1(in_h, hlast);
                const int rf = shr1(in_f, flast);
                cres = shr1(bt, cres);
                const int j = t - lane;
                const bool valid = j < lb;
                const ProfWord<R> pw = prof[cres][lane];
                const unsigned jinv = (unsigned)(0xFFFF - j) & 0xFFFFu;
                int hd = hprev, gu = rh - go_ge, fu = rf;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = max(subs(E[r], ge), G[r]);
                    const int f = max(subs(fu, ge), gu);
                    const int d = hd + sigma_at<R>(pw, r);
                    const int h = max(d, max(e, f));
                    hd = H[r];
                    H[r] = h;
                    E[r] = e;
                    const int g = h - go_ge;
                    G[r] = g;
                    gu = g;
                    fu = f;
                    if constexpr (MULTI) {
                        if ((!kTail || valid) && h > rmax[r]) {
                            rmax[r] = h;
                            rcol[r] = j;
                        }
                    } else {
                        const unsigned k = ((unsigned)h << 16) | jinv;
                        const unsigned m = k > key[r] ? k : key[r];
                        key[r] = (!kTail || valid) ? m : key[r];
                    }
                }
                hlast = H[R - 1];
                flast = fu;
                hprev = rh;
                if (MULTI && to_below && lane == kWave - 1 && j >= 0 && j < lb) {
                    bnd_h[j] = hlast;
                    bnd_f[j] = flast;
                }
            };
            for (int t = 0; t < lb; ++t) step(t, std::false_type{});
            for (int t = lb; t < lb + kWave - 1; ++t) step(t, std::true_type{});
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = base + r;
                int sc, col;
                if constexpr (MULTI) {
                    sc = rmax[r];
                    col = rcol[r];
                } else {
                    sc = (int)(key[r] >> 16);
                    col = 0xFFFF - (int)(key[r] & 0xFFFFu);
                }
                if (row < la && sc > 0) {
                    const unsigned pos = ((unsigned)row << 16) | (unsigned)col;
                    const unsigned long long k = ((unsigned long long)(unsigned)sc << 32) | (unsigned)(~pos);
                    best = k > best ? k : best;
                }
            }
            if (MULTI) __threadfence_block();  // lane 0 of the next strip reads lane 63's row
        }
        best = wave_max_u64(best);
        if (lane == 0) {
            SwPass1Out o;
            o.score = (int32_t)(best >> 32);
            const unsigned pos = ~(unsigned)best;
            o.end_a = o.score > 0 ? (int32_t)(pos >> 16) : -1;
            o.end_b = o.score > 0 ? (int32_t)(pos & 0xFFFF) : -1;
            o.pad = 0;
            out[q] = o;
        }
    }
}

// ---------------------------------------------------------------- pass 1, one workgroup per long pair

// Intra-pair mode for long sequences a: the W waves of a block work on one
// pair.  Wave w takes strips w, w + W, ... (strips of 64 R rows in 32-bit
// lanes, as in the multi-strip kernel above), so W strips run at once, each
// a little behind the one above.  The bottom row of strip s (H and F' of
// every column) reaches strip s + 1 through a full-length row buffer of slot
// s mod W in global memory.  Two monotone LDS counters per slot order the
// hand-off, in columns over all strips that used the slot for this pair:
// prod (written) and cons (loaded by the reader).  The reader of strip s + 1
// waits for prod (strip s); the writer of strip s + W waits until strip
// s + 1 has loaded the columns it overwrites.  Every wait is for an earlier
// strip, so the earliest unfinished strip never waits and the pipeline
// drains; each wait is also bounded, and a wait that runs out sets *flag and
// gives up (the call then fails) instead of spinning on.  The counters are
// released and acquired at workgroup scope, which orders the row buffer's
// global stores and loads between the waves of the block.
constexpr int kIntraWaves = 4;
constexpr int kIntraSpinLimit = 1 << 24;

__device__ __forceinline__ int lds_acquire(int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// wait until *p >= need; false when the bound runs out
__device__ __forceinline__ bool lds_wait(int *p, int need) {
    for (int spin = 0; spin < kIntraSpinLimit; ++spin) {
        if (__builtin_amdgcn_readfirstlane(lds_acquire(p)) >= need) return true;
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

template <int R>
__global__ __launch_bounds__(64 * kIntraWaves) void sw_intra_pass1_kernel(
    const uint8_t *__restrict__ codes, const PairDesc *__restrict__ pairs, const int *__restrict__ idx,
    const int *__restrict__ starts, int bin, const int8_t *__restrict__ blosum, int go_ge, int ge,
    SwPass1Out *__restrict__ out, int *scratch, int64_t scratch_per_wave, int *queue, unsigned long long *flag) {
    constexpr int W = kIntraWaves;
    __shared__ ProfWord<R> prof_all[W][kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    __shared__ int prod[W], cons[W];
    __shared__ unsigned long long s_best[W];
    __shared__ int s_take;
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    ProfWord<R>(*prof)[kWave] = prof_all[wave];
    const int item_end = starts[bin + 1];
    constexpr int RS = kWave * R;
    const int in_slot = (wave + W - 1) % W;  // the slot this wave's strips read
    // slot k's row buffer: H at row[k], F' at row[k] + scratch_per_wave / 2
    int *const out_h = scratch + ((int64_t)blockIdx.x * W + wave) * scratch_per_wave;
    int *const out_f = out_h + scratch_per_wave / 2;
    const int *const in_h = scratch + ((int64_t)blockIdx.x * W + in_slot) * scratch_per_wave;
    const int *const in_f = in_h + scratch_per_wave / 2;

    for (;;) {
        // every wave is past the last pair (the barrier at its end), so the
        // block's counters and window may be reset
        if (threadIdx.x == 0) s_take = atomicAdd(queue + bin, 1);
        if (threadIdx.x < W) {
            prod[threadIdx.x] = 0;
            cons[threadIdx.x] = 0;
        }
        __syncthreads();
        const int64_t w = starts[bin] + s_take;
        if (w >= item_end) break;
        const int q = idx[w];
        const PairDesc pd = pairs[q];
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int la = pd.la, lb = pd.lb;
        unsigned long long best = 0;  // (score << 32) | ~(row << 16 | col)
        bool ok = true;
        const int nstrips = (la > 0 && lb > 0) ? (la + RS - 1) / RS : 0;
        for (int s = wave; ok && s < nstrips; s += W) {
            const int base = s * RS + lane * R;
            build_profile<R>(prof, sblosum, a, la, base, lane);
            const bool from_above = s > 0;
            const bool to_below = s + 1 < nstrips;
            // first absolute column of the slot uses this strip reads / writes
            const int in0 = (s > 0 ? (s - 1) / W : 0) * lb, out0 = (s / W) * lb;
            int H[R], G[R], E[R], rmax[R], rcol[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                H[r] = 0;
                G[r] = -go_ge;
                E[r] = 0;
                rmax[r] = 0;
                rcol[r] = 0;
            }
            int hlast = 0, flast = 0, hprev = 0, cres = kPadCode;
            int chunk = kPadCode, nx = (lane < lb) ? (int)b[lane] : kPadCode;
            // the row above arrives in chunks of 64 columns, one chunk ahead
            int ch_h = 0, ch_f = 0, nx_h = 0, nx_f = 0;
            auto fetch_above = [&](int c0) {  // columns c0 .. c0 + 63 into nx
                const int hi = min(c0 + kWave, lb);
                if (ok && !lds_wait(&prod[in_slot], in0 + hi)) ok = false;
                nx_h = c0 + lane < lb ? in_h[c0 + lane] : 0;
                nx_f = c0 + lane < lb ? in_f[c0 + lane] : 0;
                if (lane == 0) lds_release(&cons[in_slot], in0 + hi);
            };
            if (from_above) fetch_above(0);
            auto step = [&](const int t, auto tail_tag) {
                constexpr bool kTail = decltype(tail_tag)::value;
                if ((t & (kWave - 1)) == 0) {
                    chunk = nx;
                    const int c = t + kWave + lane;
                    nx = (c < lb) ? (int)b[c] : kPadCode;
                    if (!kTail && from_above) {
                        ch_h = nx_h;
                        ch_f = nx_f;
                        if (t + kWave < lb) fetch_above(t + kWave);
                    }
                }
                const int bt = __builtin_amdgcn_readlane(chunk, t & (kWave - 1));
                int in_hv = 0, in_fv = 0;
                if (!kTail && from_above) {
                    in_hv = __builtin_amdgcn_readlane(ch_h, t & (kWave - 1));
                    in_fv = __builtin_amdgcn_readlane(ch_f, t & (kWave - 1));
                }
                const int rh = shr1(in_hv, hlast);
                const int rf = shr1(in_fv, flast);
                cres = shr1(bt, cres);
                const int j = t - lane;
                const bool valid = j < lb;
                const ProfWord<R> pw = prof[cres][lane];
                int hd = hprev, gu = rh - go_ge, fu = rf;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = max(subs(E[r], ge), G[r]);
                    const int f = max(subs(fu, ge), gu);
                    const int d = hd + sigma_at<R>(pw, r);
                    const int h = max(d, max(e, f));
                    hd = H[r];
                    H[r] = h;
                    E[r] = e;
                    const int g = h - go_ge;
                    G[r] = g;
                    gu = g;
                    fu = f;
                    if ((!kTail || valid) && h > rmax[r]) {
                        rmax[r] = h;
                        rcol[r] = j;
                    }
                }
                hlast = H[R - 1];
                flast = fu;
                hprev = rh;
                // lane 63 leaves column jw = t - 63 for the strip below
                const int jw = t - (kWave - 1);
                if (to_below && jw >= 0 && jw < lb) {
                    // the reader of the slot's previous use (strip s + 1 - W)
                    // must have loaded columns jw .. jw + 63 first
                    if ((jw & (kWave - 1)) == 0 && out0 > 0 && ok &&
                        !lds_wait(&cons[wave], out0 - lb + min(jw + kWave, lb)))
                        ok = false;
                    if (lane == kWave - 1) {
                        out_h[jw] = hlast;
                        out_f[jw] = flast;
                        if ((jw & (kWave - 1)) == kWave - 1 || jw == lb - 1) lds_release(&prod[wave], out0 + jw + 1);
                    }
                }
            };
            for (int t = 0; t < lb; ++t) step(t, std::false_type{});
            for (int t = lb; t < lb + kWave - 1; ++t) step(t, std::true_type{});
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = base + r;
                if (row < la && rmax[r] > 0) {
                    const unsigned pos = ((unsigned)row << 16) | (unsigned)rcol[r];
                    const unsigned long long k = ((unsigned long long)(unsigned)rmax[r] << 32) | (unsigned)(~pos);
                    best = k > best ? k : best;
                }
            }
        }
        if (!ok && lane == 0) atomicOr(flag, 1ull);
        best = wave_max_u64(best);
        if (lane == 0) s_best[wave] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long m = 0;
            for (int k = 0; k < W; ++k) m = s_best[k] > m ? s_best[k] : m;
            SwPass1Out o;
            o.score = (int32_t)(m >> 32);
            const unsigned pos = ~(unsigned)m;
            o.end_a = o.score > 0 ? (int32_t)(pos >> 16) : -1;
            o.end_b = o.score > 0 ? (int32_t)(pos & 0xFFFF) : -1;
            o.pad = 0;
            out[q] = o;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- pass 1, 16-bit lanes

// Two pairs per wave in the 16-bit halves of every DP word (pair P low, Q
// high), same lane layout as the 32-bit pass, one strip (R <= 16).  The two
// pairs share their shorter sequence a (pairs are sorted by bin, then a, then
// the longer b first), so one int8 profile serves both; a wave whose two
// items differ in a runs them one after the other.  Only G = H - (o + e) is
// kept per row: the diagonal term H(i-1, j-1) + s becomes G(i-1, j-1) +
// (s + o + e), with the biased scores s + o + e >= 0 in the profile (each
// row's two bytes are spread into the halves by one byte permute).  Padding
// residues score -(o + e).  Each row keeps only its maximum: cells outside a
// pair (padding rows and columns, columns before the first) score strictly
// below its best real cell, so the score and the first row holding it are
// exact; the end column is found later, for the pairs that need it (end_b =
// -1 here).  Scores stay below 11 * 1024, far from the 16-bit limit.
// The gap states are kept floored at zero, E' = max(E, 0) and F' = max(F, 0):
// their recurrences stay closed (max(E' - e, 0) = max(E - e, 0) for e >= 0,
// one saturating subtract), and max(d, E', F') then already holds the local
// alignment's zero, so a cell takes 10 packed ops instead of 11.
constexpr int kMax16R = kMaxR;

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ short2_t s2(uint32_t x) { return __builtin_bit_cast(short2_t, x); }
// max(x - y, 0) per half, for 0 <= x < 2^15
__device__ __forceinline__ short2_t psubs(short2_t x, uint32_t y) {
    return __builtin_bit_cast(short2_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(ushort2_t, x),
                                                                      __builtin_bit_cast(ushort2_t, y)));
}
__device__ __forceinline__ uint32_t u2(short2_t x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ short2_t pmax(short2_t a, short2_t b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ int shr1u(uint32_t lane0, uint32_t v) { return shr1((int)lane0, (int)v); }

// 16-bit profile: entry [c][p] holds the biased scores s + o + e >= 0 (pad
// rows: 0) of rows p * RP .. p * RP + RP - 1 of a against code c, one byte
// each.  The calling thread writes the codes c = group (mod NG) for position
// pos; NG groups of threads together cover all codes.
template <int RP, int W, int NG>
__device__ __forceinline__ void build_profile16(ProfWord<RP> (*prof)[W], const int8_t *sblosum, const uint8_t *a,
                                                int la, int pos, int group, int oe) {
    int ar[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) ar[r] = (pos * RP + r < la) ? a[pos * RP + r] : kPadCode;
    for (int c = group; c < kProfCodes; c += NG) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const int sc = max((int)sblosum[ar[r] * kProfCodes + c], -oe) + oe;
            w[r >> 2] |= (uint32_t)sc << (8 * (r & 3));
        }
        prof[c][pos] = make_word<RP>(w);
    }
}

template <int R>
__device__ __forceinline__ uint32_t prof_word(const ProfWord<R> &w, int r) {
    return word_of<R>(w, r >> 2);
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, kWave));
    return v;
}


// Full-wave layout for the wider bins.  A block takes 2 * WPB consecutive
// pairs (two per wave) and its waves share one profile, built once per
// distinct sequence a among them (pairs are sorted by a), so the LDS of a
// block does not grow with its wave count.  MULTI: sequences a of more than
// 1024 rows (and at most kMax16Rows, so that scores stay below 2^15) run in
// strips of 64 R rows, one after the other; lane 63 leaves the G and F' words
// of the strip's bottom row for every column in a per-wave buffer, and lane 0
// reads them back as the top boundary of the next strip.
template <int R, int WPB, bool MULTI>
__global__ __launch_bounds__(64 * WPB) void sw16_pass1_kernel(const uint8_t *__restrict__ codes,
                                                              const PairDesc *__restrict__ pairs,
                                                              const int *__restrict__ idx,
                                                              const int *__restrict__ starts, int bin,
                                                              const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                              SwPass1Out *__restrict__ out, uint32_t *scratch,
                                                              int64_t scratch_per_wave, int *queue) {
    static_assert(R > 8 && R <= kMax16R, "more than 512 rows per strip");
    constexpr int NI = 2 * WPB;  // pairs per block
    constexpr int RS = kWave * R;  // rows per strip
    __shared__ ProfWord<R> prof[kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    // first unfinished pair of each wave, double-buffered by round parity so
    // that a round's writes never meet the previous round's reads
    __shared__ int s_next[2][WPB];
    __shared__ int s_take;  // the block's window, claimed from the bin's queue
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int item_end = starts[bin + 1];
    const uint32_t OE2 = (uint32_t)go_ge * 0x10001u, GE2 = (uint32_t)ge * 0x10001u;
    const uint32_t G0 = ((uint32_t)(-go_ge) & 0xFFFFu) * 0x10001u;  // G of an H = 0 cell
    uint32_t *bnd_g = nullptr, *bnd_f = nullptr;
    if constexpr (MULTI) {
        bnd_g = scratch + ((int64_t)blockIdx.x * WPB + wave) * scratch_per_wave;
        bnd_f = bnd_g + scratch_per_wave / 2;
    }
    int par = 0;

    for (;;) {
        // every thread has read the last window before the round loop's
        // first barrier, so thread 0 may claim the next one
        if (threadIdx.x == 0) s_take = atomicAdd(queue + bin, NI);
        __syncthreads();
        const int64_t w = starts[bin] + s_take;
        if (w >= item_end) break;
        const int nit = (int)min((int64_t)NI, item_end - w);
        const int iP = 2 * wave, iQ = iP + 1;
        const int qP = iP < nit ? idx[w + iP] : -1;
        const int qQ = iQ < nit ? idx[w + iQ] : -1;
        const int q0 = idx[w];
        const PairDesc dP = pairs[qP < 0 ? q0 : qP], dQ = pairs[qQ < 0 ? q0 : qQ];
        bool doneP = qP < 0, doneQ = qQ < 0;
        for (;;) {
            // this round's sequence a: that of the block's first unfinished pair
            if (lane == 0) s_next[par][wave] = !doneP ? iP : !doneQ ? iQ : NI;
            __syncthreads();
            int first = NI;
#pragma unroll
            for (int k = 0; k < WPB; ++k) first = min(first, s_next[par][k]);
            par ^= 1;
            if (first >= NI) break;
            const PairDesc dA = pairs[idx[w + first]];
            const bool actP = !doneP && dP.a_seq == dA.a_seq;
            const bool actQ = !doneQ && dQ.a_seq == dA.a_seq;
            const int laA = dA.la, lbP = actP ? dP.lb : 0, lbQ = actQ ? dQ.lb : 0;
            const uint8_t *bP = codes + dP.b_off, *bQ = codes + dQ.b_off;
            const int lb = max(lbP, lbQ);
            const int steps = lb > 0 ? lb + kWave - 1 : 0;
            const int nstrips = MULTI ? (laA + RS - 1) / RS : 1;
            // best row of each pair: (score << 16) | (0xFFFF - row), maximised
            unsigned kp = 0u, kq = 0u;
            for (int sidx = 0; sidx < nstrips; ++sidx) {
                const int base = sidx * RS;
                if (sidx > 0) __syncthreads();  // every wave is done with the last strip's profile
                build_profile16<R, kWave, WPB>(prof, sblosum, codes + dA.a_off + base, laA - base, lane, wave,
                                               go_ge);
                __syncthreads();
                const bool from_above = MULTI && sidx > 0;
                const bool to_below = MULTI && sidx + 1 < nstrips;
                uint32_t G[R], E[R], M[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    G[r] = G0;
                    E[r] = 0u;
                    M[r] = 0u;
                }
                uint32_t glast = G0, flast = 0u, gprev = G0;
                // column residues travel as byte offsets into the profile, P's
                // in the low half and Q's in the high half (at most 24 * 1024)
                constexpr uint32_t kStride = (uint32_t)(sizeof(ProfWord<R>) * kWave);
                const char *plane = (const char *)&prof[0][lane];
                int cres = (int)((kPadCode * kStride) * 0x10001u);
                auto col = [&](int c) {
                    const uint32_t x = c < lbP ? (uint32_t)bP[c] : (uint32_t)kPadCode;
                    const uint32_t y = c < lbQ ? (uint32_t)bQ[c] : (uint32_t)kPadCode;
                    return (int)((x * kStride) | ((y * kStride) << 16));
                };
                int chunk = col(lane);  // columns 0..63; nx holds the next 64
                int nx = col(kWave + lane);
                // top boundary words of columns 0..63 and 64..127 (columns past
                // lb: an H = 0 row above)
                uint32_t ch_g = G0, ch_f = 0u, nx_g = G0, nx_f = 0u;
                if (from_above) {
                    if (lane < lb) {
                        ch_g = vload(bnd_g + lane);
                        ch_f = vload(bnd_f + lane);
                    }
                    if (kWave + lane < lb) {
                        nx_g = vload(bnd_g + kWave + lane);
                        nx_f = vload(bnd_f + kWave + lane);
                    }
                }
                // kTop: lane 0 takes its top boundary from the buffer (t < lb)
                auto step = [&](const int t, auto top_tag) {
                    constexpr bool kTop = decltype(top_tag)::value;
                    if ((t & (kWave - 1)) == 0 && t > 0) {
                        chunk = nx;
                        nx = col(t + kWave + lane);
                        if constexpr (kTop) {
                            ch_g = nx_g;
                            ch_f = nx_f;
                            const int c = t + kWave + lane;
                            nx_g = c < lb ? vload(bnd_g + c) : G0;
                            nx_f = c < lb ? vload(bnd_f + c) : 0u;
                        }
                    }
                    const int bt = __builtin_amdgcn_readlane(chunk, t & (kWave - 1));
                    uint32_t rg, rf;
                    if constexpr (kTop) {
                        rg = (uint32_t)shr1u((uint32_t)__builtin_amdgcn_readlane((int)ch_g, t & (kWave - 1)), glast);
                        rf = (uint32_t)shr1u((uint32_t)__builtin_amdgcn_readlane((int)ch_f, t & (kWave - 1)), flast);
                    } else {
                        rg = (uint32_t)shr1u(G0, glast);
                        rf = (uint32_t)shr1z((int)flast);
                    }
                    cres = shr1(bt, cres);
                    const ProfWord<R> cP = *(const ProfWord<R> *)(plane + ((uint32_t)cres & 0xFFFFu));
                    const ProfWord<R> cQ = *(const ProfWord<R> *)(plane + ((uint32_t)cres >> 16));
                    short2_t gd = s2(gprev), gu = s2(rg), fu = s2(rf);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        // byte r of P's and Q's words into the two halves
                        const uint32_t sel =
                            (uint32_t)(r & 3) | 0x0C00u | ((uint32_t)(4 + (r & 3)) << 16) | 0x0C000000u;
                        const short2_t sig =
                            s2(__builtin_amdgcn_perm(prof_word<R>(cQ, r), prof_word<R>(cP, r), sel));
                        const short2_t e = pmax(psubs(s2(E[r]), GE2), s2(G[r]));
                        const short2_t f = pmax(psubs(fu, GE2), gu);
                        const short2_t d = gd + sig;
                        const short2_t h = pmax(d, pmax(e, f));
                        gd = s2(G[r]);
                        const short2_t g = h - s2(OE2);
                        G[r] = u2(g);
                        E[r] = u2(e);
                        M[r] = u2(pmax(s2(M[r]), h));
                        gu = g;
                        fu = f;
                    }
                    glast = G[R - 1];
                    flast = u2(fu);
                    gprev = rg;
                    if (to_below) {
                        const int j = t - (kWave - 1);
                        if (lane == kWave - 1 && j >= 0 && j < lb) {
                            bnd_g[j] = glast;
                            bnd_f[j] = flast;
                        }
                    }
                };
                // two steps per iteration, so the old and new G registers can
                // swap roles instead of being copied back every step
                int t = 0;
                if (from_above) {
                    for (; t + 1 < lb; t += 2) {
                        step(t, std::true_type{});
                        step(t + 1, std::true_type{});
                    }
                    if (t < lb) step(t++, std::true_type{});
                }
                for (; t + 1 < steps; t += 2) {
                    step(t, std::false_type{});
                    step(t + 1, std::false_type{});
                }
                if (t < steps) step(t, std::false_type{});
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int row = base + lane * R + r;
                    const unsigned rk = 0xFFFFu - (unsigned)row;
                    if (row < laA) {
                        kp = max(kp, ((M[r] & 0xFFFFu) << 16) | rk);
                        kq = max(kq, (M[r] & 0xFFFF0000u) | rk);
                    }
                }
                if (to_below) __threadfence_block();  // lane 0 of the next strip reads lane 63's row
            }
            kp = wave_max_u32(kp);
            kq = wave_max_u32(kq);
            if (lane == 0) {
                SwPass1Out o;
                o.end_b = -1;
                o.pad = 0;
                if (actP) {
                    o.score = (int32_t)(kp >> 16);
                    o.end_a = o.score > 0 ? (int32_t)(0xFFFFu - (kp & 0xFFFFu)) : -1;
                    out[qP] = o;
                }
                if (actQ) {
                    o.score = (int32_t)(kq >> 16);
                    o.end_a = o.score > 0 ? (int32_t)(0xFFFFu - (kq & 0xFFFFu)) : -1;
                    out[qQ] = o;
                }
            }
            doneP = doneP || actP;
            doneQ = doneQ || actQ;
        }
    }
}

// ---------------------------------------------------------------- pass 1, 16-bit lanes, strips of S lanes

// For short sequences a the wave splits into 64 / S independent strips of S
// lanes (S = 16 or 32).  Each strip runs two pairs of the wave's sequence a in
// the halves of its words, with the same recurrence as above; lane p of a
// strip owns rows [p * RP, p * RP + RP), so a bin of 64 R rows takes RP =
// 64 R / S rows per lane.  A pair then pays S - 1 steps of wavefront fill and
// drain instead of 63, and the fixed work of a step (lane shifts, residue and
// profile fetches) serves 64 / S times more cells.  All strips read one
// profile of 25 codes x S lanes.  Column residues enter at a strip's first
// lane from a chunk of 16 columns held across the strip's first 16 lanes,
// rotated by one lane per step.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowRor15 = 0x12F;

// lane p of a strip receives lane p - 1's value; the strip's first lane
// receives `first`
template <int S>
__device__ __forceinline__ uint32_t strip_shr(uint32_t first, uint32_t v, int lane) {
    if constexpr (S == 16) {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, kDppRowShr1, 0xF, 0xF, false);
    } else {
        // a zero-filled shift writes every lane (no prior value of the result
        // is needed); the strips' first lanes, 0 and 32, then take `first`
        const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppWaveShr1, 0xF, 0xF, true);
        return (lane & (S - 1)) == 0 ? first : t;
    }
}

// as strip_shr with first = 0 (zero-filled by the move's bound control)
template <int S>
__device__ __forceinline__ uint32_t strip_shrz(uint32_t v, int lane) {
    if constexpr (S == 16) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr1, 0xF, 0xF, true);
    } else {
        const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppWaveShr1, 0xF, 0xF, true);
        return lane == kWave / 2 ? 0u : t;
    }
}

template <int S>
__device__ __forceinline__ unsigned strip_max_u32(unsigned v) {
#pragma unroll
    for (int off = S / 2; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}


// One launch takes one half of a bin's pairs (sorted by rows class first):
// half 0 the items [starts[bin], split[bin]), half 1 [split[bin],
// starts[bin + 1]), each with its own work-queue counter.
template <int S, int RP, int WPB>
__global__ __launch_bounds__(64 * WPB) void sw16s_pass1_kernel(const uint8_t *__restrict__ codes,
                                                               const PairDesc *__restrict__ pairs,
                                                               const int *__restrict__ idx,
                                                               const int *__restrict__ starts,
                                                               const int *__restrict__ split, int bin, int half,
                                                               const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                               SwPass1Out *__restrict__ out, int *queue) {
    static_assert((S == 16 || S == 32) && RP <= kMax16R, "strip shape");
    constexpr int NI = 2 * kWave / S;  // pairs per wave: two per strip
    __shared__ ProfWord<RP> prof_all[WPB][kProfCodes][S];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int pos = lane % S, strip = lane / S, cl = lane & 15;
    ProfWord<RP>(*prof)[S] = prof_all[wave];
    const int item_begin = half ? split[bin] : starts[bin];
    const int item_end = half ? starts[bin + 1] : split[bin];
    int *const counter = queue + (half ? 3 * kNumBins : 0) + bin;
    const uint32_t OE2 = (uint32_t)go_ge * 0x10001u, GE2 = (uint32_t)ge * 0x10001u;
    const uint32_t G0 = ((uint32_t)(-go_ge) & 0xFFFFu) * 0x10001u;  // G of an H = 0 cell

    for (int64_t w = take_from(counter, item_begin, NI); w < item_end; w = take_from(counter, item_begin, NI)) {
        const int nit = (int)min((int64_t)NI, item_end - w);
        const int iP = 2 * strip, iQ = iP + 1;
        const int qP = iP < nit ? idx[w + iP] : -1;
        const int qQ = iQ < nit ? idx[w + iQ] : -1;
        const int q0 = idx[w];
        const PairDesc dP = pairs[qP < 0 ? q0 : qP], dQ = pairs[qQ < 0 ? q0 : qQ];
        bool doneP = qP < 0, doneQ = qQ < 0;
        // one round per distinct sequence a among the wave's pairs (pairs are
        // sorted by a, so nearly always one)
        for (;;) {
            const int mine = !doneP ? iP : !doneQ ? iQ : NI;
            const int first = __builtin_amdgcn_readfirstlane(wave_min_i32(mine));
            if (first >= NI) break;
            const int src = (first >> 1) * S;
            const bool fq = (first & 1) != 0;
            const int a_seq = __builtin_amdgcn_readlane(fq ? dQ.a_seq : dP.a_seq, src);
            const int la = __builtin_amdgcn_readlane(fq ? dQ.la : dP.la, src);
            const int64_t a_off_v = fq ? dQ.a_off : dP.a_off;
            const uint32_t off_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a_off_v, src);
            const uint32_t off_hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a_off_v >> 32), src);
            const int64_t a_off = (int64_t)(((uint64_t)off_hi << 32) | off_lo);
            const bool actP = !doneP && dP.a_seq == a_seq;
            const bool actQ = !doneQ && dQ.a_seq == a_seq;
            const int lbP = actP ? dP.lb : 0, lbQ = actQ ? dQ.lb : 0;
            const uint8_t *bP = codes + dP.b_off, *bQ = codes + dQ.b_off;
            build_profile16<RP, S, kWave / S>(prof, sblosum, codes + a_off, la, pos, strip, go_ge);
            // lanes read entries written by other lanes of the wave (LDS
            // operations of one wave complete in order)
            __builtin_amdgcn_wave_barrier();
            const int lbmax = wave_max_i32(max(lbP, lbQ));
            const int steps = __builtin_amdgcn_readfirstlane(lbmax > 0 ? lbmax + S - 1 : 0);
            uint32_t G[RP], E[RP], M[RP];
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                G[r] = G0;
                E[r] = 0u;
                M[r] = 0u;
            }
            uint32_t glast = G0, flast = 0u, gprev = G0;
            // column residues travel as byte offsets into the profile, P's in
            // the low half and Q's in the high half (at most 24 * 512 bytes)
            constexpr uint32_t kStride = (uint32_t)(sizeof(ProfWord<RP>) * S);
            const char *plane = (const char *)&prof[0][pos];
            uint32_t cres = (kPadCode * kStride) * 0x10001u;
            auto col = [&](int c) -> uint32_t {
                const uint32_t x = c < lbP ? (uint32_t)bP[c] : (uint32_t)kPadCode;
                const uint32_t y = c < lbQ ? (uint32_t)bQ[c] : (uint32_t)kPadCode;
                return (x * kStride) | ((y * kStride) << 16);
            };
            auto at = [&](uint32_t off) { return *(const ProfWord<RP> *)(plane + off); };
            uint32_t chunk = col(cl);  // columns 0..15; nx holds the next 16
            uint32_t nx = col(16 + cl);
            // the residues of step tn enter at each strip's first lane
            auto feed = [&](const int tn) {
                if ((tn & 15) == 0 && tn > 0) {
                    chunk = nx;
                    nx = col(tn + 16 + cl);
                }
                cres = strip_shr<S>(chunk, cres, lane);
                chunk = (uint32_t)__builtin_amdgcn_mov_dpp((int)chunk, kDppRowRor15, 0xF, 0xF, false);
            };
            // as in the full-wave kernel: with few rows per lane the profile
            // words of step t + 1 are loaded during step t
            constexpr bool kAhead = RP <= 8;
            ProfWord<RP> wP = prof[kPadCode][pos], wQ = wP;
            auto step = [&](const int t) {
                const uint32_t rg = strip_shr<S>(G0, glast, lane);
                const uint32_t rf = strip_shrz<S>(flast, lane);
                ProfWord<RP> cP, cQ;
                if constexpr (kAhead) {
                    feed(t + 1);
                    cP = wP;
                    cQ = wQ;
                    wP = at(cres & 0xFFFFu);
                    wQ = at(cres >> 16);
                } else {
                    feed(t);
                    cP = at(cres & 0xFFFFu);
                    cQ = at(cres >> 16);
                }
                short2_t gd = s2(gprev), gu = s2(rg), fu = s2(rf);
#pragma unroll
                for (int r = 0; r < RP; ++r) {
                    const uint32_t sel =
                        (uint32_t)(r & 3) | 0x0C00u | ((uint32_t)(4 + (r & 3)) << 16) | 0x0C000000u;
                    const short2_t sig = s2(__builtin_amdgcn_perm(prof_word<RP>(cQ, r), prof_word<RP>(cP, r), sel));
                    const short2_t e = pmax(psubs(s2(E[r]), GE2), s2(G[r]));
                    const short2_t f = pmax(psubs(fu, GE2), gu);
                    const short2_t d = gd + sig;
                    const short2_t h = pmax(d, pmax(e, f));
                    gd = s2(G[r]);
                    const short2_t g = h - s2(OE2);
                    G[r] = u2(g);
                    E[r] = u2(e);
                    M[r] = u2(pmax(s2(M[r]), h));
                    gu = g;
                    fu = f;
                }
                glast = G[RP - 1];
                flast = u2(fu);
                gprev = rg;
            };
            if constexpr (kAhead) {
                feed(0);
                wP = at(cres & 0xFFFFu);
                wQ = at(cres >> 16);
            }
            int t = 0;
            for (; t + 1 < steps; t += 2) {
                step(t);
                step(t + 1);
            }
            if (t < steps) step(t);
            unsigned kp = 0u, kq = 0u;
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const int row = pos * RP + r;
                const unsigned rk = 0xFFFFu - (unsigned)row;
                if (row < la) {
                    kp = max(kp, ((M[r] & 0xFFFFu) << 16) | rk);
                    kq = max(kq, (M[r] & 0xFFFF0000u) | rk);
                }
            }
            kp = strip_max_u32<S>(kp);
            kq = strip_max_u32<S>(kq);
            if (pos == 0) {
                SwPass1Out o;
                o.end_b = -1;
                o.pad = 0;
                if (actP) {
                    o.score = (int32_t)(kp >> 16);
                    o.end_a = o.score > 0 ? (int32_t)(0xFFFFu - (kp & 0xFFFFu)) : -1;
                    out[qP] = o;
                }
                if (actQ) {
                    o.score = (int32_t)(kq >> 16);
                    o.end_a = o.score > 0 ? (int32_t)(0xFFFFu - (kq & 0xFFFFu)) : -1;
                    out[qQ] = o;
                }
            }
            doneP = doneP || actP;
            doneQ = doneQ || actQ;
        }
    }
}

// sort keys of the pairing: bin, then the rows class (strip bins of up to
// 8 rows per lane: sequences a of more than 64 R - 32 rows in class 1, which
// the strip kernel runs with one row per lane more than class 0), then
// sequence a (low 24 bits of its index; the kernel checks equality itself),
// then the longer b first
constexpr int kPairKeyBits = 48;
constexpr int kSplitBins = 8;  // one-strip bins 0..7 (up to 8 rows per lane)
__global__ void sw_pair_keys_kernel(const PairDesc *__restrict__ pairs, const int8_t *__restrict__ bin_of,
                                    int64_t npairs, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const PairDesc pd = pairs[q];
    const int bin = (uint8_t)bin_of[q];
    const int tall = bin < kSplitBins && pd.la > kWave * (bin + 1) - kWave / 2;
    keys[q] = ((uint64_t)(2 * bin + tall) << 40) | ((uint64_t)((uint32_t)pd.a_seq & 0xFFFFFFu) << 16) |
              (uint64_t)(0xFFFF - pd.lb);
    vals[q] = (uint32_t)q;
}

// split[bin] = the first sorted item of the bin's rows class 1 (a lower
// bound over the bin's keys)
__global__ void sw_split_kernel(const uint64_t *__restrict__ keys, const int *__restrict__ starts,
                                int *__restrict__ split) {
    const int bin = threadIdx.x;
    if (bin >= kNumBins) return;
    int lo = starts[bin], hi = starts[bin + 1];
    const uint64_t k1 = (uint64_t)(2 * bin + 1) << 40;
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (keys[mid] < k1)
            lo = mid + 1;
        else
            hi = mid;
    }
    split[bin] = lo;
}

// ---------------------------------------------------------------- between the passes

// Rows up to 64 * kMaxR take one strip of 64 * R rows with the smallest R;
// longer ones take the fewest strips of at most 64 * kMaxR rows, with R as
// small as that strip count allows (padding under one row per lane and strip).
__device__ __forceinline__ int rows_bin(int rows) {
    if (rows <= 0) return 0;
    const int r = (rows + kWave - 1) / kWave;
    if (r <= kSingleBins) return r - 1;
    const int strips = (rows + kWave * kSingleBins - 1) / (kWave * kSingleBins);
    const int rm = (rows + kWave * strips - 1) / (kWave * strips);  // in [kMultiMinR, kMaxR]
    return (rows <= kMax16Rows ? kMulti16Bin : kMultiBin) + rm - kMultiMinR;
}

// Bins by rows per lane; counters[0] += DP cells of the pairs, and
// counters[kCounterBinCells + bin] += those of each bin.
__global__ void sw_bin1_kernel(const PairDesc *__restrict__ pairs, int64_t npairs, int8_t *__restrict__ bin_of,
                               unsigned long long *__restrict__ counters, int *__restrict__ queue) {
    // the work queues of this call's launches (pass 1, start bound, statistics)
    if (blockIdx.x == 0 && threadIdx.x < 4 * kNumBins) queue[threadIdx.x] = 0;
    __shared__ unsigned long long cells[kNumBins];
    if (threadIdx.x < kNumBins) cells[threadIdx.x] = 0;
    __syncthreads();
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < npairs) {
        const PairDesc pd = pairs[q];
        const int bin = rows_bin(pd.la);
        bin_of[q] = (int8_t)bin;
        atomicAdd(&cells[bin], (unsigned long long)pd.la * (unsigned long long)pd.lb);
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && cells[threadIdx.x]) {
        atomicAdd(&counters[0], cells[threadIdx.x]);
        atomicAdd(&counters[kCounterBinCells + threadIdx.x], cells[threadIdx.x]);
    }
}

// Pair and cell counts are summed per block in LDS and added to counters[]
// once per block (one atomic per pair would serialise on a few addresses).
__device__ __forceinline__ void flush_counts(unsigned long long (&acc)[4], unsigned long long *counters) {
    __syncthreads();
    if (threadIdx.x < 4 && acc[threadIdx.x]) atomicAdd(&counters[1 + threadIdx.x], acc[threadIdx.x]);
}

// the final record of a pair that takes no statistics pass
__device__ __forceinline__ void sw_final_record(const PairDesc &pd, const SwPass1Out &r1, int64_t q,
                                                pastis_pair_record *__restrict__ out, int8_t *__restrict__ bin_of) {
    bin_of[q] = -1;
    pastis_pair_record rec;
    rec.score = r1.score;
    rec.beg_a = rec.beg_b = -1;
    rec.end_a = r1.end_a;
    rec.end_b = r1.end_b;
    rec.matches = rec.columns = 0;
    rec.seed_used = -1;
    rec.passed = 0;
    rec.swapped = pd.swapped;
    rec.cells = (int64_t)pd.la * pd.lb;
    out[q] = rec;
}

// Records of pairs that need no statistics pass are final here; the others
// are binned by the height of their end rectangle (counters[3], [4]: pairs
// and cells of the start-bound pass; counters[1], [2] in full-records mode).
// stats_mode: 0 = only pairs whose coverage cut can hold, 1 = every aligned
// pair, 2 = none (the normalised-score weight needs no traceback).
__global__ __launch_bounds__(256) void sw_bin2_kernel(const PairDesc *__restrict__ pairs,
                                                      SwPass1Out *__restrict__ p1, int64_t npairs, int cov_pct,
                                                      int stats_mode, int direct_pct,
                                                      pastis_pair_record *__restrict__ out,
                                                      int8_t *__restrict__ bin_of,
                                                      unsigned long long *__restrict__ counters) {
    __shared__ unsigned long long acc[4];  // counters[1..4]
    if (threadIdx.x < 4) acc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < npairs) {
        const PairDesc pd = pairs[q];
        const SwPass1Out r1 = p1[q];
        // coverage needs span_a >= cov% of la, and span_a <= end_a + 1
        const bool need = r1.score > 0 && stats_mode != 2 &&
                          (stats_mode == 1 || 100LL * (r1.end_a + 1) >= (long long)cov_pct * pd.la);
        if (need) {
            bin_of[q] = (int8_t)rows_bin(r1.end_a + 1);
            if (stats_mode == 1) {  // no start bound: every such pair takes pass 2
                atomicAdd(&acc[0], 1ull);
                atomicAdd(&acc[1], (unsigned long long)(r1.end_a + 1) * (unsigned long long)(r1.end_b + 1));
            } else if (100LL * r1.score >= (long long)direct_pct * pd.la) {
                p1[q].pad = -1;  // likely to pass: no start bound
            } else {
                const int cols = r1.end_b >= 0 ? r1.end_b + 1 : pd.lb;
                atomicAdd(&acc[2], 1ull);
                atomicAdd(&acc[3], (unsigned long long)(r1.end_a + 1) * (unsigned long long)cols);
            }
        } else {
            sw_final_record(pd, r1, q, out, bin_of);
        }
    }
    flush_counts(acc, counters);
}

// ---------------------------------------------------------------- start bound

// Scores of the packed recomputation must fit 15 bits; a local alignment
// gains at most 11 per row, so rectangles up to this many rows qualify.
constexpr int kBoundMaxRows = 32000 / 11;
constexpr int kBoundMaxRowsCoarse = (1 << 19) / 11;

// For a pair that still needs the statistics pass, recompute its end
// rectangle [0, end_a] x [0, end_b] with every DP value packed as
// score * 65536 + (65535 - start row).  Each max then keeps the higher score
// and, between equal scores, the smaller start row, so by induction a cell
// holds the smallest start row over all optimal local alignments ending in
// it (an empty alignment ending at row i starts the next path at row i + 1).
// The canonical alignment is one of those ending at the end cell, so its
// coverage of a is at most end_a - bound + 1.  The bound goes to p1[q].pad.
// Scores must fit the high bits: rectangles of up to kBoundMaxRows rows (a
// local alignment gains at most 11 per row) use 16 low bits; up to
// kBoundMaxRowsCoarse rows pack score * 4096 + (4095 - start row / 16), a
// bound rounded down to a multiple of 16 rows (still a valid bound); taller
// ones keep bound 0 (no pruning).
template <int R, bool MULTI>
__global__ __launch_bounds__(64 * wpb32(R)) void sw_bound_kernel(const uint8_t *__restrict__ codes,
                                                       const PairDesc *__restrict__ pairs,
                                                       const int *__restrict__ idx, const int *__restrict__ starts,
                                                       int bin, const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                       SwPass1Out *__restrict__ p1, int *__restrict__ scratch,
                                                       int64_t scratch_per_wave, int *queue) {
    constexpr int WPB = wpb32(R);
    __shared__ ProfWord<R> prof_all[WPB][kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    ProfWord<R>(*prof)[kWave] = prof_all[wave];
    const int64_t gwave = (int64_t)blockIdx.x * WPB + wave;
    int *bnd_h = scratch + gwave * scratch_per_wave;
    int *bnd_f = bnd_h + scratch_per_wave / 2;
    const int item_end = starts[bin + 1];
    constexpr int RS = kWave * R;
    constexpr int kNegP = -(1 << 30);
    const int GO16 = go_ge * 65536, GE16 = ge * 65536;

    // windows of two pairs per claim
    for (int64_t w0 = take(queue, starts, bin, 2); w0 < item_end; w0 = take(queue, starts, bin, 2))
    for (int64_t w = w0; w < min(w0 + 2, (int64_t)item_end); ++w) {
        const int q = idx[w];
        const PairDesc pd = pairs[q];
        const SwPass1Out r1 = p1[q];
        if (r1.pad < 0) continue;  // sent straight to the statistics pass
        // end_b < 0: unknown (16-bit pass 1); the end column is then the first
        // one where row end_a reaches the score
        const bool search = r1.end_b < 0;
        const int la = r1.end_a + 1, lb = search ? pd.lb : r1.end_b + 1;
        if (la > kBoundMaxRowsCoarse) {
            if (lane == 0) p1[q].pad = 0;
            continue;
        }
        // packing: sb low bits hold (mask - start row >> shift)
        const int sb = la > kBoundMaxRows ? 12 : 16, shift = 16 - sb;
        const int mask = (1 << sb) - 1, unit = 1 << sb;
        const int kZero = mask;  // score 0, start row 0
        const int GO = sb == 16 ? GO16 : go_ge * unit, GE = sb == 16 ? GE16 : ge * unit;
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int nstrips = MULTI ? (la + RS - 1) / RS : 1;
        const int top = nstrips * RS - la;  // padding rows above row 0
        int fin = 0, fend = -1;  // lane 63: the end cell's value and (search) its column
        // profile entries are addressed by byte offset: lane base + code * stride
        const char *prof_lane = (const char *)&prof[0][lane];
        constexpr int kStride = (int)(sizeof(ProfWord<R>) * kWave);
        for (int s = 0; s < nstrips; ++s) {
            const int base = s * RS - top + lane * R;
            build_profile<R>(prof, sblosum, a, la, base, lane);
            const bool from_above = s > 0;
            const bool to_below = s + 1 < nstrips;
            const bool last = s + 1 == nstrips;
            int H[R], G[R], E[R], Z[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Z[r] = mask - (max(base + r + 1, 0) >> shift);  // empty alignment ending in row base + r
                H[r] = Z[r];                           // column -1
                G[r] = Z[r] - GO;
                E[r] = kNegP;
            }
            int hlast = kZero, flast = kNegP, hprev = kZero, cres = kPadCode * kStride, chunk = kPadCode * kStride;
            int nx = ((lane < lb) ? (int)b[lane] : kPadCode) * kStride;
            int ch_h = kZero, ch_f = kNegP, nx_h = kZero, nx_f = kNegP;
            if (MULTI && from_above && lane < lb) {
                nx_h = vload(bnd_h + lane);
                nx_f = vload(bnd_f + lane);
            }
            const int steps = __builtin_amdgcn_readfirstlane(lb + kWave - 1);
            auto step = [&](const int t) {
                if ((t & (kWave - 1)) == 0) {
                    chunk = nx;
                    const int c = t + kWave + lane;
                    nx = ((c < lb) ? (int)b[c] : kPadCode) * kStride;
                    if (MULTI && from_above) {
                        ch_h = nx_h;
                        ch_f = nx_f;
                        if (c < lb) {
                            nx_h = vload(bnd_h + c);
                            nx_f = vload(bnd_f + c);
                        }
                    }
                }
                const int bt = __builtin_amdgcn_readlane(chunk, t & (kWave - 1));
                int in_h = kZero, in_f = kNegP;
                if (MULTI && from_above && t < lb) {
                    in_h = __builtin_amdgcn_readlane(ch_h, t & (kWave - 1));
                    in_f = __builtin_amdgcn_readlane(ch_f, t & (kWave - 1));
                }
                const int rh = shr1(in_h, hlast);
                const int rf = shr1(in_f, flast);
                cres = shr1(bt, cres);
                const ProfWord<R> pw = *(const ProfWord<R> *)(prof_lane + cres);
                int hd = hprev, gu = rh - GO, fu = rf;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // E' = max(E, Z): the row's empty-alignment floor rides
                    // along the row (max(E' - e, Z) = max(E - e, Z), since Z
                    // - e < Z), so h is one three-way max
                    const int e = max(max(E[r] - GE, G[r]), Z[r]);
                    const int f = max(fu - GE, gu);
                    const int d = hd + sigma_at<R>(pw, r) * unit;
                    const int h = max(max(d, e), f);
                    hd = H[r];
                    H[r] = h;
                    E[r] = e;
                    const int g = h - GO;
                    G[r] = g;
                    gu = g;
                    fu = f;
                }
                hlast = H[R - 1];
                flast = fu;
                hprev = rh;
                if (MULTI && to_below) {
                    const int j = t - (kWave - 1);
                    if (lane == kWave - 1 && j >= 0 && j < lb) {
                        bnd_h[j] = hlast;
                        bnd_f[j] = flast;
                    }
                }
            };
            int t = 0;
            if (!(search && last)) {
                // two steps per iteration; lane 63's last value is the end cell's
                for (; t + 1 < steps; t += 2) {
                    step(t);
                    step(t + 1);
                }
                if (t < steps) step(t);
                if (last) fin = hlast;
            } else {
                // the end column is the first where lane 63 (row end_a) reaches
                // the score; no cell exceeds it, so reaching is h >= score * unit
                const int thr = r1.score * unit;
                for (; t < kWave - 1; ++t) step(t);  // lane 63 is still left of column 0
                for (; t + 1 < steps; t += 2) {
                    step(t);
                    const int h1 = hlast;
                    step(t + 1);
                    if (__builtin_amdgcn_readlane(h1, kWave - 1) >= thr) {
                        fin = h1;
                        fend = t - (kWave - 1);
                        break;
                    }
                    if (__builtin_amdgcn_readlane(hlast, kWave - 1) >= thr) {
                        fin = hlast;
                        fend = t + 1 - (kWave - 1);
                        break;
                    }
                }
                if (fend < 0 && t < steps) {
                    step(t);
                    if (__builtin_amdgcn_readlane(hlast, kWave - 1) >= thr) {
                        fin = hlast;
                        fend = t - (kWave - 1);
                    }
                }
            }
            if (MULTI) __threadfence_block();
        }
        if (lane == kWave - 1) {
            p1[q].pad = (mask - (fin & mask)) << shift;
            if (search) p1[q].end_b = fend;
        }
    }
}

// Pairs binned for the statistics pass whose coverage bound already fails
// get their final record here; the rest keep their bin.  counters[1] and [2]
// count the pairs and cells left for pass 2.
__global__ __launch_bounds__(256) void sw_bin3_kernel(const PairDesc *__restrict__ pairs,
                                                      const SwPass1Out *__restrict__ p1, int64_t npairs,
                                                      int cov_pct, pastis_pair_record *__restrict__ out,
                                                      int8_t *__restrict__ bin_of,
                                                      unsigned long long *__restrict__ counters) {
    __shared__ unsigned long long acc[4];  // counters[1..4]; [1] and [2] here
    if (threadIdx.x < 4) acc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < npairs && bin_of[q] >= 0) {
        const PairDesc pd = pairs[q];
        const SwPass1Out r1 = p1[q];
        // pad < 0: sent straight here (bound 0 in effect: the coverage test of
        // the first binning already holds)
        if (r1.pad < 0 || 100LL * (r1.end_a - r1.pad + 1) >= (long long)cov_pct * pd.la) {
            const int cols = r1.end_b >= 0 ? r1.end_b + 1 : pd.lb;
            atomicAdd(&acc[0], 1ull);
            atomicAdd(&acc[1], (unsigned long long)(r1.end_a + 1) * (unsigned long long)cols);
        } else {
            sw_final_record(pd, r1, q, out, bin_of);
        }
    }
    flush_counts(acc, counters);
}

// ---------------------------------------------------------------- pass 2

template <int R, bool MULTI>
__global__ __launch_bounds__(64 * wpb32(R)) void sw_pass2_kernel(const uint8_t *__restrict__ codes,
                                                       const PairDesc *__restrict__ pairs,
                                                       const int *__restrict__ idx, const int *__restrict__ starts,
                                                       int bin, const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                       int cov_pct, int id_pct, const SwPass1Out *__restrict__ p1,
                                                       pastis_pair_record *__restrict__ out,
                                                       int *__restrict__ scratch, int64_t scratch_per_wave, int *queue) {
    constexpr int WPB = wpb32(R);
    // no per-wave profile: a row's score against the column residue is read
    // from the 625-byte table, so LDS does not limit the waves per SIMD
    // (occupancy matters here: the statistics selects are long dependent
    // chains).  Entries are 32-bit; the statistics increment of each code
    // pair (0x10001 for identical codes, else 1) follows the scores, so a
    // cell reads it at its score's address plus a constant.  Column residues
    // travel as byte offsets (code * 4) into a row of the table.
    constexpr int kTab = kProfCodes * kProfCodes;
    __shared__ int stab[2 * kTab];
    for (int t = threadIdx.x; t < kTab; t += blockDim.x) {
        stab[t] = blosum[t];
        stab[kTab + t] = t / kProfCodes == t % kProfCodes ? 0x10001 : 1;
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t gwave = (int64_t)blockIdx.x * WPB + wave;
    // strip bottom row per column: H, F, H.beg, H.md, F.beg, F.md
    int *bnd = scratch + gwave * scratch_per_wave;
    const int64_t plane = scratch_per_wave / 6;
    const int item_end = starts[bin + 1];
    constexpr int RS = kWave * R;

    for (int64_t w = take(queue, starts, bin, 1); w < item_end; w = take(queue, starts, bin, 1)) {
        const int q = idx[w];
        const PairDesc pd = pairs[q];
        const SwPass1Out r1 = p1[q];
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        // the rectangle ending at the end cell; with the end column unknown
        // (16-bit pass 1), the full width until row end_a first reaches the score
        const bool search = r1.end_b < 0;
        const int la = r1.end_a + 1, lb = search ? pd.lb : r1.end_b + 1;
        const int nstrips = MULTI ? (la + RS - 1) / RS : 1;
        const int top = nstrips * RS - la;  // padding rows above row 0
        unsigned fin_beg = 0, fin_md = 0;
        int fend = -1;
        for (int s = 0; s < nstrips; ++s) {
            const int base = s * RS - top + lane * R;
            const char *srow[R];  // the row's table entries, at byte offset code * 4
            unsigned rowpart[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ar = (base + r >= 0 && base + r < la) ? (int)a[base + r] : kPadCode;
                srow[r] = (const char *)(stab + ar * kProfCodes);
                rowpart[r] = (unsigned)(base + r) << 16;
            }
            const bool from_above = s > 0;
            const bool to_below = s + 1 < nstrips;
            const bool last = s + 1 == nstrips;
            int H[R], G[R], E[R];
            unsigned sHb[R], sHm[R], sEb[R], sEm[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                H[r] = 0;
                G[r] = -go_ge;
                E[r] = kNeg;
                sHb[r] = sHm[r] = sEb[r] = sEm[r] = 0u;
            }
            int hlast = 0, flast = kNeg, hprev = 0, cres = 4 * kPadCode, chunk = 4 * kPadCode;
            unsigned hb_last = 0, hm_last = 0, fb_last = 0, fm_last = 0, db_prev = 0, dm_prev = 0;
            // chunked, one-ahead prefetch of residues and boundary planes (see pass 1)
            int nx = 4 * ((lane < lb) ? (int)b[lane] : kPadCode);
            int cb[6] = {0, kNeg, 0, 0, 0, 0}, nb[6] = {0, kNeg, 0, 0, 0, 0};
            if (MULTI && from_above && lane < lb) {
#pragma unroll
                for (int p = 0; p < 6; ++p) nb[p] = vload(bnd + p * plane + lane);
            }
            const int steps = __builtin_amdgcn_readfirstlane(lb + kWave - 1);
            // one column step; true once the search has found the end column
            auto step = [&](const int t) -> bool {
                if ((t & (kWave - 1)) == 0) {
                    chunk = nx;
                    const int c = t + kWave + lane;
                    nx = 4 * ((c < lb) ? (int)b[c] : kPadCode);
                    if (MULTI && from_above) {
#pragma unroll
                        for (int p = 0; p < 6; ++p) cb[p] = nb[p];
                        if (c < lb) {
#pragma unroll
                            for (int p = 0; p < 6; ++p) nb[p] = vload(bnd + p * plane + c);
                        }
                    }
                }
                const int bt = __builtin_amdgcn_readlane(chunk, t & (kWave - 1));
                int rh, rf;
                unsigned rhb, rhm, rfb, rfm;
                if (MULTI) {
                    int in_h = 0, in_f = kNeg;
                    unsigned in_hb = 0, in_hm = 0, in_fb = 0, in_fm = 0;
                    if (from_above && t < lb) {
                        const int tt = t & (kWave - 1);
                        in_h = __builtin_amdgcn_readlane(cb[0], tt);
                        in_f = __builtin_amdgcn_readlane(cb[1], tt);
                        in_hb = (unsigned)__builtin_amdgcn_readlane(cb[2], tt);
                        in_hm = (unsigned)__builtin_amdgcn_readlane(cb[3], tt);
                        in_fb = (unsigned)__builtin_amdgcn_readlane(cb[4], tt);
                        in_fm = (unsigned)__builtin_amdgcn_readlane(cb[5], tt);
                    }
                    rh = shr1(in_h, hlast);
                    rf = shr1(in_f, flast);
                    rhb = (unsigned)shr1((int)in_hb, (int)hb_last);
                    rhm = (unsigned)shr1((int)in_hm, (int)hm_last);
                    rfb = (unsigned)shr1((int)in_fb, (int)fb_last);
                    rfm = (unsigned)shr1((int)in_fm, (int)fm_last);
                } else {
                    // row -1 above a single strip: H = 0 with empty
                    // statistics, F closed; the zero-filling shift writes
                    // lane 0's zeros itself
                    rh = shr1z(hlast);
                    rf = shr1(kNeg, flast);
                    rhb = (unsigned)shr1z((int)hb_last);
                    rhm = (unsigned)shr1z((int)hm_last);
                    rfb = (unsigned)shr1z((int)fb_last);
                    rfm = (unsigned)shr1z((int)fm_last);
                }
                cres = shr1(bt, cres);
                const int j = t - lane;
                const unsigned colpart = (unsigned)j & 0xFFFFu;
                int hd = hprev, gu = rh - go_ge, fu = rf;
                unsigned db = db_prev, dm = dm_prev, ub = rhb, um = rhm, fb = rfb, fm = rfm;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // horizontal gap: extend when at least as good as opening
                    const int e_ext = E[r] - ge;
                    const bool ee = e_ext >= G[r];
                    const int e = ee ? e_ext : G[r];
                    const unsigned eb = ee ? sEb[r] : sHb[r];
                    const unsigned em = ee ? sEm[r] : sHm[r];
                    // vertical gap
                    const int f_ext = fu - ge;
                    const bool fe = f_ext >= gu;
                    const int f = fe ? f_ext : gu;
                    const unsigned nfb = fe ? fb : ub;
                    const unsigned nfm = fe ? fm : um;
                    // diagonal; a zero predecessor starts a new path at this cell
                    const int d = hd + *(const int *)(srow[r] + cres);
                    const int h = max(max(d, 0), max(e, f));
                    const bool start = hd == 0;
                    const unsigned xb = start ? (rowpart[r] | colpart) : db;
                    const unsigned xm = (start ? 0u : dm) + *(const unsigned *)(srow[r] + 4 * kTab + cres);
                    const bool is_d = h == d, is_e = h == e;
                    const unsigned hb = is_d ? xb : (is_e ? eb : nfb);
                    const unsigned hm = is_d ? xm : (is_e ? em : nfm);
                    hd = H[r];
                    db = sHb[r];
                    dm = sHm[r];
                    H[r] = h;
                    E[r] = e;
                    const int g = h - go_ge;
                    G[r] = g;
                    sHb[r] = hb;
                    sHm[r] = hm;
                    sEb[r] = eb;
                    sEm[r] = em;
                    gu = g;
                    fu = f;
                    ub = hb;
                    um = hm;
                    fb = nfb;
                    fm = nfm;
                }
                hlast = H[R - 1];
                flast = fu;
                hb_last = ub;
                hm_last = um;
                fb_last = fb;
                fm_last = fm;
                hprev = rh;
                db_prev = rhb;
                dm_prev = rhm;
                if (last && lane == kWave - 1 && j >= 0 && j < lb &&
                    (search ? (fend < 0 && hlast == r1.score) : j == lb - 1)) {
                    fin_beg = hb_last;
                    fin_md = hm_last;
                    fend = j;
                }
                if (MULTI && to_below && lane == kWave - 1 && j >= 0 && j < lb) {
                    bnd[j] = hlast;
                    bnd[plane + j] = flast;
                    bnd[2 * plane + j] = (int)hb_last;
                    bnd[3 * plane + j] = (int)hm_last;
                    bnd[4 * plane + j] = (int)fb_last;
                    bnd[5 * plane + j] = (int)fm_last;
                }
                return search && last && __builtin_amdgcn_readlane(fend, kWave - 1) >= 0;
            };
            if constexpr (MULTI && R >= 14) {
                // the boundary planes leave no registers for a second step
                for (int t = 0; t < steps; ++t)
                    if (step(t)) break;
            } else {
                // two steps per iteration, so the rows' registers need no rotation
                int t = 0;
                bool done = false;
                for (; t + 1 < steps; t += 2) {
                    if (step(t) || step(t + 1)) {
                        done = true;
                        break;
                    }
                }
                if (!done && t < steps) step(t);
            }
            if (MULTI) __threadfence_block();
        }
        if (lane == kWave - 1) {
            pastis_pair_record rec;
            rec.score = r1.score;
            rec.end_a = r1.end_a;
            rec.end_b = fend;
            rec.beg_a = (int32_t)(fin_beg >> 16);
            rec.beg_b = (int32_t)(fin_beg & 0xFFFF);
            rec.matches = (int32_t)(fin_md >> 16);
            const int32_t diag = (int32_t)(fin_md & 0xFFFF);
            rec.columns = (rec.end_a - rec.beg_a + 1) + (rec.end_b - rec.beg_b + 1) - diag;
            rec.seed_used = -1;
            const long long span = (long long)rec.end_a - rec.beg_a + 1;
            rec.passed = (100LL * rec.matches >= (long long)id_pct * rec.columns) &&
                         (100LL * span >= (long long)cov_pct * pd.la);
            rec.swapped = pd.swapped;
            rec.cells = (int64_t)pd.la * pd.lb;
            out[q] = rec;
        }
    }
}

template <int R>
hipError_t launch_p1(int bin, int blocks, const uint8_t *codes, const PairDesc *pairs, const int *idx,
                     const int *starts, const int8_t *blosum, int go_ge, int ge, SwPass1Out *p1, int *scratch,
                     int64_t spw, int *queue, hipStream_t s) {
    if (bin >= kMultiBin)
        sw_pass1_kernel<R, true><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge, p1,
                                                                 scratch, spw, queue);
    else
        sw_pass1_kernel<R, false><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge,
                                                                  p1, scratch, spw, queue);
    return hipGetLastError();
}

template <int R>
hipError_t launch_p2(int bin, int blocks, const uint8_t *codes, const PairDesc *pairs, const int *idx,
                     const int *starts, const int8_t *blosum, int go_ge, int ge, int cov, int id,
                     const SwPass1Out *p1, pastis_pair_record *out, int *scratch, int64_t spw, int *queue,
                     hipStream_t s) {
    if (bin >= kMultiBin)
        sw_pass2_kernel<R, true><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge, cov,
                                                                 id, p1, out, scratch, spw, queue);
    else
        sw_pass2_kernel<R, false><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge,
                                                                  cov, id, p1, out, scratch, spw, queue);
    return hipGetLastError();
}

template <int R>
hipError_t launch_pb(int bin, int blocks, const uint8_t *codes, const PairDesc *pairs, const int *idx,
                     const int *starts, const int8_t *blosum, int go_ge, int ge, SwPass1Out *p1, int *scratch,
                     int64_t spw, int *queue, hipStream_t s) {
    if (bin >= kMultiBin)
        sw_bound_kernel<R, true><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge, p1,
                                                                 scratch, spw, queue);
    else
        sw_bound_kernel<R, false><<<blocks, 64 * wpb32(R), 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge,
                                                                  p1, scratch, spw, queue);
    return hipGetLastError();
}

// waves per block of the 16-bit pass (strips: one profile per wave; full
// waves: one profile per block) and the blocks that fit on the device at once
constexpr int wpb16(int R) { return 4; }
// one-strip bins of more than 512 rows share a profile between the waves of a
// block, and a block runs one round per distinct sequence a of its window:
// two waves (four pairs) per block keep those rounds few where sequences have
// few partners, and eight (six) such blocks per CU keep four (three) waves
// per SIMD within LDS
constexpr int kWpbShared = 2;
// pairs one block of the 16-bit one-strip launch takes per window
// narrow: R <= 4 bins in strips of 16 lanes (eight pairs per wave) rather
// than 32 (four pairs per wave)
static int pairs_per_block16(int R, bool narrow) {
    return R <= 4 && narrow ? 4 * 8 : R <= 8 ? 4 * 4 : 2 * kWpbShared;
}
static int blocks16(int R) { return R <= 4 ? 256 * 6 : R <= 8 ? 256 * 3 : R <= 12 ? 256 * 8 : 256 * 6; }

// R <= 4: strips of 16 lanes with 4 R rows per lane (eight pairs per wave),
// or, when not narrow, of 32 lanes with 2 R rows (four pairs per wave: fewer
// pairs that must share their sequence a); R = 5..8: strips of 32 lanes with
// 2 R rows; wider bins: the full-wave kernel (two pairs per wave)
template <int R>
hipError_t launch_p16(int bin, int blocks, bool narrow, const uint8_t *codes, const PairDesc *pairs, const int *idx,
                      const int *starts, const int *split, const int8_t *blosum, int go_ge, int ge, SwPass1Out *p1,
                      int *queue, hipStream_t s) {
    constexpr int WPB = wpb16(R);
    // strips: rows class 0 (at most 64 R - 32 rows) with one row per lane
    // less in 32-lane strips (two in 16-lane ones), then class 1
    if constexpr (R <= 4) {
        if (narrow) {
            sw16s_pass1_kernel<16, 4 * R - 2, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 0,
                                                                              blosum, go_ge, ge, p1, queue);
            sw16s_pass1_kernel<16, 4 * R, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 1,
                                                                          blosum, go_ge, ge, p1, queue);
        } else {
            sw16s_pass1_kernel<32, 2 * R - 1, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 0,
                                                                              blosum, go_ge, ge, p1, queue);
            sw16s_pass1_kernel<32, 2 * R, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 1,
                                                                          blosum, go_ge, ge, p1, queue);
        }
    } else if constexpr (R <= 8) {
        sw16s_pass1_kernel<32, 2 * R - 1, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 0,
                                                                          blosum, go_ge, ge, p1, queue);
        sw16s_pass1_kernel<32, 2 * R, WPB><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, split, bin, 1,
                                                                      blosum, go_ge, ge, p1, queue);
    } else {
        sw16_pass1_kernel<R, kWpbShared, false><<<blocks, 64 * kWpbShared, 0, s>>>(codes, pairs, idx, starts, bin,
                                                                                  blosum, go_ge, ge, p1, nullptr, 0,
                                                                                  queue);
    }
    return hipGetLastError();
}

// 16-bit multi-strip bins: one boundary buffer per wave of the grid
static int blocks16m() { return 256 * 3; }

template <int R>
hipError_t launch_p16m(int bin, int blocks, const uint8_t *codes, const PairDesc *pairs, const int *idx,
                       const int *starts, const int8_t *blosum, int go_ge, int ge, SwPass1Out *p1, int *scratch,
                       int64_t spw, int *queue, hipStream_t s) {
    constexpr int WPB = wpb16(R);
    sw16_pass1_kernel<R, WPB, true><<<blocks, 64 * WPB, 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge, ge, p1,
                                                               (uint32_t *)scratch, spw, queue);
    return hipGetLastError();
}

// intra-pair pass 1: one block of four waves per pair, one block per CU (the
// four strip profiles take up to 100 KB of LDS); the row buffers of the
// block's slots are four of the per-wave boundary buffers
constexpr int kIntraBlocks = 256;

typedef hipError_t (*PIFn)(int, const uint8_t *, const PairDesc *, const int *, const int *, const int8_t *, int, int,
                           SwPass1Out *, int *, int64_t, int *, unsigned long long *, hipStream_t);

template <int R>
hipError_t launch_pi(int bin, const uint8_t *codes, const PairDesc *pairs, const int *idx, const int *starts,
                     const int8_t *blosum, int go_ge, int ge, SwPass1Out *p1, int *scratch, int64_t spw, int *queue,
                     unsigned long long *flag, hipStream_t s) {
    sw_intra_pass1_kernel<R><<<kIntraBlocks, 64 * kIntraWaves, 0, s>>>(codes, pairs, idx, starts, bin, blosum, go_ge,
                                                                      ge, p1, scratch, spw, queue, flag);
    return hipGetLastError();
}

typedef hipError_t (*P1Fn)(int, int, const uint8_t *, const PairDesc *, const int *, const int *, const int8_t *, int,
                           int, SwPass1Out *, int *, int64_t, int *, hipStream_t);
typedef hipError_t (*P2Fn)(int, int, const uint8_t *, const PairDesc *, const int *, const int *, const int8_t *, int,
                           int, int, int, const SwPass1Out *, pastis_pair_record *, int *, int64_t, int *,
                           hipStream_t);

const P1Fn kP1[kNumBins] = {launch_p1<1>,  launch_p1<2>,  launch_p1<3>,  launch_p1<4>,  launch_p1<5>,  launch_p1<6>,
                            launch_p1<7>,  launch_p1<8>,  launch_p1<9>,  launch_p1<10>, launch_p1<11>, launch_p1<12>,
                            launch_p1<13>, launch_p1<14>, launch_p1<15>, launch_p1<16>, launch_p1<9>,  launch_p1<10>,
                            launch_p1<11>, launch_p1<12>, launch_p1<13>, launch_p1<14>, launch_p1<15>, launch_p1<16>,
                            launch_p1<9>,  launch_p1<10>, launch_p1<11>, launch_p1<12>, launch_p1<13>, launch_p1<14>,
                            launch_p1<15>, launch_p1<16>};
typedef hipError_t (*P16Fn)(int, int, bool, const uint8_t *, const PairDesc *, const int *, const int *,
                            const int *, const int8_t *, int, int, SwPass1Out *, int *, hipStream_t);
const P16Fn kP16[kMax16R] = {launch_p16<1>,  launch_p16<2>,  launch_p16<3>,  launch_p16<4>,
                            launch_p16<5>,  launch_p16<6>,  launch_p16<7>,  launch_p16<8>,
                            launch_p16<9>,  launch_p16<10>, launch_p16<11>, launch_p16<12>,
                            launch_p16<13>, launch_p16<14>, launch_p16<15>, launch_p16<16>};
const PIFn kPI[kMaxR - kMultiMinR + 1] = {launch_pi<9>,  launch_pi<10>, launch_pi<11>, launch_pi<12>,
                                          launch_pi<13>, launch_pi<14>, launch_pi<15>, launch_pi<16>};
const P1Fn kP16M[kMaxR - kMultiMinR + 1] = {launch_p16m<9>,  launch_p16m<10>, launch_p16m<11>, launch_p16m<12>,
                                           launch_p16m<13>, launch_p16m<14>, launch_p16m<15>, launch_p16m<16>};
const P1Fn kPB[kNumBins] = {launch_pb<1>,  launch_pb<2>,  launch_pb<3>,  launch_pb<4>,  launch_pb<5>,  launch_pb<6>,
                            launch_pb<7>,  launch_pb<8>,  launch_pb<9>,  launch_pb<10>, launch_pb<11>, launch_pb<12>,
                            launch_pb<13>, launch_pb<14>, launch_pb<15>, launch_pb<16>, launch_pb<9>,  launch_pb<10>,
                            launch_pb<11>, launch_pb<12>, launch_pb<13>, launch_pb<14>, launch_pb<15>, launch_pb<16>,
                            launch_pb<9>,  launch_pb<10>, launch_pb<11>, launch_pb<12>, launch_pb<13>, launch_pb<14>,
                            launch_pb<15>, launch_pb<16>};
const P2Fn kP2[kNumBins] = {launch_p2<1>,  launch_p2<2>,  launch_p2<3>,  launch_p2<4>,  launch_p2<5>,  launch_p2<6>,
                            launch_p2<7>,  launch_p2<8>,  launch_p2<9>,  launch_p2<10>, launch_p2<11>, launch_p2<12>,
                            launch_p2<13>, launch_p2<14>, launch_p2<15>, launch_p2<16>, launch_p2<9>,  launch_p2<10>,
                            launch_p2<11>, launch_p2<12>, launch_p2<13>, launch_p2<14>, launch_p2<15>, launch_p2<16>,
                            launch_p2<9>,  launch_p2<10>, launch_p2<11>, launch_p2<12>, launch_p2<13>, launch_p2<14>,
                            launch_p2<15>, launch_p2<16>};

// Resident blocks per CU of the one-strip statistics kernels: they keep no
// profile in LDS, so registers set their occupancy, which the runtime reports
// for the compiled code; a grid of that many blocks per CU drains each bin.
int stats_blocks_per_cu[kMaxR + 1];

template <int R>
void stats_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sw_pass2_kernel<R, false>, 64 * wpb32(R), 0) != hipSuccess ||
        nb < 1) {
        (void)hipGetLastError();
        nb = 2;
    }
    stats_blocks_per_cu[R] = nb;
}

template <int... Rs>
void stats_occupancy_all(std::integer_sequence<int, Rs...>) {
    (stats_occupancy<Rs + 1>(), ...);
}

}  // namespace

void sw_init_occupancy() {
    if (stats_blocks_per_cu[1] == 0) stats_occupancy_all(std::make_integer_sequence<int, kMaxR>{});
}

int sw_num_bins() { return kNumBins; }

void sw_bin_shape(int bin, int32_t *rows_per_lane, int32_t *multi) {
    *multi = bin >= kMultiBin;
    *rows_per_lane = rows_of_bin(bin);
}

// Blocks per bin launch: the blocks of the bin's LDS footprint (25 codes x
// 64 lanes x 4, 8 or 16 profile bytes per wave) resident on 256 CUs at once;
// the grid-stride loop reads the bin size on the device.
static int blocks_for_bin(int bin) {
    const int r = rows_of_bin(bin);
    return r <= 4 ? 256 * 6 : (r > 8 && r <= 12) ? 256 * 4 : 256 * 3;
}

// Only the multi-strip bins use the boundary buffers (one per wave of the
// grid, 32-bit or 16-bit kernel).
int sw_one_strip_max_rows() { return kWave * kSingleBins; }

int64_t sw_scratch_waves() {
    int64_t w = 0;
    for (int b = kMultiBin; b < kNumBins; ++b) {
        w = std::max<int64_t>(w, (int64_t)blocks_for_bin(b) * wpb32(rows_of_bin(b)));
        w = std::max<int64_t>(w, (int64_t)blocks16m() * wpb16(rows_of_bin(b)));
        w = std::max<int64_t>(w, (int64_t)kIntraBlocks * kIntraWaves);
    }
    return w;
}

// The 16-bit profile holds each biased score s + o + e in one byte, with
// s <= 11 in BLOSUM62; other gap costs run in 32-bit lanes.
bool sw16_supported(const Scoring &sc) {
    const int oe = sc.gap_open + sc.gap_extend;
    return oe >= 4 && oe + 11 <= 255;
}

bool sw_bin_is16(int bin, int max16) {
    return (bin < kSingleBins || bin >= kMulti16Bin) && rows_of_bin(bin) <= max16;
}

hipError_t launch_sw(pastis_ctx *ctx, const uint8_t *codes, const PairDesc *pairs, int64_t npairs,
                     const int8_t *blosum, const Scoring &sc, SwPass1Out *p1, pastis_pair_record *out,
                     const SwWork &wk, int stats_mode, int max16, int grid_scale, int grid_scale_wide, int intra,
                     int narrow16, int long_blocks, bool timed, hipStream_t s) {
    // timed = false (graph capture): no stage or per-bin events
    // multi-strip launches: at most long_blocks blocks per CU (they run beside
    // the one-strip bins on the second stream; fewer resident waves leave the
    // one-strip kernels more room).  Fewer blocks than the default never
    // exceed the boundary buffers, which are sized for the default grids.
    auto long_cap = [&](int blocks) { return std::min(blocks, 256 * long_blocks); };
    const bool use16 = max16 > 0;
    auto begin = [&](int st) { return timed ? stage_begin(ctx, st, s) : hipSuccess; };
    auto end = [&](int st) { return timed ? stage_end(ctx, st, s) : hipSuccess; };
    auto mark = [&](hipEvent_t ev, hipStream_t st) { return timed ? hipEventRecord(ev, st) : hipSuccess; };
    // multi-strip bins (long sequences a, few pairs, long tails) run on the
    // context's second stream beside the one-strip bins; they share the
    // boundary buffers, so they stay in order among themselves there
    const hipStream_t ls = ctx->long_stream;
    auto fork = [&](int i) {
        hipError_t r = hipEventRecord(ctx->long_fork[i], s);
        return r != hipSuccess ? r : hipStreamWaitEvent(ls, ctx->long_fork[i], 0);
    };
    auto join = [&](int i) {
        hipError_t r = hipEventRecord(ctx->long_join[i], ls);
        return r != hipSuccess ? r : hipStreamWaitEvent(s, ctx->long_join[i], 0);
    };
    if (npairs <= 0) return hipSuccess;
    const int go_ge = sc.gap_open + sc.gap_extend, ge = sc.gap_extend;
    // Every launch drains its bin's work queue with a resident grid (times
    // the grid scale); no launch needs more blocks than the call's pairs
    // could fill (per_block pairs each).
    auto capped = [&](int blocks, int per_block) {
        const int64_t fill = (npairs + per_block - 1) / per_block;
        return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, fill));
    };
    const int nb = (int)((npairs + 255) / 256);
    hipError_t e = begin(kStSched);
    if (e != hipSuccess) return e;
    sw_bin1_kernel<<<nb, 256, 0, s>>>(pairs, npairs, wk.bin_of, wk.counters, wk.queue);
    if ((e = launch_bins(wk.bin_of, npairs, kNumBins, wk.counts, wk.starts, wk.cursor, wk.idx, s)) != hipSuccess)
        return e;
    const int *idx1 = wk.idx;
    if (use16) {
        // pair up pairs of one sequence a with similar column counts
        sw_pair_keys_kernel<<<nb, 256, 0, s>>>(pairs, wk.bin_of, npairs, wk.sort_keys, (uint32_t *)wk.idx);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        bool alt = false;
        if ((e = radix_sort(wk.sort_keys, (uint32_t *)wk.idx, wk.sort_keys_alt, wk.sort_vals_alt, npairs,
                            kPairKeyBits, wk.sort_temp, s, &alt)) != hipSuccess)
            return e;
        if (alt) idx1 = (const int *)wk.sort_vals_alt;
        sw_split_kernel<<<1, 64, 0, s>>>(alt ? wk.sort_keys_alt : wk.sort_keys, wk.starts, wk.split);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = end(kStSched)) != hipSuccess || (e = begin(kStAlign1)) != hipSuccess || (e = fork(0)) != hipSuccess)
        return e;
    // long bins first, so that their tails overlap the one-strip bins
    for (int k = 0; k < kNumBins; ++k) {
        const int bin = (k + kMultiBin) % kNumBins;
        const hipStream_t st = bin >= kMultiBin ? ls : s;
        if ((e = mark(ctx->bin_ev[2 * bin], st)) != hipSuccess) return e;
        // multi-strip bins use per-wave boundary buffers: they keep their grid
        const int R = rows_of_bin(bin);
        const int scale = bin >= kMultiBin ? 1 : R <= 8 ? grid_scale : grid_scale_wide;
        if (sw_bin_is16(bin, max16) && bin >= kMulti16Bin)
            e = kP16M[bin - kMulti16Bin](bin, long_cap(blocks16m()), codes, pairs, idx1, wk.starts, blosum, go_ge, ge,
                                         p1, wk.scratch, wk.scratch_per_wave, wk.queue, st);
        else if (intra && bin >= kMultiBin)
            e = kPI[R - kMultiMinR](bin, codes, pairs, idx1, wk.starts, blosum, go_ge, ge, p1, wk.scratch,
                                    wk.scratch_per_wave, wk.queue, wk.counters + kCounterIntraFlag, st);
        else if (sw_bin_is16(bin, max16))
            e = kP16[bin](bin, capped(scale * blocks16(R), pairs_per_block16(R, R <= narrow16)), R <= narrow16, codes,
                          pairs, idx1, wk.starts, wk.split, blosum, go_ge, ge, p1, wk.queue, st);
        else
            e = kP1[bin](bin,
                         capped(bin >= kMultiBin ? long_cap(blocks_for_bin(bin)) : scale * blocks_for_bin(bin),
                                wpb32(R)),
                         codes, pairs, idx1, wk.starts, blosum, go_ge, ge, p1, wk.scratch, wk.scratch_per_wave,
                         wk.queue, st);
        if (e != hipSuccess) return e;
        if ((e = mark(ctx->bin_ev[2 * bin + 1], st)) != hipSuccess) return e;
    }
    if ((e = join(0)) != hipSuccess || (e = end(kStAlign1)) != hipSuccess || (e = begin(kStAlign2)) != hipSuccess)
        return e;
    // the start-bound and statistics launches take the same grid scales
    // (multi-strip bins keep a resident grid: one boundary buffer per wave)
    auto scale2 = [&](int bin) {
        return bin >= kMultiBin ? 1 : rows_of_bin(bin) <= 8 ? grid_scale : grid_scale_wide;
    };
    auto blocks2 = [&](int bin) {
        return bin >= kMultiBin ? long_cap(blocks_for_bin(bin)) : scale2(bin) * blocks_for_bin(bin);
    };
    auto blocks_stats = [&](int bin) {
        const int per_cu = stats_blocks_per_cu[rows_of_bin(bin)];
        return bin >= kMultiBin || per_cu < 1 ? blocks2(bin) : scale2(bin) * 256 * per_cu;
    };
    sw_bin2_kernel<<<nb, 256, 0, s>>>(pairs, p1, npairs, sc.cov_pct, stats_mode, sc.direct_pct, out, wk.bin_of,
                                      wk.counters);
    if ((e = launch_bins(wk.bin_of, npairs, kNumBins, wk.counts, wk.starts2, wk.cursor, wk.idx2, s)) != hipSuccess)
        return e;
    if (stats_mode == 0) {
        // start bound, then only the pairs whose coverage can still hold
        if ((e = fork(1)) != hipSuccess) return e;
        for (int k = 0; k < kNumBins; ++k) {
            const int bin = (k + kMultiBin) % kNumBins;
            const hipStream_t st = bin >= kMultiBin ? ls : s;
            const int R = rows_of_bin(bin);
            e = kPB[bin](bin, capped(blocks2(bin), wpb32(R)), codes, pairs,
                         wk.idx2, wk.starts2, blosum, go_ge, ge, p1, wk.scratch, wk.scratch_per_wave,
                         wk.queue + kNumBins, st);
            if (e != hipSuccess) return e;
        }
        if ((e = join(1)) != hipSuccess) return e;
        sw_bin3_kernel<<<nb, 256, 0, s>>>(pairs, p1, npairs, sc.cov_pct, out, wk.bin_of, wk.counters);
        if ((e = launch_bins(wk.bin_of, npairs, kNumBins, wk.counts, wk.starts2, wk.cursor, wk.idx2, s)) !=
            hipSuccess)
            return e;
    }
    if ((e = fork(2)) != hipSuccess) return e;
    for (int k = 0; k < kNumBins; ++k) {
        const int bin = (k + kMultiBin) % kNumBins;
        const hipStream_t st = bin >= kMultiBin ? ls : s;
        const int R = rows_of_bin(bin);
        e = kP2[bin](bin, capped(blocks_stats(bin), wpb32(R)), codes, pairs,
                     wk.idx2, wk.starts2, blosum, go_ge, ge, sc.cov_pct, sc.id_pct, p1, out, wk.scratch,
                     wk.scratch_per_wave, wk.queue + 2 * kNumBins, st);
        if (e != hipSuccess) return e;
    }
    if ((e = join(2)) != hipSuccess) return e;
    return end(kStAlign2);
}

}  // namespace pastis
