// Smith-Waterman alignment of candidate pairs (Section IV-E), one 64-lane
// wavefront per pair, 32-bit DP words.
//
// Layout: the rows of the shorter sequence a are split into strips of 64*R
// rows; lane l of the wave owns rows [l*R, l*R + R) of the strip and sweeps
// the columns of b with a one-column skew per lane (lane l is at column t - l
// in step t), so all of a lane's DP state lives in registers and only the
// bottom row of its block crosses to the next lane, once per step.  Between
// strips the bottom row of the strip goes through a per-wave global buffer.
//
// Substitution scores come from a per-lane profile in LDS: for every column
// residue code c, the R scores of the lane's rows packed as R int8, read with
// one 64-bit LDS load per step.
//
// Pass 1 computes the score and the canonical end (the smallest row, then
// column, holding the maximum).  Pass 2 recomputes the rectangle
// [0, end_a] x [0, end_b] carrying, for every cell and state (H, E, F), the
// start cell, identical pairs and diagonal columns of the canonical path that
// ends there: the predecessor each cell takes is the one a traceback would
// take (diagonal before horizontal before vertical gap, extension before
// opening; a zero cell starts a new path), so the statistics at the end cell
// are those of the traceback without storing it.
#include "internal.hpp"

namespace pastis {
namespace {

constexpr int kWave = 64;
constexpr int kNeg = -(1 << 28);
constexpr int kWavesPerBlock = 4;
constexpr int kProfCodes = kAlpha + 1;  // 24 residues + the pad code

__device__ __forceinline__ int shfl_up1(int v) { return __shfl_up(v, 1, kWave); }

template <int R>
__device__ __forceinline__ void build_profile(uint64_t (*prof)[kWave], const int8_t *sblosum, const uint8_t *a, int la,
                                              int base, int lane) {
    uint8_t ar[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ar[r] = (base + r < la) ? a[base + r] : (uint8_t)kPadCode;
    for (int c = 0; c < kProfCodes; ++c) {
        uint64_t w = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) w |= (uint64_t)(uint8_t)sblosum[ar[r] * kProfCodes + c] << (8 * r);
        prof[c][lane] = w;
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

template <int R>
__global__ __launch_bounds__(256) void sw_pass1_kernel(const uint8_t *__restrict__ codes,
                                                       const PairDesc *__restrict__ pairs, int64_t npairs,
                                                       const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                       SwPass1Out *__restrict__ out, int2 *__restrict__ scratch,
                                                       int64_t scratch_per_wave) {
    __shared__ uint64_t prof_all[kWavesPerBlock][kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    uint64_t(*prof)[kWave] = prof_all[wave];
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int2 *bnd = scratch + gwave * scratch_per_wave;

    for (int64_t q = gwave; q < npairs; q += (int64_t)gridDim.x * kWavesPerBlock) {
        const PairDesc pd = pairs[q];
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int la = pd.la, lb = pd.lb;
        unsigned long long best = 0;  // (score << 32) | ~(row << 16 | col)
        for (int r0 = 0; r0 < la && lb > 0; r0 += kWave * R) {
            const int base = r0 + lane * R;
            build_profile<R>(prof, sblosum, a, la, base, lane);
            const bool first = (r0 == 0);
            const bool has_next = (r0 + kWave * R) < la;
            int H[R], E[R], rmax[R], rcol[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                H[r] = 0;
                E[r] = kNeg;
                rmax[r] = 0;
                rcol[r] = 0;
            }
            int hlast = 0, flast = kNeg, hdiag0 = 0;
            int cres = kPadCode;  // residue of this lane's current column
            const int steps = lb + kWave - 1;
            for (int t = 0; t < steps; ++t) {
                const int j = t - lane;
                int rh = shfl_up1(hlast), rf = shfl_up1(flast);
                int rc = shfl_up1(cres);
                if (lane == 0) {
                    rc = (t < lb) ? b[t] : kPadCode;
                    if (first) {
                        rh = 0;
                        rf = kNeg;
                    } else if (t < lb) {
                        const int2 v = bnd[t];
                        rh = v.x;
                        rf = v.y;
                    }
                }
                cres = rc;
                const bool valid = (j >= 0) && (j < lb);
                const uint64_t pw = prof[cres][lane];
                int hdiag = hdiag0, hup = rh, fup = rf;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int sigma = (int)(int8_t)(pw >> (8 * r));
                    const int e = max(E[r] - ge, H[r] - go_ge);
                    const int f = max(fup - ge, hup - go_ge);
                    const int h = max(max(hdiag + sigma, 0), max(e, f));
                    hdiag = H[r];
                    H[r] = h;
                    E[r] = e;
                    hup = h;
                    fup = f;
                    if (valid && h > rmax[r]) {
                        rmax[r] = h;
                        rcol[r] = j;
                    }
                }
                hlast = hup;
                flast = fup;
                hdiag0 = rh;
                if (has_next && lane == kWave - 1 && valid) bnd[j] = make_int2(hlast, flast);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (base + r < la && rmax[r] > 0) {
                    const unsigned pos = ((unsigned)(base + r) << 16) | (unsigned)rcol[r];
                    const unsigned long long key = ((unsigned long long)(unsigned)rmax[r] << 32) | (unsigned)(~pos);
                    best = key > best ? key : best;
                }
            }
            __threadfence_block();  // the next strip's lane 0 reads what lane 63 wrote
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

struct Stat {
    unsigned beg;  // (row << 16) | col of the first aligned pair
    unsigned md;   // (identical pairs << 16) | diagonal columns
};

__device__ __forceinline__ Stat shfl_up_stat(Stat s) {
    Stat o;
    o.beg = (unsigned)shfl_up1((int)s.beg);
    o.md = (unsigned)shfl_up1((int)s.md);
    return o;
}

__device__ __forceinline__ Stat sel(bool c, Stat x, Stat y) { return c ? x : y; }

template <int R>
__global__ __launch_bounds__(256) void sw_pass2_kernel(const uint8_t *__restrict__ codes,
                                                       const PairDesc *__restrict__ pairs, int64_t npairs,
                                                       const int8_t *__restrict__ blosum, int go_ge, int ge,
                                                       int cov_pct, int id_pct, int full,
                                                       const SwPass1Out *__restrict__ p1,
                                                       pastis_pair_record *__restrict__ out,
                                                       int4 *__restrict__ scratch, int64_t scratch_per_wave) {
    __shared__ uint64_t prof_all[kWavesPerBlock][kProfCodes][kWave];
    __shared__ int8_t sblosum[kProfCodes * kProfCodes];
    load_blosum(sblosum, blosum);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    uint64_t(*prof)[kWave] = prof_all[wave];
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    // per column: (H, F, H.beg, H.md) and (F.beg, F.md) of the strip's bottom row
    int4 *bnd_a = scratch + gwave * scratch_per_wave;
    int2 *bnd_b = (int2 *)(bnd_a + scratch_per_wave / 2);

    for (int64_t q = gwave; q < npairs; q += (int64_t)gridDim.x * kWavesPerBlock) {
        const PairDesc pd = pairs[q];
        const SwPass1Out r1 = p1[q];
        const int la_full = pd.la;
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
        // coverage needs span_a >= cov% of la, and span_a <= end_a + 1
        const bool need = r1.score > 0 && (full || 100LL * (r1.end_a + 1) >= (long long)cov_pct * la_full);
        if (!need) {
            if (lane == 0) out[q] = rec;
            continue;
        }
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int la = r1.end_a + 1, lb = r1.end_b + 1;  // the rectangle ending at the end cell
        Stat fin = {0u, 0u};
        for (int r0 = 0; r0 < la; r0 += kWave * R) {
            const int base = r0 + lane * R;
            build_profile<R>(prof, sblosum, a, la, base, lane);
            uint8_t ar[R];
#pragma unroll
            for (int r = 0; r < R; ++r) ar[r] = (base + r < la) ? a[base + r] : (uint8_t)kPadCode;
            const bool first = (r0 == 0);
            const bool has_next = (r0 + kWave * R) < la;
            int H[R], E[R];
            Stat sH[R], sE[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                H[r] = 0;
                E[r] = kNeg;
                sH[r] = Stat{0u, 0u};
                sE[r] = Stat{0u, 0u};
            }
            int hlast = 0, flast = kNeg, hdiag0 = 0;
            Stat shlast = {0u, 0u}, sflast = {0u, 0u}, sdiag0 = {0u, 0u};
            int cres = kPadCode;
            const int steps = lb + kWave - 1;
            for (int t = 0; t < steps; ++t) {
                const int j = t - lane;
                int rh = shfl_up1(hlast), rf = shfl_up1(flast);
                Stat rsh = shfl_up_stat(shlast), rsf = shfl_up_stat(sflast);
                int rc = shfl_up1(cres);
                if (lane == 0) {
                    rc = (t < lb) ? b[t] : kPadCode;
                    if (first) {
                        rh = 0;
                        rf = kNeg;
                        rsh = Stat{0u, 0u};
                        rsf = Stat{0u, 0u};
                    } else if (t < lb) {
                        const int4 v = bnd_a[t];
                        const int2 w = bnd_b[t];
                        rh = v.x;
                        rf = v.y;
                        rsh = Stat{(unsigned)v.z, (unsigned)v.w};
                        rsf = Stat{(unsigned)w.x, (unsigned)w.y};
                    }
                }
                cres = rc;
                const bool valid = (j >= 0) && (j < lb);
                const uint64_t pw = prof[cres][lane];
                int hdiag = hdiag0, hup = rh, fup = rf;
                Stat sdiag = sdiag0, shup = rsh, sfup = rsf;
                const unsigned here0 = ((unsigned)base << 16) | (unsigned)(j & 0xFFFF);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int sigma = (int)(int8_t)(pw >> (8 * r));
                    // horizontal gap: extend when it is at least as good as opening
                    const int e_ext = E[r] - ge, e_open = H[r] - go_ge;
                    const bool e_is_ext = e_ext >= e_open;
                    const int e = e_is_ext ? e_ext : e_open;
                    const Stat se = sel(e_is_ext, sE[r], sH[r]);
                    // vertical gap
                    const int f_ext = fup - ge, f_open = hup - go_ge;
                    const bool f_is_ext = f_ext >= f_open;
                    const int f = f_is_ext ? f_ext : f_open;
                    const Stat sf = sel(f_is_ext, sfup, shup);
                    // diagonal: a zero predecessor starts a new path here
                    const int d = hdiag + sigma;
                    const int h = max(max(d, 0), max(e, f));
                    Stat sd = sel(hdiag == 0, Stat{here0 + ((unsigned)r << 16), 0u}, sdiag);
                    sd.md += (ar[r] == (uint8_t)cres) ? 0x10001u : 1u;
                    const Stat sh = sel(h == d, sd, sel(h == e, se, sf));
                    hdiag = H[r];
                    sdiag = sH[r];
                    H[r] = h;
                    E[r] = e;
                    sH[r] = sh;
                    sE[r] = se;
                    hup = h;
                    fup = f;
                    shup = sh;
                    sfup = sf;
                    if (valid && j == lb - 1 && base + r == la - 1) fin = sh;
                }
                hlast = hup;
                flast = fup;
                shlast = shup;
                sflast = sfup;
                hdiag0 = rh;
                sdiag0 = rsh;
                if (has_next && lane == kWave - 1 && valid) {
                    bnd_a[j] = make_int4(hlast, flast, (int)shlast.beg, (int)shlast.md);
                    bnd_b[j] = make_int2((int)sflast.beg, (int)sflast.md);
                }
            }
            __threadfence_block();
        }
        // the end cell belongs to exactly one lane; combine by max (others hold 0)
        unsigned long long key = ((unsigned long long)fin.beg << 32) | fin.md;
        key = wave_max_u64(key);
        if (lane == 0) {
            const unsigned beg = (unsigned)(key >> 32), md = (unsigned)key;
            rec.beg_a = (int32_t)(beg >> 16);
            rec.beg_b = (int32_t)(beg & 0xFFFF);
            rec.matches = (int32_t)(md >> 16);
            const int32_t diag = (int32_t)(md & 0xFFFF);
            rec.columns = (rec.end_a - rec.beg_a + 1) + (rec.end_b - rec.beg_b + 1) - diag;
            const long long span = (long long)rec.end_a - rec.beg_a + 1;
            rec.passed = (100LL * rec.matches >= (long long)id_pct * rec.columns) &&
                         (100LL * span >= (long long)cov_pct * la_full);
            out[q] = rec;
        }
    }
}

}  // namespace

hipError_t launch_sw(const uint8_t *codes, const PairDesc *pairs, int64_t npairs, const int8_t *blosum,
                     const Scoring &sc, SwPass1Out *p1, pastis_pair_record *out, int32_t *scratch,
                     int64_t scratch_ints_per_wave, int full, int waves, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    const int go_ge = sc.gap_open + sc.gap_extend, ge = sc.gap_extend;
    int blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks < 1) blocks = 1;
    sw_pass1_kernel<8><<<blocks, 256, 0, s>>>(codes, pairs, npairs, blosum, go_ge, ge, p1, (int2 *)scratch,
                                              scratch_ints_per_wave / 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sw_pass2_kernel<8><<<blocks, 256, 0, s>>>(codes, pairs, npairs, blosum, go_ge, ge, sc.cov_pct, sc.id_pct, full,
                                              p1, out, (int4 *)scratch, scratch_ints_per_wave / 4);
    return hipGetLastError();
}

}  // namespace pastis
