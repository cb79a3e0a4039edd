// Seed-and-extend with gapped x-drop (Section IV-E, XD), one 64-lane
// wavefront per candidate pair.
//
// For each stored seed (at most two), the k seed columns are scored, then the
// alignment is extended to the right of the seed and, on reversed prefixes,
// to the left.  An extension is an anchored affine-gap DP (no zero floor)
// processed by anti-diagonals d = u + v: a cell with no live predecessor is
// not computed; a computed cell is live when its score is at least
// (best score of earlier anti-diagonals) - X; the extension stops at the first
// anti-diagonal without a live cell.  Its end is the best live cell, the
// earliest anti-diagonal and then the smallest row winning ties.  The pair
// keeps the best-scoring seed among those that pass the identity / coverage
// cut (the first seed on a tie), or the best-scoring seed when none passes.
//
// Layout.  Every cell carries, for each state (H, E, F), the packed
// (identical pairs << 16 | diagonal columns) of the canonical path reaching
// it: each cell takes the predecessor a traceback would take (diagonal, then
// horizontal, then vertical gap; extension before opening), and since every
// extension path starts at the anchor, columns = u + v - diagonal columns.
// The first pass keeps the band of an anti-diagonal in registers (cell u in
// lane u mod 64, see extend_reg); pairs with a band wider than 64 rows are
// redone by a second kernel that keeps the last three anti-diagonals in a
// ring in global memory indexed by u.
#include <climits>

#include "internal.hpp"

namespace pastis {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kNeg = -(1 << 28);
constexpr int kGlobalCap = 65536;
constexpr int kProfCodes = kAlpha + 1;
// extensions of at most this many rows and columns keep both sequences whole
// in the wave's LDS buffer (kWaveLds bytes, also the two rings' home)
constexpr int kWholeMax = 1024;
constexpr int kWaveLds = 3 * (kWholeMax + 64);
static_assert(kWaveLds >= 768, "the rings fit the buffer");

struct Ring {
    int *H, *E, *F;
    unsigned *SH, *SE, *SF;  // 3 slots of `cap` entries each
    int cap;
};

struct Ext {
    int score, u, v;
    unsigned md;
    int cells;
    bool overflow;
};

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

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One extension from the anchor over a'[t] = a0[t * adir], b'[t] = b0[t * bdir].
template <bool GLOBAL>
__device__ Ext extend(const uint8_t *a0, int la, int adir, const uint8_t *b0, int lb, int bdir, const int8_t *sbl,
                      int o, int e, int X, const Ring &R, int lane) {
    const int oe = o + e;
    const int mask = R.cap - 1;
    if (lane == 0) {  // anti-diagonal 0: the anchor, slot 0
        R.H[0] = 0;
        R.E[0] = kNeg;
        R.F[0] = kNeg;
        R.SH[0] = 0u;
        R.SE[0] = 0u;
        R.SF[0] = 0u;
    }
    if (GLOBAL) __threadfence_block();
    int clo1 = 0, chi1 = 0, llo1 = 0, lhi1 = 0;  // anti-diagonal d-1: computed / live ranges
    int clo2 = 1, chi2 = 0, llo2 = 1, lhi2 = 0;  // d-2 (none yet)
    int best = 0, bu = 0, bv = 0;
    unsigned bmd = 0u;
    int cells = 0;
    bool overflow = false;
    const int dmax = la + lb;
    for (int d = 1; d <= dmax; ++d) {
        int lo = INT_MAX, hi = -1;
        if (llo1 <= lhi1) {
            lo = llo1;
            hi = lhi1 + 1;
        }
        if (llo2 <= lhi2) {
            lo = min(lo, llo2 + 1);
            hi = max(hi, lhi2 + 1);
        }
        lo = max(lo, max(0, d - lb));
        hi = min(hi, min(d, la));
        if (lo > hi) break;
        if (hi - lo + 1 > R.cap) {
            overflow = true;
            break;
        }
        const int s0 = (d % 3) * R.cap, s1 = ((d + 2) % 3) * R.cap, s2 = ((d + 1) % 3) * R.cap;
        const int floor_ = best - X;
        int lbest = INT_MIN, lbu = 0;
        unsigned lbmd = 0u;
        int lmin = INT_MAX, lmax = -1;
        for (int u0 = lo; u0 <= hi; u0 += kWave) {
            const int u = u0 + lane;
            if (u > hi) continue;
            const int v = d - u;
            int Hu = kNeg, Fu = kNeg, Hl = kNeg, El = kNeg, Hd = kNeg;
            unsigned sHu = 0u, sFu = 0u, sHl = 0u, sEl = 0u, sHd = 0u;
            if (u - 1 >= clo1 && u - 1 <= chi1) {  // (u-1, v): vertical
                const int x = s1 + ((u - 1) & mask);
                Hu = R.H[x];
                Fu = R.F[x];
                sHu = R.SH[x];
                sFu = R.SF[x];
            }
            if (v >= 1 && u >= clo1 && u <= chi1) {  // (u, v-1): horizontal
                const int x = s1 + (u & mask);
                Hl = R.H[x];
                El = R.E[x];
                sHl = R.SH[x];
                sEl = R.SE[x];
            }
            if (u >= 1 && v >= 1 && u - 1 >= clo2 && u - 1 <= chi2) {  // (u-1, v-1)
                const int x = s2 + ((u - 1) & mask);
                Hd = R.H[x];
                sHd = R.SH[x];
            }
            const bool lu = Hu > kNeg / 2, ll = Hl > kNeg / 2, ld = Hd > kNeg / 2;
            const bool any = lu || ll || ld;
            const int e_ext = El - e, e_open = Hl - oe;
            const bool ee = e_ext >= e_open;
            const int E_ = ee ? e_ext : e_open;
            const int f_ext = Fu - e, f_open = Hu - oe;
            const bool fe = f_ext >= f_open;
            const int F_ = fe ? f_ext : f_open;
            int D_ = kNeg;
            unsigned sD = 0u;
            if (ld) {
                const int ca = a0[(u - 1) * adir], cb = b0[(v - 1) * bdir];
                D_ = Hd + sbl[ca * kProfCodes + cb];
                sD = sHd + (ca == cb ? 0x10001u : 1u);
            }
            const int H_ = max(D_, max(E_, F_));
            const unsigned sE_ = ee ? sEl : sHl;
            const unsigned sF_ = fe ? sFu : sHu;
            const unsigned sH_ = (ld && H_ == D_) ? sD : (H_ == E_ ? sE_ : sF_);
            const bool live = any && H_ >= floor_;
            cells += any ? 1 : 0;
            const int x = s0 + (u & mask);
            R.H[x] = live ? H_ : kNeg;
            R.E[x] = live ? E_ : kNeg;
            R.F[x] = live ? F_ : kNeg;
            R.SH[x] = sH_;
            R.SE[x] = sE_;
            R.SF[x] = sF_;
            if (live) {
                lmin = min(lmin, u);
                lmax = max(lmax, u);
                if (H_ > lbest) {  // u increases along a lane: the first maximum wins
                    lbest = H_;
                    lbu = u;
                    lbmd = sH_;
                }
            }
        }
        if (GLOBAL) __threadfence_block();
        // best live cell of this anti-diagonal: highest score, then smallest u
        unsigned long long key = 0ull;
        if (lbest != INT_MIN)
            key = ((unsigned long long)(unsigned)(lbest + (1 << 30)) << 32) | (0xFFFFFFFFu - (unsigned)lbu);
        const unsigned long long wkey = wave_max_u64(key);
        const int wmin = wave_min_i(lmin), wmax = wave_max_i(lmax);
        clo2 = clo1;
        chi2 = chi1;
        llo2 = llo1;
        lhi2 = lhi1;
        clo1 = lo;
        chi1 = hi;
        if (wkey == 0ull) {
            llo1 = 1;
            lhi1 = 0;
            break;
        }
        llo1 = wmin;
        lhi1 = wmax;
        const int dbest = (int)(unsigned)(wkey >> 32) - (1 << 30);
        if (dbest > best) {
            const unsigned long long hit = __ballot(key == wkey);
            const int winner = __ffsll((long long)hit) - 1;
            best = dbest;
            bu = (int)(0xFFFFFFFFu - (unsigned)wkey);
            bv = d - bu;
            bmd = (unsigned)__builtin_amdgcn_readlane((int)lbmd, winner);
        }
    }
    Ext r;
    r.score = best;
    r.u = bu;
    r.v = bv;
    r.md = bmd;
    r.cells = wave_sum_i(cells);
    r.overflow = overflow;
    return r;
}


// ---------------------------------------------------------------- register band
//
// The same extension with the band in registers: cell u of an anti-diagonal
// lives in lane u mod 64 (the computed range [lo, hi] must fit 64 rows, else
// the pair is redone with a ring in global memory).  Predecessors come from
// the lane itself (horizontal, d-1) and, by a one-lane wave rotation, from
// lane u-1 (vertical at d-1; diagonal at d-2, the rotation kept from the step
// before).  A predecessor counts only if its row was in the computed range of
// its anti-diagonal, so stale lanes never leak in.  Residues stream through
// 256-entry LDS rings per sequence, filled in 64-entry chunks one chunk ahead
// of the largest index the band can reach (the band moves at most one row and
// one column per anti-diagonal).

constexpr int kDppWaveRor1 = 0x13C;  // lane l receives lane l-1 (lane 0 from 63)

// a full rotation has no out-of-range lanes, so no prior value of the result
// register is needed
__device__ __forceinline__ int ror1(int v) { return __builtin_amdgcn_mov_dpp(v, kDppWaveRor1, 0xF, 0xF, false); }

// A ring holds residue codes times MUL (T wide enough): the rows' stream
// keeps code * 100 and the columns' code * 4, so one add gives a code pair's
// byte offset into the 25 x 25 tables of 32-bit entries.
template <typename T, int MUL>
struct Stream {
    const uint8_t *p;
    int len, dir;
    T *ring;      // 256 entries, index & 255
    int next;     // chunks [0, next) are in the ring
    int pending;  // this lane's element of chunk `next` (times MUL), loaded ahead
};

template <typename T, int MUL>
__device__ __forceinline__ int stream_elem(const Stream<T, MUL> &w, int c, int lane) {
    const int t = c * kWave + lane;
    return (t < w.len ? (int)w.p[(int64_t)t * w.dir] : kPadCode) * MUL;
}

template <typename T, int MUL>
__device__ __forceinline__ void stream_init(Stream<T, MUL> &w, int lane) {
    w.ring[lane] = (T)stream_elem(w, 0, lane);
    w.ring[kWave + lane] = (T)stream_elem(w, 1, lane);
    w.ring[2 * kWave + lane] = (T)(kPadCode * MUL);  // every ring entry is a valid code
    w.ring[3 * kWave + lane] = (T)(kPadCode * MUL);
    w.pending = stream_elem(w, 2, lane);
    w.next = 2;
}

// make every index <= frontier + 64 readable; frontier (wave-uniform) grows
// by at most one per call, so one chunk at a time suffices
template <typename T, int MUL>
__device__ __forceinline__ void stream_ensure(Stream<T, MUL> &w, int frontier, int lane) {
    if ((frontier >> 6) + 1 >= w.next) {
        w.ring[(w.next & 3) * kWave + lane] = (T)w.pending;
        ++w.next;
        w.pending = stream_elem(w, w.next, lane);
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ unsigned long long rotr64(unsigned long long m, int s) {
    return s == 0 ? m : (m >> s) | (m << (64 - s));
}

__device__ __forceinline__ int wave_max_dpp(int v) {
    // within rows of 16, then across rows; lane 63 ends with the maximum
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// An empty statement that hands x back in a scalar register: it emits no
// instruction, but the compiler can no longer fold the expressions on its two
// sides into one three-operand vector max / min, which would move the
// wave-uniform band range through vector registers and back (seven vector
// instructions instead of four scalar ones per anti-diagonal)
__device__ __forceinline__ void sgpr_opaque(int &x) { asm("" : "+s"(x)); }

// (unsigned)(x - base) < len: x in [base, base + len) with one compare
__device__ __forceinline__ bool in_range(int x, int base, int len) { return (unsigned)(x - base) < (unsigned)len; }

// Lane masks of one compare each (a ballot of a computed predicate costs a
// select and a second compare).  A lane that is not live holds kNeg in H1,
// below every bound these take, so H1 alone tells live lanes, those above
// the best score, and those equal to a live maximum.
__device__ __forceinline__ unsigned long long wave_mask_ne(int x, int y) { return __builtin_amdgcn_sicmp(x, y, 33); }
__device__ __forceinline__ unsigned long long wave_mask_gt(int x, int y) { return __builtin_amdgcn_sicmp(x, y, 38); }
__device__ __forceinline__ unsigned long long wave_mask_eq(int x, int y) { return __builtin_amdgcn_sicmp(x, y, 32); }

// WHOLE: both extension sequences fit the wave's LDS buffer whole (at most
// kWholeMax residues each): ring_a[u] holds the code of row u - 1 times 100
// (pad codes at 0 and past la) and ring_b[v + 63] the code of column v - 1
// times 4 (pad codes before and after), so every lane's reads stay in the buffer
// without index masks or refills.  Otherwise both stream through 256-entry
// rings.
template <bool WHOLE>
__device__ Ext extend_reg(const uint8_t *a0, int la, int adir, const uint8_t *b0, int lb, int bdir,
                          const int *sbl4, const unsigned *minc, int o, int e, int X, uint16_t *ring_a,
                          uint8_t *ring_b, int lane) {
    const int oe = o + e;
    Stream<uint16_t, 4 * kProfCodes> sa{a0, la, adir, ring_a, 0, 0};
    Stream<uint8_t, 4> sb{b0, lb, bdir, ring_b, 0, 0};
    if constexpr (WHOLE) {
        for (int t = lane; t < la + kWave; t += kWave)
            ring_a[t] = (uint16_t)((t >= 1 && t <= la ? (int)a0[(int64_t)(t - 1) * adir] : kPadCode) * 4 * kProfCodes);
        for (int t = lane; t < lb + kWave; t += kWave)
            ring_b[t] = (uint8_t)((t >= kWave ? (int)b0[(int64_t)(t - kWave) * bdir] : kPadCode) * 4);
        __builtin_amdgcn_wave_barrier();
    } else {
        stream_init(sa, lane);
        stream_init(sb, lane);
    }
    // anti-diagonal 0: the anchor in lane 0
    int H1 = lane == 0 ? 0 : kNeg, E1 = kNeg, F1 = kNeg;
    unsigned SH1 = 0u, SE1 = 0u, SF1 = 0u;
    int VH = kNeg;  // lane u-1's H two anti-diagonals back (rotated one step ago)
    unsigned VSH = 0u;
    // computed row ranges of anti-diagonals d-1 and d-2 as (first row,
    // count), and their live rows [s, e); s2p is d-2's first live row plus
    // one.  The range before anti-diagonal 0 bounds nothing.
    int c1 = 0, n1 = 1, s1 = 0, e1 = 1;
    int c2 = 0, n2 = 0, s2p = 1 << 24, e2 = -(1 << 24);
    int best = 0, bu = 0, bv = 0;
    unsigned bmd = 0u;
    int cells = 0;
    bool overflow = false;
    // past anti-diagonal la + lb the range is empty (lo >= d - lb > la >= hi)
    for (int d = 1;; ++d) {
        // both live ranges are non-empty: an empty one ends the loop
        int lo = min(s1, s2p), hi = max(e1, e2);
        int lo_floor = max(0, d - lb), hi_ceil = min(d, la);
        sgpr_opaque(lo_floor);
        sgpr_opaque(hi_ceil);
        lo = max(lo, lo_floor);
        hi = min(hi, hi_ceil);
        if (lo > hi) break;
        if (hi - lo + 1 > kWave) {
            overflow = true;
            break;
        }
        const int u = lo + ((lane - lo) & (kWave - 1));
        const int v = d - u;
        // predecessors: (u-1, v) and (u, v-1) at d-1, (u-1, v-1) at d-2; v >= 1
        // means u <= d-1, and rows of d-2 are <= d-2
        const int rH = ror1(H1), rF = ror1(F1);
        const unsigned rSH = (unsigned)ror1((int)SH1), rSF = (unsigned)ror1((int)SF1);
        // After every anti-diagonal a lane holds its row's live values or
        // kNeg, and the band's first row never decreases; so while the two
        // previous bands are narrower than 64 rows, every lane (and its
        // rotation) holds exactly the predecessor row it needs, or kNeg when
        // that row was not computed.  Only a band of 64 rows reuses a lane
        // for another row, and then the ranges are checked.
        int Hu = rH, Fu = rF, Hl = H1, El = E1, Hd = VH;
        if ((n1 | n2) & kWave) {  // a width of 64 (widths never exceed it)
            const int nh = uni(max(min(c1 + n1, d) - c1, 0));  // rows of d-1 in [c1, d-1]
            const bool okv = in_range(u, c1 + 1, n1);
            const bool okh = in_range(u, c1, nh);
            const bool okd = in_range(u, c2 + 1, n2);
            Hu = okv ? rH : kNeg;
            Fu = okv ? rF : kNeg;
            Hl = okh ? H1 : kNeg;
            El = okh ? E1 : kNeg;
            Hd = okd ? VH : kNeg;
        }
        const unsigned sHd = VSH;
        VH = rH;
        VSH = rSH;
        // residues of the diagonal move (indices always in range)
        int cab;  // a * 25 + b
        if constexpr (WHOLE) {
            cab = (int)ring_a[u] + (int)ring_b[v + kWave - 1];
        } else {
            stream_ensure(sa, hi - 1, lane);
            stream_ensure(sb, d - lo - 1, lane);
            cab = (int)ring_a[(u - 1) & 255] + (int)ring_b[(v - 1) & 255];
        }
        const int sig = *(const int *)((const char *)sbl4 + cab);
        const int e_ext = El - e, e_open = Hl - oe;
        const bool ee = e_ext >= e_open;
        const int E_ = max(e_ext, e_open);
        const int f_ext = Fu - e, f_open = Hu - oe;
        const bool fe = f_ext >= f_open;
        const int F_ = max(f_ext, f_open);
        const int D_ = Hd + sig;  // dead predecessors stay far below kNeg / 2
        const unsigned sD = sHd + *(const unsigned *)((const char *)minc + cab);
        const int H_ = max(D_, max(E_, F_));
        const unsigned sE_ = ee ? SE1 : SH1;
        const unsigned sF_ = fe ? rSF : rSH;
        // the diagonal wins ties
        const unsigned sEF = H_ == E_ ? sE_ : sF_;
        const unsigned sH_ = H_ == D_ ? sD : sEF;
        const bool any = u <= hi && max(Hd, max(Hu, Hl)) > kNeg / 2;
        const bool live = any && H_ >= best - X;
        cells += any ? 1 : 0;
        // Only H is cleared where the cell is dead.  A dead cell's E and F
        // are at most its H, below best - X; the gap chains they start only
        // fall, while best - X only rises, so they never reach a live
        // cell's H (nor tie with it) and choose neither its value nor its
        // statistics.
        H1 = live ? H_ : kNeg;
        E1 = E_;
        F1 = F_;
        SH1 = sH_;
        SE1 = sE_;
        SF1 = sF_;
        // live range and best cell of this anti-diagonal (u = lo + rotated lane)
        const int sh = lo & (kWave - 1);
        const unsigned long long lm = rotr64(wave_mask_ne(H1, kNeg), sh);
        c2 = c1;
        n2 = n1;
        s2p = s1 + 1;
        e2 = e1;
        c1 = lo;
        n1 = hi - lo + 1;
        if (lm == 0ull) break;
        s1 = lo + __ffsll((long long)lm) - 1;
        e1 = lo + 64 - __clzll((long long)lm);
        const unsigned long long up = wave_mask_gt(H1, best);
        if (up != 0ull) {
            const int dbest = wave_max_dpp(live ? H_ : INT_MIN);
            const unsigned long long hit = rotr64(wave_mask_eq(H1, dbest), sh);
            const int off = __ffsll((long long)hit) - 1;
            best = dbest;
            bu = lo + off;
            bv = d - bu;
            bmd = (unsigned)__builtin_amdgcn_readlane((int)sH_, bu & (kWave - 1));
        }
    }
    Ext r;
    r.score = best;
    r.u = bu;
    r.v = bv;
    r.md = bmd;
    r.cells = wave_sum_i(cells);
    r.overflow = overflow;
    return r;
}

struct SeedAln {
    int score, beg_a, end_a, beg_b, end_b, matches, columns, cells;
    bool overflow;
};

// GLOBAL = false: the register band (rings: 256 entries of code * 100 as
// uint16, then 256 of code * 4; sbl4 and minc: the score and the statistics
// increment of each code pair, 32-bit);
// GLOBAL = true: the ring in global memory.
template <bool GLOBAL>
__device__ SeedAln align_seed(const uint8_t *a, int la, const uint8_t *b, int lb, int pa, int pb, int k,
                              const int8_t *sbl, const int *sbl4, const unsigned *minc, int o, int e, int X,
                              const Ring &R,
                              uint8_t *rings, int lane) {
    int sc = 0, sm = 0;
    for (int t = 0; t < k; ++t) {
        const int ca = a[pa + t], cb = b[pb + t];
        sc += sbl[ca * kProfCodes + cb];
        sm += ca == cb;
    }
    Ext rt, lf;
    if constexpr (GLOBAL) {
        rt = extend<true>(a + pa + k, la - pa - k, 1, b + pb + k, lb - pb - k, 1, sbl, o, e, X, R, lane);
        lf = extend<true>(a + pa - 1, pa, -1, b + pb - 1, pb, -1, sbl, o, e, X, R, lane);
    } else {
        // whole sequences: kWholeMax + 64 entries of code * 100, then as many
        // of code * 4; rings: 256 entries of code * 100, then 256 of code * 4
        uint16_t *ring_a = (uint16_t *)rings;
        uint8_t *whole_b = rings + 2 * (kWholeMax + kWave), *ring_b = rings + 512;
        const int ra = la - pa - k, rb = lb - pb - k;
        rt = ra <= kWholeMax && rb <= kWholeMax
                 ? extend_reg<true>(a + pa + k, ra, 1, b + pb + k, rb, 1, sbl4, minc, o, e, X, ring_a, whole_b, lane)
                 : extend_reg<false>(a + pa + k, ra, 1, b + pb + k, rb, 1, sbl4, minc, o, e, X, ring_a, ring_b, lane);
        if (rt.overflow)
            lf = rt;
        else if (pa <= kWholeMax && pb <= kWholeMax)
            lf = extend_reg<true>(a + pa - 1, pa, -1, b + pb - 1, pb, -1, sbl4, minc, o, e, X, ring_a, whole_b, lane);
        else
            lf = extend_reg<false>(a + pa - 1, pa, -1, b + pb - 1, pb, -1, sbl4, minc, o, e, X, ring_a, ring_b, lane);
    }
    SeedAln s;
    s.score = lf.score + sc + rt.score;
    s.beg_a = pa - lf.u;
    s.beg_b = pb - lf.v;
    s.end_a = pa + k - 1 + rt.u;
    s.end_b = pb + k - 1 + rt.v;
    s.matches = (int)(lf.md >> 16) + sm + (int)(rt.md >> 16);
    s.columns = (lf.u + lf.v - (int)(lf.md & 0xFFFFu)) + k + (rt.u + rt.v - (int)(rt.md & 0xFFFFu));
    s.cells = lf.cells + rt.cells;
    s.overflow = lf.overflow || rt.overflow;
    return s;
}

__device__ __forceinline__ bool passes(const SeedAln &s, int la, int id_pct, int cov_pct) {
    if (s.score <= 0 || s.columns <= 0) return false;
    const long long span = (long long)s.end_a - s.beg_a + 1;
    return 100LL * s.matches >= (long long)id_pct * s.columns && 100LL * span >= (long long)cov_pct * la;
}

// GLOBAL = false: every pair of [0, npairs), LDS ring; pairs whose band
// outgrows it are listed in redo[] and left for GLOBAL = true, which walks
// that list with rings in global memory.
// The register band asks for eight waves per SIMD (at most 64 registers):
// its per-anti-diagonal chain of LDS reads (residues, then score and
// statistics increment) needs the other waves to hide it (0.82 s at six
// waves per SIMD against 0.74 s at eight on the large workload).
template <bool GLOBAL>
__global__ __launch_bounds__(256, GLOBAL ? 1 : 8) void xd_kernel(const uint8_t *__restrict__ codes, const PairDesc *__restrict__ pairs,
                                                 int64_t npairs, const int8_t *__restrict__ blosum, int k, int o, int e,
                                                 int X, int id_pct, int cov_pct, pastis_pair_record *__restrict__ out,
                                                 uint32_t *__restrict__ redo, uint32_t *__restrict__ n_redo,
                                                 int *__restrict__ gring, unsigned long long *__restrict__ counters) {
    __shared__ int8_t sbl[kProfCodes * kProfCodes];
    // the register band reads scores and statistics increments at the byte
    // offset 4 * (code_a * 25 + code_b) of 32-bit tables
    // per code pair: identical pairs << 16 | diagonal columns added by a match
    // or mismatch column (codes compared, as everywhere: two pad codes match)
    __shared__ unsigned minc[kProfCodes * kProfCodes];
    __shared__ int sbl4[GLOBAL ? 1 : kProfCodes * kProfCodes];
    for (int t = threadIdx.x; t < kProfCodes * kProfCodes; t += blockDim.x) {
        sbl[t] = blosum[t];
        if constexpr (!GLOBAL) sbl4[t] = blosum[t];
        minc[t] = t / kProfCodes == t % kProfCodes ? 0x10001u : 1u;
    }
    __shared__ __align__(16) uint8_t lds_rings[GLOBAL ? 1 : kWavesPerBlock * kWaveLds];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    Ring R{};
    uint8_t *rings = nullptr;
    if constexpr (GLOBAL) {
        int *base = gring + gwave * (int64_t)18 * kGlobalCap;
        R.cap = kGlobalCap;
        R.H = base;
        R.E = base + 3 * R.cap;
        R.F = base + 6 * R.cap;
        R.SH = (unsigned *)(base + 9 * R.cap);
        R.SE = (unsigned *)(base + 12 * R.cap);
        R.SF = (unsigned *)(base + 15 * R.cap);
    } else {
        rings = lds_rings + wave * kWaveLds;
    }
    const int64_t count = GLOBAL ? (int64_t)*n_redo : npairs;
    unsigned long long my_cells = 0;
    // register band: pairs claimed one at a time from the call's queue
    // counter (extension lengths vary widely); global ring: grid stride
    auto next = [&](int64_t w) -> int64_t {
        if constexpr (GLOBAL) {
            return w + (int64_t)gridDim.x * kWavesPerBlock;
        } else {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(&counters[kCounterXdQueue], 1ull);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
            return (int64_t)(((uint64_t)hi << 32) | lo);
        }
    };
    for (int64_t w = GLOBAL ? gwave : next(0); w < count; w = next(w)) {
        const int64_t q = GLOBAL ? (int64_t)redo[w] : w;
        const PairDesc pd = pairs[q];
        const uint8_t *a = codes + pd.a_off;
        const uint8_t *b = codes + pd.b_off;
        const int pa[2] = {pd.pa1, pd.pa2}, pb[2] = {pd.pb1, pd.pb2};
        pastis_pair_record rec;
        rec.score = 0;
        rec.beg_a = rec.end_a = rec.beg_b = rec.end_b = -1;
        rec.matches = rec.columns = 0;
        rec.seed_used = -1;
        rec.passed = 0;
        rec.swapped = pd.swapped;
        bool have = false, best_pass = false, overflow = false;
        int cells = 0;
        for (int s = 0; s < 2; ++s) {
            if (pa[s] < 0) continue;
            const SeedAln t =
                align_seed<GLOBAL>(a, pd.la, b, pd.lb, pa[s], pb[s], k, sbl, sbl4, minc, o, e, X, R, rings, lane);
            overflow |= t.overflow;
            cells += t.cells;
            const bool pass = passes(t, pd.la, id_pct, cov_pct);
            if (!have || (pass && !best_pass) || (pass == best_pass && t.score > rec.score)) {
                rec.score = t.score;
                rec.beg_a = t.beg_a;
                rec.end_a = t.end_a;
                rec.beg_b = t.beg_b;
                rec.end_b = t.end_b;
                rec.matches = t.matches;
                rec.columns = t.columns;
                rec.seed_used = s;
                best_pass = pass;
                have = true;
            }
        }
        rec.passed = best_pass ? 1 : 0;
        rec.cells = cells;
        if (!GLOBAL && overflow) {  // a band wider than 64 rows
            if (lane == 0) redo[atomicAdd(n_redo, 1u)] = (uint32_t)q;
            continue;
        }
        my_cells += (unsigned long long)cells;
        if (lane == 0) out[q] = rec;
    }
    if (lane == 0 && my_cells) atomicAdd(&counters[0], my_cells);
}

}  // namespace

int64_t xd_global_waves() { return 64 * kWavesPerBlock; }
size_t xd_ring_bytes_per_wave() { return sizeof(int) * 18 * (size_t)kGlobalCap; }

hipError_t launch_xd(pastis_ctx *ctx, const uint8_t *codes, const PairDesc *pairs, int64_t npairs,
                     const int8_t *blosum, const Scoring &sc, int k, pastis_pair_record *out, uint32_t *redo,
                     uint32_t *n_redo, int *gring, unsigned long long *counters, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    hipError_t e = stage_begin(ctx, kStAlign1, s);
    if (e != hipSuccess) return e;
    // a resident grid (six blocks of four waves per CU) draining the queue
    int64_t blocks = (npairs + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 256 * 6 * 2) blocks = 256 * 6 * 2;
    xd_kernel<false><<<(unsigned)blocks, 256, 0, s>>>(codes, pairs, npairs, blosum, k, sc.gap_open, sc.gap_extend,
                                                       sc.xdrop, sc.id_pct, sc.cov_pct, out, redo, n_redo, gring,
                                                       counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = stage_end(ctx, kStAlign1, s)) != hipSuccess || (e = stage_begin(ctx, kStAlign2, s)) != hipSuccess)
        return e;
    xd_kernel<true><<<(unsigned)(xd_global_waves() / kWavesPerBlock), 256, 0, s>>>(
        codes, pairs, npairs, blosum, k, sc.gap_open, sc.gap_extend, sc.xdrop, sc.id_pct, sc.cov_pct, out, redo,
        n_redo, gring, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return stage_end(ctx, kStAlign2, s);
}

}  // namespace pastis
