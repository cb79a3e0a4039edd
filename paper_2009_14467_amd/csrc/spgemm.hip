// Candidate discovery: the sparse products A A^T and (A S) A^T under the
// count + seed semiring (Sections IV-A and IV-C), the common-k-mer threshold
// (Section VI) and symmetrisation.
//
// Row i of the product visits, for every entry (s, pos_i) of its row (a k-mer
// of A_i, or a substitute of (A S)_i), every posting (j, pos_j) of s, and adds
// one to entry j with seed key (pos_lo << 16 | pos_hi), keeping the two
// smallest keys.  Exact k-mers give a symmetric B, so only j > i is visited.
// Substitutes give a directional count c(i -> j); both directions are made and
// each pair keeps the larger count (lo -> hi on a tie), which equals B when
// m = 0.
//
// One workgroup owns one row.  Entries are expanded in chunks: the posting
// lengths of a chunk are prefix-summed in LDS and every thread takes products
// by binary search, so a long posting list is shared by the whole group.
// Phase 1 counts into an LDS hash whose 32-bit slots pack (j << 14 | count)
// and stages every product's (slot, seed key) in a per-block buffer; entries
// reaching the threshold get a candidate slot; phase 2 replays the stage and
// keeps the two smallest seed keys of candidates only (lock-free: the key
// displaced from the first slot falls to the second).  Rows too large for LDS
// use the same scheme with 64-bit slots in global memory, where phase 2
// expands the row again.
#include <algorithm>

#include "internal.hpp"
#include "kmers.hpp"
#include "prim.hpp"
#include "spgemm.hpp"

namespace pastis {

hipError_t launch_bins(const int8_t *bin_of, int64_t n, int nbins, int *counts, int *starts, int *cursor, int *idx,
                       hipStream_t s);

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kProductTiers = 5;  // LDS tables of 2K, 4K, 8K, 16K and 32K slots
// blocks per launch of each tier: resident blocks per CU (LDS and wave
// limits) times the 256 CUs
constexpr int kTierBlocks[kProductTiers] = {256 * 8, 256 * 5, 256 * 3, 256 * 2, 256};
constexpr int kChunk = 512;
constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t hash32(uint32_t x) { return x * 0x9E3779B1u; }

// A row's entries: exact (A_i: k-mer + position) or substitute ((A S)_i:
// substitute + (distance, position)); a k-mer is named by the header index of
// its posting group.
struct RowView {
    const uint32_t *start32;  // exact: row_start [n+1]
    const uint64_t *start64;  // substitutes: as_start [n+1]
    const uint32_t *len;      // substitutes: as_len [n]
    const uint32_t *ent_s;
    const uint16_t *ent_pos16;  // exact
    const uint32_t *ent_dp;     // substitutes: ((d + 128) << 16) | pos
    int exact;
    const uint32_t *ent_len;    // exact: the posting length of each entry (else read from the header)
    // row block: only pairs whose lower index lies in [blk_lo, blk_hi) are kept
    uint32_t blk_lo, blk_hi;

    // a product (i, j) that names no pair of this block: the diagonal, the
    // lower triangle of the (symmetric) exact product, or a pair whose lower
    // index lies outside the block
    __device__ __forceinline__ bool skip(uint32_t i, uint32_t j) const {
        const uint32_t lo = i < j ? i : j;
        return j == i || (exact && j < i) || lo - blk_lo >= blk_hi - blk_lo;
    }
    // rows whose products can name a pair of the block: its own rows, and
    // with substitutes (both directions are counted) every later row too
    __device__ __forceinline__ bool active(uint32_t i) const { return i >= blk_lo && (!exact || i < blk_hi); }

    __device__ __forceinline__ void bounds(uint32_t i, uint64_t &b, uint64_t &e) const {
        if (exact) {
            b = start32[i];
            e = start32[i + 1];
        } else {
            b = start64[i];
            e = b + len[i];
        }
    }
    __device__ __forceinline__ uint32_t pos(uint64_t x) const {
        return exact ? (uint32_t)ent_pos16[x] : (ent_dp[x] & 0xFFFFu);
    }
};

// Postings of A^T as headed records: an entry names its k-mer's group by
// the index h of its header; rec[h] = (length, distinct k-mer index) and the
// group's (sequence, position) records follow at h + 1.  The header shares a
// line with the first records, so an entry costs one scattered line for its
// length and (for the usual short lists) its products.  Rows of A carry each
// entry's length beside it, so for them the row scan reads no header and the
// product's first scattered access is the records themselves.
struct Postings {
    const uint2 *rec;
};

struct Emit {
    unsigned long long *count;  // device counter (64-bit: it keeps counting past cap without wrapping)
    uint32_t *overflow;
    uint64_t *key;
    uint32_t *cnt, *s1, *s2, *dir;
    uint32_t cap;
    int nbits;  // key = lo << nbits | hi
};

__device__ __forceinline__ void seed_min2(uint32_t *s1, uint32_t *s2, uint32_t key) {
    const uint32_t old = atomicMin(s1, key);
    if (old == kEmpty) return;
    atomicMin(s2, key < old ? old : key);
}

__device__ __forceinline__ uint32_t seed_key(uint32_t i, uint32_t j, uint32_t pi, uint32_t pj) {
    return i < j ? ((pi << 16) | pj) : ((pj << 16) | pi);
}

__device__ __forceinline__ void emit(const Emit &em, uint32_t i, uint32_t j, uint32_t c, uint32_t a, uint32_t b) {
    const unsigned long long slot = atomicAdd(em.count, 1ull);
    if (slot >= em.cap) {
        atomicOr(em.overflow, 1u);
        return;
    }
    const uint32_t lo = i < j ? i : j, hi = i < j ? j : i;
    em.key[slot] = ((uint64_t)lo << em.nbits) | hi;
    em.cnt[slot] = c;
    em.s1[slot] = a;
    em.s2[slot] = b;
    em.dir[slot] = i < j ? 0u : 1u;
}

// Chunk expansion shared by both table kinds: calls f(pos_i, j, pos_j, q)
// for every product of row i, q numbering the row's products from 0 (the
// same numbers in every expansion of the row); returns the product count.
struct ChunkLds {
    uint32_t pref[kChunk + 1];
    uint32_t pbeg[kChunk];
    uint32_t epos[kChunk];
    uint32_t wsum[kThreads / 64];
};

template <typename F>
__device__ __forceinline__ uint32_t expand_row(const RowView &rv, const Postings &P, uint32_t i, ChunkLds &C, F &&f) {
    uint64_t b, e;
    rv.bounds(i, b, e);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t done = 0;
    for (uint64_t c0 = b; c0 < e; c0 += kChunk) {
        const int ce = (int)((e - c0) < (uint64_t)kChunk ? (e - c0) : (uint64_t)kChunk);
        // lengths of this chunk's posting lists, prefix-summed over the block
        uint32_t len0 = 0, len1 = 0;
        const int t0 = threadIdx.x * 2, t1 = t0 + 1;
        if (t0 < ce) {
            const uint32_t h = rv.ent_s[c0 + t0];
            len0 = rv.ent_len ? rv.ent_len[c0 + t0] : P.rec[h].x;
            C.pbeg[t0] = h + 1;
            C.epos[t0] = rv.pos(c0 + t0);
        }
        if (t1 < ce) {
            const uint32_t h = rv.ent_s[c0 + t1];
            len1 = rv.ent_len ? rv.ent_len[c0 + t1] : P.rec[h].x;
            C.pbeg[t1] = h + 1;
            C.epos[t1] = rv.pos(c0 + t1);
        }
        uint32_t v = len0 + len1, inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane == 63) C.wsum[wave] = inc;
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < wave; ++w) add += C.wsum[w];
        const uint32_t excl = inc - v + add;
        if (t0 < ce) C.pref[t0] = excl;
        if (t1 < ce) C.pref[t1] = excl + len0;
        if (threadIdx.x == kThreads - 1) C.pref[ce] = excl + v;
        __syncthreads();
        const uint32_t total = C.pref[ce];
        for (uint32_t p = threadIdx.x; p < total; p += kThreads) {
            // entry x with pref[x] <= p < pref[x + 1]
            int lo = 0, hi = ce;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (C.pref[mid] <= p)
                    lo = mid;
                else
                    hi = mid;
            }
            const uint2 r = P.rec[C.pbeg[lo] + (p - C.pref[lo])];
            f(C.epos[lo], r.x, r.y, done + p);
        }
        done += total;
        __syncthreads();
    }
    return done;
}

// ------------------------------------------------------------ LDS kernel

// CAP slots for rows of at most 3/4 CAP products (so at most that many keys),
// and up to CC candidates, each staged as one word (j << 14 | count).  A
// count that would pass 2^14 - 1 (possible only where a row has more products
// than that) or more than CC candidates send the row to the global path.  A
// row's candidates take consecutive output entries, reserved by one atomic;
// their two smallest seed keys are kept in place in the output arrays.
template <int CAP, int CC>
struct RowLds {
    uint32_t slot[CAP];  // (j << 14) | count, then (j << 14) | (candidate + 1)
    uint32_t cand[CC];   // (j << 14) | count
    ChunkLds chunk;
    uint32_t ncand;
    uint32_t spill;
    uint32_t base;
};

template <int CAP, int CC>
__global__ __launch_bounds__(kThreads) void spgemm_lds_kernel(RowView rv, Postings P, const int *__restrict__ idx,
                                                              const int *__restrict__ starts, int bin, int ck,
                                                              Emit em, uint32_t *__restrict__ spill_rows,
                                                              uint32_t *__restrict__ spill_count,
                                                              uint2 *__restrict__ stage_all) {
    static_assert(CC < (1 << 14), "candidate tags fit 14 bits");
    __shared__ RowLds<CAP, CC> L;
    constexpr uint32_t mask = CAP - 1;
    // this block's stage: (slot, seed key) of each product of the current
    // row, kEmpty for the skipped ones (a row has at most 3/4 CAP products)
    uint2 *stage = stage_all + (size_t)blockIdx.x * (3 * CAP / 4);
    for (int t = threadIdx.x; t < CAP; t += kThreads) L.slot[t] = kEmpty;
    if (threadIdx.x == 0) {
        L.ncand = 0;
        L.spill = 0;
    }
    __syncthreads();
    const int b0 = starts[bin];
    const XcdWalk it = xcd_walk(starts[bin + 1] - b0);
    for (int64_t t = it.first; t < it.end; t += it.step) {
        const uint32_t i = (uint32_t)idx[b0 + t];
        // phase 1: counts, and each product's slot and seed key staged
        const uint32_t total = expand_row(rv, P, i, L.chunk, [&](uint32_t pi, uint32_t j, uint32_t pj, uint32_t q) {
            if (rv.skip(i, j)) {
                stage[q] = make_uint2(kEmpty, 0u);
                return;
            }
            uint32_t h = hash32(j) & mask;
            for (;;) {
                uint32_t v = L.slot[h];
                if (v == kEmpty) {
                    const uint32_t old = atomicCAS(&L.slot[h], kEmpty, (j << 14) | 1u);
                    if (old == kEmpty) break;
                    v = old;
                }
                if ((v >> 14) == j) {
                    // a count of 2^14 - 1 carries into j: the row is redone
                    // with 64-bit slots (the table keeps fewer than CAP keys,
                    // so later probes still end)
                    if ((atomicAdd(&L.slot[h], 1u) & 0x3FFFu) == 0x3FFFu) L.spill = 1;
                    break;
                }
                h = (h + 1) & mask;
            }
            stage[q] = make_uint2(h, seed_key(i, j, pi, pj));
        });
        __syncthreads();
        for (int t = threadIdx.x; t < CAP; t += kThreads) {
            const uint32_t v = L.slot[t];
            if (v == kEmpty) continue;
            const uint32_t c = v & 0x3FFFu, j = v >> 14;
            uint32_t tag = 0;
            if (c >= (uint32_t)ck) {
                const uint32_t q = atomicAdd(&L.ncand, 1u);
                if (q < (uint32_t)CC) {
                    L.cand[q] = v;
                    tag = q + 1;
                } else {
                    L.spill = 1;
                }
            }
            L.slot[t] = (j << 14) | tag;
        }
        __syncthreads();
        if (L.spill) {
            // too many candidates for this table: the global path redoes the row
            if (threadIdx.x == 0) spill_rows[atomicAdd(spill_count, 1u)] = i;
        } else if (L.ncand > 0) {
            const uint32_t nc = L.ncand;
            if (threadIdx.x == 0) {
                const unsigned long long b = atomicAdd(em.count, (unsigned long long)nc);
                if (b + nc > em.cap) {
                    atomicOr(em.overflow, 1u);  // the call is redone with more room
                    L.base = kEmpty;
                } else {
                    L.base = (uint32_t)b;
                }
            }
            __syncthreads();
            const uint32_t base = L.base;
            if (base != kEmpty) {
                for (uint32_t q = threadIdx.x; q < nc; q += kThreads) {
                    const uint32_t v = L.cand[q], j = v >> 14;
                    const uint32_t lo = i < j ? i : j, hi = i < j ? j : i;
                    em.key[base + q] = ((uint64_t)lo << em.nbits) | hi;
                    em.cnt[base + q] = v & 0x3FFFu;
                    em.s1[base + q] = kEmpty;
                    em.s2[base + q] = kEmpty;
                    em.dir[base + q] = i < j ? 0u : 1u;
                }
                __threadfence_block();
                __syncthreads();
                // phase 2: seeds of candidate entries, from the stage (its
                // slots now hold j << 14 | candidate + 1, or 0 for none)
                for (uint32_t q = threadIdx.x; q < total; q += kThreads) {
                    const uint2 r = stage[q];
                    if (r.x == kEmpty) continue;
                    const uint32_t tag = L.slot[r.x] & 0x3FFFu;
                    if (tag) seed_min2(&em.s1[base + tag - 1], &em.s2[base + tag - 1], r.y);
                }
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < CAP; t += kThreads) L.slot[t] = kEmpty;
        if (threadIdx.x == 0) {
            L.ncand = 0;
            L.spill = 0;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ global kernel

// Rows listed in rows[0..*nrows) with a per-block table of cap 64-bit slots
// (j << 32 | count, later j << 32 | candidate + 1) and cap / 2 candidates.
// Each row uses the first next_pow2(2 * work) slots of its block's table (at
// least 4096, at most cap), so clearing and scanning cost follow the row.
__global__ __launch_bounds__(kThreads) void spgemm_global_kernel(RowView rv, Postings P, const uint32_t *__restrict__ rows,
                                                                 const uint32_t *__restrict__ nrows_p,
                                                                 const uint64_t *__restrict__ work, int ck, Emit em,
                                                                 unsigned long long *__restrict__ tables, uint32_t cap,
                                                                 uint32_t *__restrict__ cand) {
    __shared__ ChunkLds C;
    __shared__ uint32_t ncand;
    unsigned long long *slot = tables + (size_t)blockIdx.x * cap;
    uint32_t *cj = cand + (size_t)blockIdx.x * 2 * cap;  // cap/2 entries x 4 arrays
    uint32_t *cc = cj + cap / 2, *c1 = cc + cap / 2, *c2 = c1 + cap / 2;
    const unsigned long long empty = ~0ull;
    for (uint32_t t = threadIdx.x; t < cap; t += kThreads) slot[t] = empty;
    if (threadIdx.x == 0) ncand = 0;
    __threadfence_block();
    __syncthreads();
    const uint32_t nrows = *nrows_p;
    for (uint32_t w = blockIdx.x; w < nrows; w += gridDim.x) {
        const uint32_t i = rows[w];
        uint64_t want = 2 * work[i];
        uint32_t rcap = 4096;
        while (rcap < want && rcap < cap) rcap <<= 1;
        const uint32_t mask = rcap - 1;
        expand_row(rv, P, i, C, [&](uint32_t, uint32_t j, uint32_t, uint32_t) {
            if (rv.skip(i, j)) return;
            uint32_t h = hash32(j) & mask;
            for (;;) {
                unsigned long long v = slot[h];
                if (v == empty) {
                    const unsigned long long old = atomicCAS(&slot[h], empty, ((unsigned long long)j << 32) | 1ull);
                    if (old == empty) return;
                    v = old;
                }
                if ((uint32_t)(v >> 32) == j) {
                    atomicAdd(&slot[h], 1ull);
                    return;
                }
                h = (h + 1) & mask;
            }
        });
        __threadfence_block();
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < rcap; t += kThreads) {
            const unsigned long long v = slot[t];
            if (v == empty) continue;
            const uint32_t c = (uint32_t)v, j = (uint32_t)(v >> 32);
            uint32_t tag = 0;
            if (c >= (uint32_t)ck) {
                const uint32_t q = atomicAdd(&ncand, 1u);
                cj[q] = j;
                cc[q] = c;
                c1[q] = kEmpty;
                c2[q] = kEmpty;
                tag = q + 1;
            }
            slot[t] = ((unsigned long long)j << 32) | tag;
        }
        __threadfence_block();
        __syncthreads();
        if (ncand > 0) {
            expand_row(rv, P, i, C, [&](uint32_t pi, uint32_t j, uint32_t pj, uint32_t) {
                if (rv.skip(i, j)) return;
                uint32_t h = hash32(j) & mask;
                unsigned long long v = slot[h];
                while ((uint32_t)(v >> 32) != j) {
                    h = (h + 1) & mask;
                    v = slot[h];
                }
                const uint32_t tag = (uint32_t)v;
                if (tag) seed_min2(&c1[tag - 1], &c2[tag - 1], seed_key(i, j, pi, pj));
            });
            __threadfence_block();
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < ncand; q += kThreads) emit(em, i, cj[q], cc[q], c1[q], c2[q]);
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < rcap; t += kThreads) slot[t] = empty;
        if (threadIdx.x == 0) ncand = 0;
        __threadfence_block();
        __syncthreads();
    }
}

// ------------------------------------------------------------ A S rows

constexpr int kAsCap = 8192;

struct AsIn {
    const uint32_t *row_start;  // A rows
    const uint32_t *row_u;
    const uint16_t *row_pos;
    const uint32_t *s_u;  // S rows, m + 1 slots each
    const int8_t *s_d;
    const uint32_t *s_cnt;
    int W;  // m + 1
};

// (A S)_{i,s}: the closest k-mer of row i reaching s, then the smaller
// position (Section IV-C), reduced with atomicMin on ((d + 128) << 16 | pos).
template <typename Slots>
__device__ __forceinline__ void as_reduce(const AsIn &in, uint32_t i, Slots &tab, uint32_t mask) {
    const uint32_t b = in.row_start[i], e = in.row_start[i + 1];
    const uint32_t total = (e - b) * (uint32_t)in.W;
    for (uint32_t p = threadIdx.x; p < total; p += kThreads) {
        const uint32_t x = b + p / in.W, q = p % in.W;
        const uint32_t u = in.row_u[x];
        if (q >= in.s_cnt[u]) continue;
        const uint32_t s = in.s_u[(size_t)u * in.W + q];
        const uint32_t dp = ((uint32_t)(in.s_d[(size_t)u * in.W + q] + 128) << 16) | in.row_pos[x];
        uint32_t h = hash32(s) & mask;
        for (;;) {
            uint32_t k = tab.key(h);
            if (k == kEmpty) {
                const uint32_t old = tab.cas(h, s);
                if (old == kEmpty || old == s) {
                    tab.vmin(h, dp);
                    break;
                }
                k = old;
            }
            if (k == s) {
                tab.vmin(h, dp);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

struct LdsSlots {
    uint32_t *k, *v;
    __device__ uint32_t key(uint32_t h) { return k[h]; }
    __device__ uint32_t cas(uint32_t h, uint32_t s) { return atomicCAS(&k[h], kEmpty, s); }
    __device__ void vmin(uint32_t h, uint32_t dp) { atomicMin(&v[h], dp); }
};

// CAP slots (8 bytes each) for rows of at most 3/4 CAP entries
template <int CAP>
__global__ __launch_bounds__(kThreads) void as_lds_kernel(AsIn in, const int *__restrict__ idx,
                                                          const int *__restrict__ starts, int bin,
                                                          const uint64_t *__restrict__ as_start,
                                                          uint32_t *__restrict__ as_len, uint32_t *__restrict__ as_s,
                                                          uint32_t *__restrict__ as_dp) {
    __shared__ uint32_t K[CAP], V[CAP];
    __shared__ uint32_t n_out;
    LdsSlots tab{K, V};
    for (int t = threadIdx.x; t < CAP; t += kThreads) {
        K[t] = kEmpty;
        V[t] = kEmpty;
    }
    if (threadIdx.x == 0) n_out = 0;
    __syncthreads();
    const int b0 = starts[bin];
    const XcdWalk it = xcd_walk(starts[bin + 1] - b0);
    for (int64_t t = it.first; t < it.end; t += it.step) {
        const uint32_t i = (uint32_t)idx[b0 + t];
        as_reduce(in, i, tab, CAP - 1);
        __syncthreads();
        const uint64_t base = as_start[i];
        for (int t = threadIdx.x; t < CAP; t += kThreads) {
            if (K[t] == kEmpty) continue;
            const uint32_t q = atomicAdd(&n_out, 1u);
            as_s[base + q] = K[t];
            as_dp[base + q] = V[t];
            K[t] = kEmpty;
            V[t] = kEmpty;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            as_len[i] = n_out;
            n_out = 0;
        }
        __syncthreads();
    }
}

struct GlobalSlots {
    uint32_t *k, *v;
    __device__ uint32_t key(uint32_t h) { return __builtin_nontemporal_load(&k[h]); }
    __device__ uint32_t cas(uint32_t h, uint32_t s) { return atomicCAS(&k[h], kEmpty, s); }
    __device__ void vmin(uint32_t h, uint32_t dp) { atomicMin(&v[h], dp); }
};

__global__ __launch_bounds__(kThreads) void as_global_kernel(AsIn in, const int *__restrict__ idx,
                                                             const int *__restrict__ starts, int bin,
                                                             const uint64_t *__restrict__ as_start,
                                                             uint32_t *__restrict__ as_len,
                                                             uint32_t *__restrict__ as_s, uint32_t *__restrict__ as_dp,
                                                             uint32_t *__restrict__ tables, uint32_t cap) {
    __shared__ uint32_t n_out;
    uint32_t *K = tables + (size_t)blockIdx.x * 2 * cap, *V = K + cap;
    GlobalSlots tab{K, V};
    for (uint32_t t = threadIdx.x; t < cap; t += kThreads) {
        K[t] = kEmpty;
        V[t] = kEmpty;
    }
    if (threadIdx.x == 0) n_out = 0;
    __threadfence_block();
    __syncthreads();
    const int end = starts[bin + 1];
    for (int w = starts[bin] + blockIdx.x; w < end; w += gridDim.x) {
        const uint32_t i = (uint32_t)idx[w];
        as_reduce(in, i, tab, cap - 1);
        __threadfence_block();
        __syncthreads();
        const uint64_t base = as_start[i];
        for (uint32_t t = threadIdx.x; t < cap; t += kThreads) {
            if (K[t] == kEmpty) continue;
            const uint32_t q = atomicAdd(&n_out, 1u);
            as_s[base + q] = K[t];
            as_dp[base + q] = V[t];
            K[t] = kEmpty;
            V[t] = kEmpty;
        }
        __threadfence_block();
        __syncthreads();
        if (threadIdx.x == 0) {
            as_len[i] = n_out;
            n_out = 0;
        }
        __syncthreads();
    }
}

// upper bound of (A S)_i entries = sum of present S-row sizes of i's k-mers;
// every row's length starts at 0 (rows without k-mers are never filled)
// (one wave per row: lanes stride the row's k-mers, then a wave sum)
__global__ __launch_bounds__(256) void as_ub_kernel(AsIn in, int64_t n, uint32_t *__restrict__ ub,
                                                    uint32_t *__restrict__ as_len, int8_t *__restrict__ bin_of,
                                                    unsigned long long *__restrict__ max_ub) {
    const int lane = threadIdx.x & 63;
    const XcdWalk it = xcd_walk(n, blockDim.x / 64, threadIdx.x / 64);
    for (int64_t i = it.first; i < it.end; i += it.step) {
        uint32_t s = 0;
        for (uint32_t x = in.row_start[i] + lane; x < in.row_start[i + 1]; x += 64) s += in.s_cnt[in.row_u[x]];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += (uint32_t)__shfl_xor((int)s, off, 64);
        if (lane != 0) continue;
        ub[i] = s;
        as_len[i] = 0;
        // bins: 0 = 8192 LDS slots, 1 = 16384 LDS slots, 2 = a table in global memory
        const int8_t bin = s * 4u <= (uint32_t)kAsCap * 3u ? 0 : s * 4u <= (uint32_t)kAsCap * 6u ? 1 : 2;
        bin_of[i] = s == 0 ? (int8_t)-1 : bin;
        if (bin == 2) atomicMax(max_ub, (unsigned long long)s);
    }
}

// headed records: posting x of group u goes to x + u + 1; the group's first
// posting also writes the header (length, u) just before it
__global__ void posting_records_kernel(const uint32_t *__restrict__ seq, const uint16_t *__restrict__ pos,
                                       const uint32_t *__restrict__ post_u, const uint32_t *__restrict__ uk_start,
                                       int64_t n, uint2 *__restrict__ rec) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = post_u[x];
        const uint32_t b = uk_start[u];
        rec[x + u + 1] = make_uint2(seq[x], (uint32_t)pos[x]);
        if ((uint32_t)x == b) rec[x + u] = make_uint2(uk_start[u + 1] - b, u);
    }
}

// products of row i (postings visited), and the row's bin; one wave per row
// (lanes stride the row's entries, then a wave sum)
__global__ __launch_bounds__(256) void work_kernel(RowView rv, Postings P, int64_t n, int n_big_ok,
                                                   uint64_t *__restrict__ work, int8_t *__restrict__ bin_of,
                                                   unsigned long long *__restrict__ max_big,
                                                   uint32_t *__restrict__ big_rows, uint32_t *__restrict__ n_big,
                                                   unsigned long long *__restrict__ products) {
    const int lane = threadIdx.x & 63;
    const XcdWalk it = xcd_walk(n, blockDim.x / 64, threadIdx.x / 64);
    // the products of this wave's rows, added to *products once per block
    // (one atomic per row would serialise on the one address)
    __shared__ unsigned long long wave_products[4];
    unsigned long long mine = 0;
    for (int64_t i = it.first; i < it.end; i += it.step) {
        uint64_t b, e;
        rv.bounds((uint32_t)i, b, e);
        if (!rv.active((uint32_t)i)) e = b;  // no pair of the block: no products, no bin
        uint64_t w = 0;
        if (rv.ent_len) {
            for (uint64_t x = b + lane; x < e; x += 64) w += rv.ent_len[x];
        } else {
            for (uint64_t x = b + lane; x < e; x += 64) w += P.rec[rv.ent_s[x]].x;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)w, off, 64);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(w >> 32), off, 64);
            w += ((uint64_t)hi << 32) | lo;
        }
        if (lane != 0) continue;
        work[i] = w;
        mine += w;
        // tables of 2^(11 + bin) slots hold rows of up to 3/4 of that many products
        int8_t bin = -1;
        if (w > 0 && n_big_ok)
            for (int b = 0; b < kProductTiers; ++b)
                if (w <= (3ull << (9 + b))) {
                    bin = (int8_t)b;
                    break;
                }
        bin_of[i] = bin;
        if (w > 0 && bin < 0) {
            big_rows[atomicAdd(n_big, 1u)] = (uint32_t)i;
            atomicMax(max_big, (unsigned long long)w);
        }
    }
    if (lane == 0) wave_products[threadIdx.x / 64] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) t += wave_products[k];
        if (t) atomicAdd(products, t);
    }
}

// ------------------------------------------------------------ symmetrise

// entries sorted by key; each (lo, hi) keeps the larger direction (lo -> hi on
// a tie); out_flag marks the kept representative
__global__ void merge_flag_kernel(const uint64_t *__restrict__ skey, const uint32_t *__restrict__ perm,
                                  const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ dir,
                                  const uint32_t *__restrict__ n_p, uint8_t *__restrict__ flag,
                                  uint32_t *__restrict__ pick) {
    const uint32_t n = *n_p;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        if (x > 0 && skey[x - 1] == skey[x]) {
            flag[x] = 0;
            continue;
        }
        flag[x] = 1;
        uint32_t best = perm[x];
        if (x + 1 < n && skey[x + 1] == skey[x]) {
            const uint32_t o = perm[x + 1];
            const bool take_o = cnt[o] > cnt[best] || (cnt[o] == cnt[best] && dir[o] < dir[best]);
            if (take_o) best = o;
        }
        pick[x] = best;
    }
}

__global__ void merge_write_kernel(const uint64_t *__restrict__ skey, const uint8_t *__restrict__ flag,
                                   const uint32_t *__restrict__ pick, const uint32_t *__restrict__ opos,
                                   const uint32_t *__restrict__ n_p, const uint32_t *__restrict__ cnt,
                                   const uint32_t *__restrict__ s1, const uint32_t *__restrict__ s2, int nbits,
                                   Candidates out) {
    const uint32_t n = *n_p;
    const uint64_t hmask = (1ull << nbits) - 1ull;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        if (!flag[x]) continue;
        const uint32_t q = opos[x], b = pick[x];
        out.lo[q] = (uint32_t)(skey[x] >> nbits);
        out.hi[q] = (uint32_t)(skey[x] & hmask);
        out.count[q] = cnt[b];
        out.seed1[q] = s1[b];
        out.seed2[q] = s2[b];
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t spgemm_stage_entries() {
    size_t m = 0;
    for (int b = 0; b < kProductTiers; ++b) m = std::max(m, (size_t)kTierBlocks[b] * (3u << (9 + b)));
    return m;
}

int key_bits(int64_t n) {
    int b = 1;
    while (b < 32 && (1ll << b) < n) ++b;
    return b;
}

hipError_t as_stage(const AsArgs &a, hipStream_t s) {
    AsIn in{a.kt->row_start, a.kt->row_u, a.kt->row_pos, a.s_u, a.s_d, a.s_cnt, a.W};
    hipError_t e;
    if ((e = fill<unsigned long long>(a.max_ub, 1, 0ull, s)) != hipSuccess) return e;
    as_ub_kernel<<<grid_for(64 * a.n), 256, 0, s>>>(in, a.n, a.ub, a.as_len, a.bin_of, a.max_ub);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = exclusive_scan<uint32_t, uint64_t>(a.ub, a.n, a.as_start, a.as_start + a.n, a.scan_temp, s);
    if (e != hipSuccess) return e;
    return launch_bins(a.bin_of, a.n, 3, a.bins.counts, a.bins.starts, a.bins.cursor, a.bins.idx, s);
}

hipError_t as_run(const AsArgs &a, uint32_t gcap, hipStream_t s) {
    AsIn in{a.kt->row_start, a.kt->row_u, a.kt->row_pos, a.s_u, a.s_d, a.s_cnt, a.W};
    // LDS per block: 64 KB (two blocks per CU), 128 KB (one)
    as_lds_kernel<kAsCap><<<512, kThreads, 0, s>>>(in, a.bins.idx, a.bins.starts, 0, a.as_start, a.as_len, a.as_s,
                                                   a.as_dp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    as_lds_kernel<2 * kAsCap><<<256, kThreads, 0, s>>>(in, a.bins.idx, a.bins.starts, 1, a.as_start, a.as_len,
                                                       a.as_s, a.as_dp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (gcap > 0) {
        as_global_kernel<<<a.global_blocks, kThreads, 0, s>>>(in, a.bins.idx, a.bins.starts, 2, a.as_start, a.as_len,
                                                               a.as_s, a.as_dp, a.gtables, gcap);
        e = hipGetLastError();
    }
    return e;
}

hipError_t spgemm_plan(const SpgemmArgs &a, hipStream_t s) {
    RowView rv{a.row_start32, a.row_start64, a.row_len, a.ent_s, a.ent_pos16, a.ent_dp, a.exact, a.ent_len,
               a.blk_lo, a.blk_hi};
    Postings P{a.post_rec};
    hipError_t e;
    if ((e = fill<unsigned long long>(a.max_big, 1, 0ull, s)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(a.n_big, 2, 0u, s)) != hipSuccess) return e;
    if ((e = fill<unsigned long long>(a.products, 1, 0ull, s)) != hipSuccess) return e;
    posting_records_kernel<<<grid_for(a.nnz), 256, 0, s>>>(a.kt->post_seq, a.kt->post_pos, a.kt->post_u,
                                                            a.kt->uk_start, a.nnz, a.post_rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    work_kernel<<<grid_for(64 * a.n), 256, 0, s>>>(rv, P, a.n, a.n < (1ll << 18) ? 1 : 0, a.work, a.bin_of,
                                                   a.max_big, a.big_rows, a.n_big, a.products);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_bins(a.bin_of, a.n, kProductTiers, a.bins.counts, a.bins.starts, a.bins.cursor, a.bins.idx, s);
}

hipError_t spgemm_run(const SpgemmArgs &a, uint32_t gcap, hipStream_t s) {
    RowView rv{a.row_start32, a.row_start64, a.row_len, a.ent_s, a.ent_pos16, a.ent_dp, a.exact, a.ent_len,
               a.blk_lo, a.blk_hi};
    Postings P{a.post_rec};
    Emit em{a.d_count, a.d_overflow, a.d_key, a.d_cnt, a.d_s1, a.d_s2, a.d_dir, a.cap, a.nbits};
    hipError_t e;
    if ((e = fill<unsigned long long>(a.d_count, 1, 0ull, s)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(a.d_overflow, 1, 0u, s)) != hipSuccess) return e;
    // spilled rows (too many candidates for LDS) join the big-row list.
    // LDS per block: 18 KB (eight blocks per CU, the wave limit), 30 KB
    // (five), 51 KB (three), 78 KB (two), 150 KB (one).  The kernel is bound
    // by the latency of its dependent loads (entry, then posting header or
    // records),
    // so the small tables, where most rows of short sequences land, pay off
    // through the blocks they keep resident.
    spgemm_lds_kernel<2048, 1024><<<kTierBlocks[0], kThreads, 0, s>>>(rv, P, a.bins.idx, a.bins.starts, 0, a.ck,
                                                                      em, a.big_rows, a.n_big, a.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    spgemm_lds_kernel<4096, 2048><<<kTierBlocks[1], kThreads, 0, s>>>(rv, P, a.bins.idx, a.bins.starts, 1, a.ck,
                                                                      em, a.big_rows, a.n_big, a.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    spgemm_lds_kernel<8192, 3072><<<kTierBlocks[2], kThreads, 0, s>>>(rv, P, a.bins.idx, a.bins.starts, 2, a.ck,
                                                                      em, a.big_rows, a.n_big, a.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    spgemm_lds_kernel<16384, 2048><<<kTierBlocks[3], kThreads, 0, s>>>(rv, P, a.bins.idx, a.bins.starts, 3, a.ck,
                                                                       em, a.big_rows, a.n_big, a.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    spgemm_lds_kernel<32768, 4096><<<kTierBlocks[4], kThreads, 0, s>>>(rv, P, a.bins.idx, a.bins.starts, 4, a.ck,
                                                                       em, a.big_rows, a.n_big, a.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (gcap > 0) {
        spgemm_global_kernel<<<a.global_blocks, kThreads, 0, s>>>(rv, P, a.big_rows, a.n_big, a.work, a.ck, em,
                                                                   a.gtables, gcap, a.gcand);
        e = hipGetLastError();
    }
    return e;
}

hipError_t symmetrise(const SymArgs &a, hipStream_t s) {
    hipError_t e;
    bool alt = false;
    if ((e = iota(a.perm, a.n_dir, s)) != hipSuccess) return e;
    if ((e = radix_sort(a.key, a.perm, a.key_alt, a.perm_alt, a.n_dir, 2 * a.nbits, a.sort_temp, s, &alt)) !=
        hipSuccess)
        return e;
    const uint64_t *sk = alt ? a.key_alt : a.key;
    const uint32_t *pm = alt ? a.perm_alt : a.perm;
    merge_flag_kernel<<<grid_for(a.n_dir), 256, 0, s>>>(sk, pm, a.cnt, a.dir, a.d_ndir, a.flag, a.pick);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = exclusive_scan<uint8_t, uint32_t>(a.flag, a.n_dir, a.opos, a.d_ncand, a.sort_temp, s)) != hipSuccess)
        return e;
    merge_write_kernel<<<grid_for(a.n_dir), 256, 0, s>>>(sk, a.flag, a.pick, a.opos, a.d_ndir, a.cnt, a.s1, a.s2,
                                                          a.nbits, a.out);
    return hipGetLastError();
}

}  // namespace pastis
