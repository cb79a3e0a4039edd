// k-mer extraction and the two views of the sequences-by-k-mers matrix A.
//
// A k-mer's id is sum_t code[t] * 24^(k-1-t) over residue codes 0..23
// (Section V-B); A_ij holds the start position of k-mer j in sequence i
// (Section IV-A), the first one when the k-mer repeats inside the sequence.
//
// Windows are emitted in (sequence, position) order and sorted stably by id,
// so the first entry of every (id, sequence) run is the first occurrence.
// Outputs (device, sized by the residue count so no host round trip is needed
// before the next stage):
//   postings (A^T): post_seq / post_pos, grouped by distinct k-mer, sequences
//                   ascending inside a group; uk_id / uk_start index the groups;
//   rows (A):       row_start[n+1], row_u (distinct k-mer index), row_pos,
//                   a row's entries by position (the kept windows in window
//                   order, each window carrying its distinct k-mer back from
//                   the sorted order);
//   kmap:           dense map id -> head of the distinct k-mer's posting group
//                   (uk_start[u] + u) or -1 (24^k entries), for k <=
//                   kDenseMapMaxK only;
//   row_h (if set): per row entry, the head of its k-mer's posting group;
//   row_len (if set with row_h): per row entry, the length of that group.
// Ids are 64-bit (24^8 < 2^37); a window that runs past its sequence gets
// the key 24^k, which sorts after every id.
#include "internal.hpp"
#include "kmers.hpp"
#include "prim.hpp"

namespace pastis {
namespace {

__device__ __forceinline__ int64_t seq_of(const int64_t *__restrict__ offsets, int64_t n, int64_t g) {
    // largest i with offsets[i] <= g (offsets non-decreasing, offsets[0] = 0)
    int64_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (offsets[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ void window_keys_kernel(const uint8_t *__restrict__ codes, const int64_t *__restrict__ offsets, int64_t n,
                                   int64_t n_res, int k, uint64_t invalid, uint64_t *__restrict__ keys,
                                   uint32_t *__restrict__ vals, uint32_t *__restrict__ gseq) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_res;
         g += (int64_t)gridDim.x * blockDim.x) {
        // skip empty sequences: the owner of residue g is the last i with offsets[i] <= g
        const int64_t i = seq_of(offsets, n, g);
        const int64_t end = offsets[i + 1];
        uint64_t key = invalid;
        if (g + k <= end) {
            uint64_t id = 0;
            for (int t = 0; t < k; ++t) id = id * 24u + codes[g + t];
            key = id;
        }
        keys[g] = key;
        vals[g] = (uint32_t)g;
        gseq[g] = (uint32_t)i;
    }
}

// For sorted position x: owning sequence, and whether x starts a new k-mer
// group or a new (k-mer, sequence) run.
__global__ void mark_kernel(const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                            const uint32_t *__restrict__ gseq, int64_t m, uint64_t invalid,
                            uint32_t *__restrict__ sseq, uint8_t *__restrict__ keep, uint8_t *__restrict__ newk) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = skeys[x];
        if (key == invalid) {
            keep[x] = 0;
            newk[x] = 0;
            sseq[x] = 0xFFFFFFFFu;
            continue;
        }
        const uint32_t i = gseq[svals[x]];
        sseq[x] = i;
        bool nk = (x == 0) || skeys[x - 1] != key;
        bool first = nk;
        if (!nk) first = gseq[svals[x - 1]] != i;  // the neighbouring lane's line
        keep[x] = first ? 1 : 0;
        newk[x] = nk ? 1 : 0;
    }
}

// gent[g]: the distinct k-mer index of window g when it is kept (the first
// occurrence of its k-mer in its sequence), else kNone
constexpr uint32_t kNone = 0xFFFFFFFFu;

__global__ void postings_kernel(const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                                const uint32_t *__restrict__ sseq, const int64_t *__restrict__ offsets, int64_t m,
                                const uint8_t *__restrict__ keep, const uint8_t *__restrict__ newk,
                                const uint32_t *__restrict__ kpos, const uint32_t *__restrict__ upos,
                                uint32_t *__restrict__ post_seq, uint16_t *__restrict__ post_pos,
                                uint32_t *__restrict__ post_u, uint64_t *__restrict__ uk_id,
                                uint32_t *__restrict__ uk_start, uint32_t *__restrict__ gent) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[x]) {
            gent[svals[x]] = kNone;
            continue;
        }
        const uint32_t p = kpos[x];
        const uint32_t i = sseq[x];
        const uint32_t u = upos[x] + newk[x] - 1u;
        post_seq[p] = i;
        post_pos[p] = (uint16_t)((int64_t)svals[x] - offsets[i]);
        post_u[p] = u;
        if (newk[x]) {
            uk_id[u] = skeys[x];
            uk_start[u] = p;
        }
        gent[svals[x]] = u;
    }
}

__global__ void kept_flags_kernel(const uint32_t *__restrict__ gent, int64_t m, uint8_t *__restrict__ flag) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m; g += (int64_t)gridDim.x * blockDim.x)
        flag[g] = gent[g] != kNone ? 1 : 0;
}

// row_start[i] = kept windows before sequence i (gslot: the exclusive scan of
// the kept flags in window order, gslot[m] = their total); uk_start[nu] = nnz
__global__ void close_kernel(const uint32_t *__restrict__ nnz, const uint32_t *__restrict__ nu,
                             uint32_t *__restrict__ uk_start, const uint32_t *__restrict__ gslot,
                             const int64_t *__restrict__ offsets, int64_t n, int64_t m,
                             uint32_t *__restrict__ row_start) {
    if (blockIdx.x == 0 && threadIdx.x == 0) uk_start[*nu] = *nnz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = i < n ? offsets[i] : m;
        row_start[i] = gslot[g < m ? g : m];
    }
}

// A's rows in window order: a row's entries are its kept windows by position
__global__ void rows_kernel(const uint32_t *__restrict__ gent, const uint32_t *__restrict__ gslot,
                            const uint32_t *__restrict__ gseq, const int64_t *__restrict__ offsets, int64_t m,
                            const uint32_t *__restrict__ uk_start, uint32_t *__restrict__ row_u,
                            uint16_t *__restrict__ row_pos, uint32_t *__restrict__ row_h,
                            uint32_t *__restrict__ row_len) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m; g += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = gent[g];
        if (u == kNone) continue;
        const uint32_t slot = gslot[g];
        row_u[slot] = u;
        row_pos[slot] = (uint16_t)(g - offsets[gseq[g]]);
        if (row_h) {
            const uint32_t b = uk_start[u];
            row_h[slot] = b + u;
            if (row_len) row_len[slot] = uk_start[u + 1] - b;
        }
    }
}

__global__ void kmap_kernel(const uint64_t *__restrict__ uk_id, const uint32_t *__restrict__ uk_start,
                            const uint32_t *__restrict__ nu_p, int32_t *__restrict__ kmap) {
    const uint32_t nu = *nu_p;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += gridDim.x * blockDim.x)
        kmap[uk_id[u]] = (int32_t)(uk_start[u] + u);
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t kmers_temp_bytes(int64_t n_res, int64_t n) {
    const int64_t m = n_res > 0 ? n_res : 1;
    size_t b = 0;
    b += 2 * sizeof(uint64_t) * m + 2 * sizeof(uint32_t) * m;  // keys, vals, ping-pong
    b += sizeof(uint32_t) * m * 5 + 2 * m;                    // sseq, kpos, upos, gseq, gent, keep, newk
    size_t t = radix_temp_bytes(m);
    size_t t2 = scan_temp_bytes(m > n + 1 ? m : n + 1);
    b += (t > t2 ? t : t2);
    return b + 4096;
}

int64_t kmap_entries(int k) {
    int64_t e = 1;
    for (int t = 0; t < k; ++t) e *= 24;
    return e;
}

hipError_t build_kmers(const uint8_t *codes, const int64_t *offsets, int64_t n, int64_t n_res, int k, bool want_kmap,
                       KmerTables &kt, void *temp, hipStream_t s) {
    hipError_t e;
    const int64_t m = n_res;
    const uint64_t invalid = (uint64_t)kmap_entries(k);  // one past the largest id
    int bits = 8;
    while (bits < 64 && (invalid >> bits) != 0) ++bits;
    char *tp = (char *)temp;
    auto take = [&](size_t bytes) {
        void *p = tp;
        tp += (bytes + 255) & ~(size_t)255;
        return p;
    };
    uint64_t *keys = (uint64_t *)take(sizeof(uint64_t) * (m + 1));
    uint64_t *keys2 = (uint64_t *)take(sizeof(uint64_t) * (m + 1));
    uint32_t *vals = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *vals2 = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *sseq = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *kpos = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *upos = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *gseq = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint32_t *gent = (uint32_t *)take(sizeof(uint32_t) * (m + 1));
    uint8_t *keep = (uint8_t *)take(m + 1);
    uint8_t *newk = (uint8_t *)take(m + 1);
    void *stemp = take(0);
    // after the postings, keep holds the kept flags in window order and kpos
    // their scan
    uint8_t *gflag = keep;
    uint32_t *gslot = kpos;

    if ((e = fill<uint32_t>(kt.counts, 4, 0u, s)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(gslot, 1, 0u, s)) != hipSuccess) return e;  // m = 0: no rows
    if (m > 0) {
        window_keys_kernel<<<grid_for(m), 256, 0, s>>>(codes, offsets, n, m, k, invalid, keys, vals, gseq);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        bool alt = false;
        if ((e = radix_sort(keys, vals, keys2, vals2, m, bits, stemp, s, &alt)) != hipSuccess) return e;
        uint64_t *sk = alt ? keys2 : keys;
        uint32_t *sv = alt ? vals2 : vals;
        mark_kernel<<<grid_for(m), 256, 0, s>>>(sk, sv, gseq, m, invalid, sseq, keep, newk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan<uint8_t, uint32_t>(keep, m, kpos, kt.counts + 0, stemp, s)) != hipSuccess) return e;
        if ((e = exclusive_scan<uint8_t, uint32_t>(newk, m, upos, kt.counts + 1, stemp, s)) != hipSuccess) return e;
        postings_kernel<<<grid_for(m), 256, 0, s>>>(sk, sv, sseq, offsets, m, keep, newk, kpos, upos, kt.post_seq,
                                                    kt.post_pos, kt.post_u, kt.uk_id, kt.uk_start, gent);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kept_flags_kernel<<<grid_for(m), 256, 0, s>>>(gent, m, gflag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan<uint8_t, uint32_t>(gflag, m, gslot, gslot + m, stemp, s)) != hipSuccess) return e;
    }
    close_kernel<<<grid_for(n + 1), 256, 0, s>>>(kt.counts + 0, kt.counts + 1, kt.uk_start, gslot, offsets, n, m,
                                                  kt.row_start);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (m > 0) {
        rows_kernel<<<grid_for(m), 256, 0, s>>>(gent, gslot, gseq, offsets, m, kt.uk_start, kt.row_u, kt.row_pos,
                                                kt.row_h, kt.row_len);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (want_kmap && k <= kDenseMapMaxK) {
        if ((e = fill<int>(kt.kmap, kmap_entries(k), -1, s)) != hipSuccess) return e;
        if (m > 0) {
            kmap_kernel<<<grid_for(m), 256, 0, s>>>(kt.uk_id, kt.uk_start, kt.counts + 1, kt.kmap);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace pastis
