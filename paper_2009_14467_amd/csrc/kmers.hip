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
//   rows (A):       row_start[n+1], row_u (distinct k-mer index), row_pos;
//   kmap:           dense map id -> head of the distinct k-mer's posting group
//                   (uk_start[u] + u) or -1 (24^k entries), for k <=
//                   kDenseMapMaxK only;
//   row_h (if set): per row entry, the head of its k-mer's posting group.
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
                                   uint32_t *__restrict__ vals) {
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
    }
}

// For sorted position x: owning sequence, and whether x starts a new k-mer
// group or a new (k-mer, sequence) run.
__global__ void mark_kernel(const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                            const int64_t *__restrict__ offsets, int64_t n, int64_t m, uint64_t invalid,
                            uint32_t *__restrict__ sseq, uint8_t *__restrict__ keep, uint8_t *__restrict__ newk) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = skeys[x];
        if (key == invalid) {
            keep[x] = 0;
            newk[x] = 0;
            sseq[x] = 0xFFFFFFFFu;
            continue;
        }
        const uint32_t i = (uint32_t)seq_of(offsets, n, (int64_t)svals[x]);
        sseq[x] = i;
        bool nk = (x == 0) || skeys[x - 1] != key;
        bool first = nk;
        if (!nk) {
            const uint32_t ip = (uint32_t)seq_of(offsets, n, (int64_t)svals[x - 1]);
            first = ip != i;
        }
        keep[x] = first ? 1 : 0;
        newk[x] = nk ? 1 : 0;
    }
}

__global__ void postings_kernel(const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                                const uint32_t *__restrict__ sseq, const int64_t *__restrict__ offsets, int64_t m,
                                const uint8_t *__restrict__ keep, const uint8_t *__restrict__ newk,
                                const uint32_t *__restrict__ kpos, const uint32_t *__restrict__ upos,
                                uint32_t *__restrict__ post_seq, uint16_t *__restrict__ post_pos,
                                uint32_t *__restrict__ post_u, uint64_t *__restrict__ uk_id,
                                uint32_t *__restrict__ uk_start, uint32_t *__restrict__ row_cnt) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[x]) continue;
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
        atomicAdd(&row_cnt[i], 1u);
    }
}

__global__ void close_kernel(const uint32_t *__restrict__ nnz, const uint32_t *__restrict__ nu,
                             uint32_t *__restrict__ uk_start, const uint32_t *__restrict__ row_start_total,
                             uint32_t *__restrict__ row_start, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uk_start[*nu] = *nnz;
        row_start[n] = *row_start_total;
    }
}

__global__ void rows_kernel(const uint32_t *__restrict__ post_seq, const uint16_t *__restrict__ post_pos,
                            const uint32_t *__restrict__ post_u, const uint32_t *__restrict__ nnz_p,
                            const uint32_t *__restrict__ row_start, const uint32_t *__restrict__ uk_start,
                            uint32_t *__restrict__ cursor, uint32_t *__restrict__ row_u, uint16_t *__restrict__ row_pos,
                            uint32_t *__restrict__ row_h) {
    const uint32_t nnz = *nnz_p;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += gridDim.x * blockDim.x) {
        const uint32_t i = post_seq[p];
        const uint32_t u = post_u[p];
        const uint32_t slot = row_start[i] + atomicAdd(&cursor[i], 1u);
        row_u[slot] = u;
        row_pos[slot] = post_pos[p];
        if (row_h) row_h[slot] = uk_start[u] + u;  // postings are grouped by u: these reads run in order
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
    b += sizeof(uint32_t) * m * 3 + 2 * m;                    // sseq, kpos, upos, keep, newk
    b += sizeof(uint32_t) * (n + 1);                          // cursor
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
    uint8_t *keep = (uint8_t *)take(m + 1);
    uint8_t *newk = (uint8_t *)take(m + 1);
    uint32_t *cursor = (uint32_t *)take(sizeof(uint32_t) * (n + 1));
    void *stemp = take(0);

    if ((e = fill<uint32_t>(kt.counts, 4, 0u, s)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(kt.row_cnt, n + 1, 0u, s)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(cursor, n + 1, 0u, s)) != hipSuccess) return e;
    if (m > 0) {
        window_keys_kernel<<<grid_for(m), 256, 0, s>>>(codes, offsets, n, m, k, invalid, keys, vals);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        bool alt = false;
        if ((e = radix_sort(keys, vals, keys2, vals2, m, bits, stemp, s, &alt)) != hipSuccess) return e;
        uint64_t *sk = alt ? keys2 : keys;
        uint32_t *sv = alt ? vals2 : vals;
        mark_kernel<<<grid_for(m), 256, 0, s>>>(sk, sv, offsets, n, m, invalid, sseq, keep, newk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan<uint8_t, uint32_t>(keep, m, kpos, kt.counts + 0, stemp, s)) != hipSuccess) return e;
        if ((e = exclusive_scan<uint8_t, uint32_t>(newk, m, upos, kt.counts + 1, stemp, s)) != hipSuccess) return e;
        postings_kernel<<<grid_for(m), 256, 0, s>>>(sk, sv, sseq, offsets, m, keep, newk, kpos, upos, kt.post_seq,
                                                    kt.post_pos, kt.post_u, kt.uk_id, kt.uk_start, kt.row_cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = exclusive_scan<uint32_t, uint32_t>(kt.row_cnt, n, kt.row_start, kt.counts + 2, stemp, s)) != hipSuccess)
        return e;
    close_kernel<<<1, 64, 0, s>>>(kt.counts + 0, kt.counts + 1, kt.uk_start, kt.counts + 2, kt.row_start, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (m > 0) {
        rows_kernel<<<grid_for(m), 256, 0, s>>>(kt.post_seq, kt.post_pos, kt.post_u, kt.counts + 0, kt.row_start,
                                                kt.uk_start, cursor, kt.row_u, kt.row_pos, kt.row_h);
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
