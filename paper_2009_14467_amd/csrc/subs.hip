// Substitute k-mers: the rows of S (Section IV-B).
//
// For a k-mer r, expense(a -> b) = C[a][a] - C[a][b] (E = Sort(Diag(C) - C))
// and Dist(s, r) sums the expenses position by position.  The row of r holds r
// itself (distance 0) and its m nearest other k-mers over the substitute
// alphabet, ties broken by the smaller id.  Substitutes that occur in no
// sequence cannot produce a match and are dropped after selection.
//
// Algorithms 1-3 of the paper find the m nearest with heaps.  Here one thread
// handles one k-mer without a heap:
//   1. count the k-mers within distance D for D = lower bound, +1, ... until
//      at least m others fit (depth-first walk, children in expense order, a
//      branch cut as soon as its partial sum plus the smallest possible rest
//      exceeds D); call the final radius D*;
//   2. emit every k-mer strictly closer than D*;
//   3. walk the k-mers at exactly D* in id order (children in residue order)
//      and emit the first ones until m are emitted.
// Every k-mer within a radius is reachable (each position may change to any
// residue), so this returns exactly the (Dist, id)-ordered first m.
#include "internal.hpp"
#include "subs.hpp"

namespace pastis {
namespace {

struct SubsTables {
    int8_t ex[kAlpha][kAlpha];       // expense(a -> b)
    uint8_t ord_b[kAlpha][kAlpha];   // row a: bases by (expense, base)
    int8_t ord_e[kAlpha][kAlpha];    // their expenses
};

__device__ void load_tables(SubsTables &T, const int8_t *blosum25, int alpha) {
    for (int t = threadIdx.x; t < kAlpha * kAlpha; t += blockDim.x) {
        const int a = t / kAlpha, b = t % kAlpha;
        T.ex[a][b] = (int8_t)(blosum25[a * 25 + a] - blosum25[a * 25 + b]);
    }
    __syncthreads();
    if (threadIdx.x < kAlpha) {
        const int a = threadIdx.x;
        int n = 0;
        for (int b = 0; b < alpha; ++b) {
            const int e = T.ex[a][b];
            int t = n++;
            while (t > 0 && (T.ord_e[a][t - 1] > e || (T.ord_e[a][t - 1] == e && T.ord_b[a][t - 1] > b))) {
                T.ord_e[a][t] = T.ord_e[a][t - 1];
                T.ord_b[a][t] = T.ord_b[a][t - 1];
                --t;
            }
            T.ord_e[a][t] = (int8_t)e;
            T.ord_b[a][t] = (uint8_t)b;
        }
    }
    __syncthreads();
}

struct Walk {
    const SubsTables *T;
    int rc[kMaxK];
    int minrest[kMaxK + 1];
    int alpha, D;
    uint64_t r;
};

// number of k-mers within distance D (r included when it qualifies), or any
// number >= limit once that many are found: only "at least limit" matters,
// and a radius can hold up to 20^k k-mers (every k-mer of X is at distance
// <= 0 from XX...X)
template <int T, int K>
__device__ __forceinline__ uint32_t count_within(const Walk &w, int partial, uint32_t limit) {
    if constexpr (T == K) {
        return 1u;
    } else {
        uint32_t c = 0;
        const int a = w.rc[T];
        for (int q = 0; q < w.alpha && c < limit; ++q) {
            const int p = partial + w.T->ord_e[a][q];
            if (p + w.minrest[T + 1] > w.D) break;  // children come in expense order
            c += count_within<T + 1, K>(w, p, limit - c);
        }
        return c;
    }
}

struct Sink {
    uint64_t *ids;
    int8_t *dist;
    int n, cap;
};

// emit every k-mer s != r with Dist < D (expense order)
template <int T, int K>
__device__ __forceinline__ void emit_below(const Walk &w, int partial, uint64_t id, Sink &out) {
    if constexpr (T == K) {
        if (partial < w.D && id != w.r && out.n < out.cap) {
            out.ids[out.n] = id;
            out.dist[out.n] = (int8_t)partial;
            ++out.n;
        }
    } else {
        const int a = w.rc[T];
        for (int q = 0; q < w.alpha; ++q) {
            const int p = partial + w.T->ord_e[a][q];
            if (p + w.minrest[T + 1] > w.D - 1) break;
            emit_below<T + 1, K>(w, p, id * 24u + (uint64_t)w.T->ord_b[a][q], out);
        }
    }
}

// emit k-mers s != r with Dist == D in id order until the sink is full
template <int T, int K>
__device__ __forceinline__ void emit_at(const Walk &w, int partial, uint64_t id, Sink &out) {
    if constexpr (T == K) {
        if (partial == w.D && id != w.r && out.n < out.cap) {
            out.ids[out.n] = id;
            out.dist[out.n] = (int8_t)partial;
            ++out.n;
        }
    } else {
        const int a = w.rc[T];
        for (int b = 0; b < w.alpha && out.n < out.cap; ++b) {
            const int p = partial + w.T->ex[a][b];
            if (p + w.minrest[T + 1] > w.D) continue;
            emit_at<T + 1, K>(w, p, id * 24u + (uint64_t)b, out);
        }
    }
}

template <int K>
__device__ int nearest(const SubsTables &T, uint64_t r, int alpha, int m, uint64_t *ids, int8_t *dist) {
    Walk w;
    w.T = &T;
    w.alpha = alpha;
    w.r = r;
    uint64_t x = r;
    bool in_alpha = true;
    for (int t = K - 1; t >= 0; --t) {
        w.rc[t] = (int)(x % 24u);
        x /= 24u;
        in_alpha &= w.rc[t] < alpha;
    }
    w.minrest[K] = 0;
    for (int t = K - 1; t >= 0; --t) w.minrest[t] = w.minrest[t + 1] + T.ord_e[w.rc[t]][0];
    uint64_t total = 1;
    for (int t = 0; t < K; ++t) total *= (uint64_t)alpha;
    const uint64_t others = total - (in_alpha ? 1 : 0);
    const int want = (int)(others < (uint64_t)m ? others : (uint64_t)m);
    if (want <= 0) return 0;
    // r is within every radius D >= 0 when its residues are all substitutable
    for (w.D = w.minrest[0];; ++w.D) {
        uint32_t c = count_within<0, K>(w, 0, (uint32_t)want + 1);
        if (in_alpha && w.D >= 0) --c;
        if (c >= (uint32_t)want) break;
    }
    Sink out{ids, dist, 0, want};
    emit_below<0, K>(w, 0, 0ull, out);
    emit_at<0, K>(w, 0, 0ull, out);
    return out.n;
}

__device__ int nearest_k(int k, const SubsTables &T, uint64_t r, int alpha, int m, uint64_t *ids, int8_t *dist) {
    switch (k) {
        case 1: return nearest<1>(T, r, alpha, m, ids, dist);
        case 2: return nearest<2>(T, r, alpha, m, ids, dist);
        case 3: return nearest<3>(T, r, alpha, m, ids, dist);
        case 4: return nearest<4>(T, r, alpha, m, ids, dist);
        case 5: return nearest<5>(T, r, alpha, m, ids, dist);
        case 6: return nearest<6>(T, r, alpha, m, ids, dist);
        case 7: return nearest<7>(T, r, alpha, m, ids, dist);
        default: return nearest<8>(T, r, alpha, m, ids, dist);
    }
}

// compact index of k-mer id among the nu ascending distinct ids, or -1
__device__ __forceinline__ int32_t find_compact(const uint64_t *__restrict__ uk_id, uint32_t nu, uint64_t id) {
    uint32_t lo = 0, hi = nu;  // first index with uk_id >= id in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (uk_id[mid] < id)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < nu && uk_id[lo] == id) ? (int32_t)lo : -1;
}

// Rows of S for the distinct k-mers of the data: row u holds (m + 1) slots;
// slot 0 is u itself; present substitutes follow; s_cnt[u] counts them.  A
// slot names its k-mer v by the head of v's posting group, uk_start[v] + v
// (the dense map holds heads already).
__global__ __launch_bounds__(256) void s_rows_kernel(const uint64_t *__restrict__ uk_id, const uint32_t *__restrict__ nu_p,
                                                     const uint32_t *__restrict__ uk_start,
                                                     const int32_t *__restrict__ kmap, const int8_t *__restrict__ blosum25,
                                                     int k, int m, int alpha, uint32_t *__restrict__ s_u,
                                                     int8_t *__restrict__ s_d, uint32_t *__restrict__ s_cnt,
                                                     uint64_t *__restrict__ tmp_ids, int8_t *__restrict__ tmp_d) {
    __shared__ SubsTables T;
    load_tables(T, blosum25, alpha);
    const uint32_t nu = *nu_p;
    const int W = m + 1;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += gridDim.x * blockDim.x) {
        uint64_t *ids = tmp_ids + (size_t)(blockIdx.x * blockDim.x + threadIdx.x) * m;
        int8_t *dd = tmp_d + (size_t)(blockIdx.x * blockDim.x + threadIdx.x) * m;
        const int got = nearest_k(k, T, uk_id[u], alpha, m, ids, dd);
        uint32_t *row = s_u + (size_t)u * W;
        int8_t *drow = s_d + (size_t)u * W;
        row[0] = uk_start[u] + u;
        drow[0] = 0;
        int c = 1;
        for (int q = 0; q < got; ++q) {
            int64_t hv = -1;
            if (kmap) {
                hv = kmap[ids[q]];
            } else {
                const int32_t cu = find_compact(uk_id, nu, ids[q]);
                if (cu >= 0) hv = (int64_t)uk_start[cu] + cu;
            }
            if (hv < 0) continue;
            row[c] = (uint32_t)hv;
            drow[c] = dd[q];
            ++c;
        }
        s_cnt[u] = (uint32_t)c;
    }
}

// Neighbourhoods of arbitrary k-mer ids (checking entry point).
__global__ void nearest_ids_kernel(const uint64_t *__restrict__ kid, int64_t n, const int8_t *__restrict__ blosum25,
                                   int k, int m, int alpha, uint64_t *__restrict__ out_ids, int8_t *__restrict__ out_d,
                                   int32_t *__restrict__ out_n) {
    __shared__ SubsTables T;
    load_tables(T, blosum25, alpha);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out_n[q] = nearest_k(k, T, kid[q], alpha, m, out_ids + q * m, out_d + q * m);
}

}  // namespace

int s_rows_threads() { return 256 * 1024; }

hipError_t launch_s_rows(const uint64_t *uk_id, const uint32_t *nu, const uint32_t *uk_start, const int32_t *kmap,
                         const int8_t *blosum25, int k, int m, int alpha, uint32_t *s_u, int8_t *s_d, uint32_t *s_cnt,
                         uint64_t *tmp_ids, int8_t *tmp_d, hipStream_t s) {
    s_rows_kernel<<<1024, 256, 0, s>>>(uk_id, nu, uk_start, kmap, blosum25, k, m, alpha, s_u, s_d, s_cnt, tmp_ids,
                                       tmp_d);
    return hipGetLastError();
}

hipError_t launch_nearest_ids(const uint64_t *kid, int64_t n, const int8_t *blosum25, int k, int m, int alpha,
                              uint64_t *out_ids, int8_t *out_d, int32_t *out_n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    nearest_ids_kernel<<<(unsigned)blocks, 256, 0, s>>>(kid, n, blosum25, k, m, alpha, out_ids, out_d, out_n);
    return hipGetLastError();
}

}  // namespace pastis
