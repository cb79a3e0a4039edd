// Connected components of the similarity graph and their agreement with
// reference families (Section VI-B, Table II: components taken directly as
// protein families, scored by weighted precision and recall).
//
// Components: lock-free union-find.  Every edge hooks the larger of its two
// roots under the smaller one with a compare-and-swap on the larger root's
// parent; finds halve paths as they go.  A parent never exceeds its child
// and a vertex that stopped being a root never becomes one again, so every
// write a find makes points a vertex at one of its ancestors and concurrent
// hooks and finds only ever shorten paths.  The smallest vertex of a
// component is never hooked, so after a last full compression every vertex
// holds the smallest vertex of its component: a canonical labelling.
//
// Scores: with n_cf the sequences of cluster c in family f, weighted
// precision = sum_c max_f n_cf / N and recall = sum_f max_c n_cf / N.  The
// (cluster, family) keys are sorted; every run of equal keys is one n_cf,
// folded into the per-cluster and per-family maxima with atomics.
#include <algorithm>

#include "internal.hpp"
#include "prim.hpp"

namespace pastis {
namespace {

__device__ __forceinline__ uint32_t load_parent(const uint32_t *p, uint32_t x) {
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (each vertex visited is pointed at
// its grandparent, an ancestor in the same component).
__device__ uint32_t find_root(uint32_t *parent, uint32_t x) {
    uint32_t px = load_parent(parent, x);
    while (px != x) {
        const uint32_t gp = load_parent(parent, px);
        if (gp != px) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = px;
        px = gp;
    }
    return x;
}

__global__ void cc_init_kernel(uint32_t *__restrict__ parent, int64_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = (uint32_t)v;
}

__global__ void cc_hook_kernel(const pastis_edge *__restrict__ edges, int64_t m, int64_t n, uint32_t *parent,
                               unsigned long long *__restrict__ bad) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = edges[e].i, v = edges[e].j;
        if ((int64_t)u >= n || (int64_t)v >= n) {
            atomicMin(bad, (unsigned long long)e);
            continue;
        }
        uint32_t a = find_root(parent, u), b = find_root(parent, v);
        while (a != b) {
            if (a > b) {
                const uint32_t t = a;
                a = b;
                b = t;
            }
            // hook the larger root b under a; if b stopped being a root
            // meanwhile, continue from the roots as they are now
            const uint32_t old = atomicCAS(parent + b, b, a);
            if (old == b) break;
            a = find_root(parent, a);
            b = find_root(parent, old);
        }
    }
}

__global__ void cc_label_kernel(uint32_t *parent, int64_t n, uint32_t *__restrict__ label) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        label[v] = find_root(parent, (uint32_t)v);
}

// key = cluster << 32 | family, a sequence outside every family being the
// family n + v of its own; bad[0] gets the smallest v whose cluster or
// family is >= n
__global__ void score_keys_kernel(const uint32_t *__restrict__ cluster, const int32_t *__restrict__ family,
                                  int64_t n, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                  unsigned long long *__restrict__ bad) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c = cluster[v];
        const int32_t f = family[v];
        if ((int64_t)c >= n || (int64_t)f >= n) {
            atomicMin(bad, (unsigned long long)v);
            c = 0;  // keeps the key inside the tables; the call fails anyway
        }
        const uint32_t fk = f >= 0 && (int64_t)f < n ? (uint32_t)f : (uint32_t)(n + v);
        keys[v] = ((uint64_t)c << 32) | fk;
        vals[v] = (uint32_t)v;
    }
}

__global__ void run_start_kernel(const uint64_t *__restrict__ keys, int64_t n, uint32_t *__restrict__ start) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        start[x] = (x == 0 || keys[x] != keys[x - 1]) ? 1u : 0u;
}

// run_of[x] = exclusive scan of run starts: the run of sorted position x is
// run_of[x] + start[x] - 1; every run adds its length into len[run]
__global__ void run_len_kernel(const uint32_t *__restrict__ start, const uint32_t *__restrict__ run_of, int64_t n,
                               uint32_t *__restrict__ len) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(len + (run_of[x] + start[x] - 1u), 1u);
}

__global__ void run_max_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ start,
                               const uint32_t *__restrict__ run_of, const uint32_t *__restrict__ len, int64_t n,
                               uint32_t *__restrict__ cmax, uint32_t *__restrict__ fmax) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        if (!start[x]) continue;
        const uint32_t m = len[run_of[x]];
        atomicMax(cmax + (keys[x] >> 32), m);
        atomicMax(fmax + (uint32_t)keys[x], m);
    }
}

__global__ void sum_kernel(const uint32_t *__restrict__ a, int64_t n, unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        acc += a[x];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

inline unsigned blocks_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

inline int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

enum CcBuf { kCcParent = kBufCount + 64, kCcFlag, kCcKeys, kCcKeysAlt, kCcVals, kCcValsAlt, kCcTemp, kCcStart,
             kCcRunOf, kCcLen, kCcMax, kCcEnd };
static_assert(kCcEnd <= kNumBufs, "buffer ids");

template <typename T>
pastis_status get(pastis_ctx *ctx, int id, size_t count, T **out) {
    void *p = nullptr;
    PASTIS_TRY(ensure(ctx, id, sizeof(T) * (count > 0 ? count : 1), &p));
    *out = (T *)p;
    return PASTIS_OK;
}

}  // namespace
}  // namespace pastis

using namespace pastis;

extern "C" {

pastis_status pastis_components(pastis_ctx *ctx, const pastis_edge *edges, int64_t n_edges, int64_t n,
                                uint32_t *label, void *stream) {
    if (!ctx) return PASTIS_E_INVAL;
    if (n < 0 || n > 0xFFFFFFFFll || n_edges < 0 || (n_edges > 0 && !edges) || (n > 0 && !label))
        return set_error(ctx, PASTIS_E_INVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (n == 0) {
        if (n_edges > 0) return set_error(ctx, PASTIS_E_INVAL, "edges on an empty vertex set");
        return PASTIS_OK;
    }
    uint32_t *parent = nullptr;
    unsigned long long *bad = nullptr;
    PASTIS_TRY(get(ctx, kCcParent, (size_t)n, &parent));
    PASTIS_TRY(get(ctx, kCcFlag, 1, &bad));
    HIP_TRY(ctx, fill<unsigned long long>(bad, 1, ~0ull, s), "reset");
    cc_init_kernel<<<blocks_for(n), 256, 0, s>>>(parent, n);
    HIP_TRY(ctx, hipGetLastError(), "component kernels");
    if (n_edges > 0) {
        cc_hook_kernel<<<blocks_for(n_edges), 256, 0, s>>>(edges, n_edges, n, parent, bad);
        HIP_TRY(ctx, hipGetLastError(), "component kernels");
    }
    cc_label_kernel<<<blocks_for(n), 256, 0, s>>>(parent, n, label);
    HIP_TRY(ctx, hipGetLastError(), "component kernels");
    unsigned long long h_bad = 0;
    PASTIS_TRY(read_device(ctx, bad, &h_bad, sizeof(h_bad), s));
    if (h_bad != ~0ull)
        return set_error(ctx, PASTIS_E_INVAL, "edge " + std::to_string(h_bad) + " has an endpoint >= n");
    return PASTIS_OK;
}

pastis_status pastis_cluster_scores(pastis_ctx *ctx, const uint32_t *cluster, const int32_t *family, int64_t n,
                                    double *precision, double *recall, void *stream) {
    if (!ctx || !precision || !recall) return PASTIS_E_INVAL;
    if (n < 0 || n >= (1ll << 31) || (n > 0 && (!cluster || !family)))
        return set_error(ctx, PASTIS_E_INVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (n == 0) {
        *precision = *recall = 1.0;
        return PASTIS_OK;
    }
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt, *start, *run_of, *len, *mx;
    unsigned long long *flag;
    char *temp;
    PASTIS_TRY(get(ctx, kCcKeys, (size_t)n, &keys));
    PASTIS_TRY(get(ctx, kCcKeysAlt, (size_t)n, &keys_alt));
    PASTIS_TRY(get(ctx, kCcVals, (size_t)n, &vals));
    PASTIS_TRY(get(ctx, kCcValsAlt, (size_t)n, &vals_alt));
    PASTIS_TRY(get(ctx, kCcTemp, std::max(radix_temp_bytes(n), scan_temp_bytes(n)) + 256, &temp));
    PASTIS_TRY(get(ctx, kCcStart, (size_t)n, &start));
    PASTIS_TRY(get(ctx, kCcRunOf, (size_t)n + 1, &run_of));
    PASTIS_TRY(get(ctx, kCcLen, (size_t)n, &len));
    // cluster maxima [n], family maxima [2n] (families < n, own families n + v)
    PASTIS_TRY(get(ctx, kCcMax, 3 * (size_t)n, &mx));
    PASTIS_TRY(get(ctx, kCcFlag, 3, &flag));
    HIP_TRY(ctx, fill<unsigned long long>(flag, 1, ~0ull, s), "reset");
    HIP_TRY(ctx, fill<unsigned long long>(flag + 1, 2, 0ull, s), "reset");
    HIP_TRY(ctx, fill<uint32_t>(len, n, 0u, s), "reset");
    HIP_TRY(ctx, fill<uint32_t>(mx, 3 * n, 0u, s), "reset");
    score_keys_kernel<<<blocks_for(n), 256, 0, s>>>(cluster, family, n, keys, vals, flag);
    HIP_TRY(ctx, hipGetLastError(), "score kernels");
    unsigned long long h0 = 0;
    PASTIS_TRY(read_device(ctx, flag, &h0, sizeof(h0), s));
    if (h0 != ~0ull)
        return set_error(ctx, PASTIS_E_INVAL, "cluster label or family >= n at sequence " + std::to_string(h0));
    bool alt = false;
    HIP_TRY(ctx, radix_sort(keys, vals, keys_alt, vals_alt, n, 32 + bits_for((uint64_t)n), temp, s, &alt), "sort");
    const uint64_t *sk = alt ? keys_alt : keys;
    run_start_kernel<<<blocks_for(n), 256, 0, s>>>(sk, n, start);
    HIP_TRY(ctx, hipGetLastError(), "score kernels");
    HIP_TRY(ctx, (exclusive_scan<uint32_t, uint32_t>(start, n, run_of, run_of + n, temp, s)), "scan");
    run_len_kernel<<<blocks_for(n), 256, 0, s>>>(start, run_of, n, len);
    run_max_kernel<<<blocks_for(n), 256, 0, s>>>(sk, start, run_of, len, n, mx, mx + n);
    sum_kernel<<<blocks_for(n), 256, 0, s>>>(mx, n, flag + 1);
    sum_kernel<<<blocks_for(2 * n), 256, 0, s>>>(mx + n, 2 * n, flag + 2);
    HIP_TRY(ctx, hipGetLastError(), "score kernels");
    unsigned long long h[2];
    PASTIS_TRY(read_device(ctx, flag + 1, h, sizeof(h), s));
    *precision = (double)h[0] / (double)n;
    *recall = (double)h[1] / (double)n;
    return PASTIS_OK;
}

}  // extern "C"
