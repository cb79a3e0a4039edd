// Device primitives: fill, exclusive scan, and a stable LSD radix sort of
// 64-bit keys with 32-bit payloads.  All are enqueued on a stream with no host
// round trip; temporary storage comes from the caller.
#include "internal.hpp"
#include "prim.hpp"

namespace pastis {
namespace {

constexpr int kWave = 64;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__global__ void fill_kernel(T *p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// inclusive prefix over the 256 threads of a block
__device__ __forceinline__ uint64_t block_inclusive(uint64_t v, uint64_t *smem_waves) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    if (lane == kWave - 1) smem_waves[wave] = v;
    __syncthreads();
    uint64_t add = 0;
    for (int w = 0; w < wave; ++w) add += smem_waves[w];
    __syncthreads();
    return v + add;
}

template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void scan_partials_kernel(const TIn *__restrict__ in, int64_t n,
                                                                     uint64_t *__restrict__ partial) {
    __shared__ uint64_t sw[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += (uint64_t)in[i];
    }
    const uint64_t inc = block_inclusive(s, sw);
    if (threadIdx.x == kScanThreads - 1) partial[blockIdx.x] = inc;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(const TIn *__restrict__ in, int64_t n,
                                                                  const uint64_t *__restrict__ offs,
                                                                  TOut *__restrict__ out, TOut *__restrict__ total) {
    __shared__ uint64_t sw[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = (i < n) ? (uint64_t)in[i] : 0;
        s += v[k];
    }
    const uint64_t inc = block_inclusive(s, sw);
    uint64_t run = inc - s + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = (TOut)run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total = (TOut)run;
}

// ---- radix sort (8-bit digits, stable) ----
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;  // per thread per pass over a tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kWavesPerSortBlock = kSortThreads / kWave;
constexpr int kWaveTile = kSortTile / kWavesPerSortBlock;  // consecutive elements per wave
constexpr int kWaveChunks = kWaveTile / kWave;

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t *__restrict__ keys, int64_t n,
                                                                  int shift, int nblocks, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// One tile per block.  The tile is ranked stably by digit in LDS (each wave
// ranks its contiguous quarter 64 elements at a time with ballots), then
// written out in digit order, so a digit's run of the tile goes to
// consecutive addresses from consecutive threads.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n, int shift, int nblocks,
    const uint64_t *__restrict__ offs, uint64_t *__restrict__ okeys, uint32_t *__restrict__ ovals) {
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t whist[kWavesPerSortBlock][256];  // then each wave's next local slot per digit
    __shared__ uint32_t dstart[256];                     // the digit's first slot in the tile
    __shared__ uint64_t gbase[256];                      // the digit's first output address of this tile
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int d = threadIdx.x; d < kWavesPerSortBlock * 256; d += kSortThreads) (&whist[0][0])[d] = 0;
    __syncthreads();
    const int64_t tstart = (int64_t)blockIdx.x * kSortTile;
    const int64_t wstart = tstart + (int64_t)wave * kWaveTile;
    uint64_t k[kWaveChunks];
    uint32_t v[kWaveChunks];
#pragma unroll
    for (int c = 0; c < kWaveChunks; ++c) {
        const int64_t i = wstart + c * kWave + lane;
        const bool ok = i < n;
        k[c] = ok ? keys[i] : 0;
        v[c] = ok ? vals[i] : 0;
        if (ok) atomicAdd(&whist[wave][(k[c] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // 256 threads, one digit each
        gbase[d] = offs[(int64_t)d * nblocks + blockIdx.x];
        uint32_t tot = 0;
        for (int w = 0; w < kWavesPerSortBlock; ++w) tot += whist[w][d];
        dstart[d] = tot;  // the digit's count, scanned below
    }
    __syncthreads();
    // exclusive scan of the 256 counts (one wave, four per lane)
    if (wave == 0) {
        uint32_t c4[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c4[j] = dstart[4 * lane + j];
            sum += c4[j];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)inc, off, kWave);
            if (lane >= off) inc += o;
        }
        uint32_t run = inc - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dstart[4 * lane + j] = run;
            run += c4[j];
        }
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = dstart[d];
        for (int w = 0; w < kWavesPerSortBlock; ++w) {
            const uint32_t c = whist[w][d];
            whist[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int c = 0; c < kWaveChunks; ++c) {
        const int64_t i = wstart + c * kWave + lane;
        const bool ok = i < n;
        const int d = (int)((k[c] >> shift) & 0xFF);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        const int before = __popcll(peers & lt);
        uint32_t slot = 0;
        if (ok) slot = whist[wave][d] + (uint32_t)before;
        __builtin_amdgcn_wave_barrier();
        if (ok && before == 0) whist[wave][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (ok) {
            skey[slot] = k[c];
            sval[slot] = v[c];
        }
    }
    __syncthreads();
    const int count = (int)((n - tstart) < (int64_t)kSortTile ? (n - tstart) : (int64_t)kSortTile);
    for (int p = threadIdx.x; p < count; p += kSortThreads) {
        const uint64_t key = skey[p];
        const int d = (int)((key >> shift) & 0xFF);
        const uint64_t pos = gbase[d] + (uint64_t)(p - (int)dstart[d]);
        okeys[pos] = key;
        ovals[pos] = sval[p];
    }
}

__global__ void iota_kernel(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T>
hipError_t fill(T *p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_kernel<T><<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}
template hipError_t fill<int>(int *, int64_t, int, hipStream_t);
template hipError_t fill<uint32_t>(uint32_t *, int64_t, uint32_t, hipStream_t);
template hipError_t fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template hipError_t fill<uint64_t>(uint64_t *, int64_t, uint64_t, hipStream_t);
template hipError_t fill<unsigned long long>(unsigned long long *, int64_t, unsigned long long, hipStream_t);

hipError_t iota(uint32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    iota_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

size_t scan_temp_bytes(int64_t n) {
    size_t total = 0;
    int64_t m = n;
    while (m > 1) {
        m = (m + kScanTile - 1) / kScanTile;
        total += sizeof(uint64_t) * (size_t)(2 * m + 2);
    }
    return total + 256;
}

template <typename TIn, typename TOut>
hipError_t exclusive_scan(const TIn *in, int64_t n, TOut *out, TOut *total, void *temp, hipStream_t s) {
    if (n <= 0) {
        if (total) return fill<TOut>(total, 1, (TOut)0, s);
        return hipSuccess;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        scan_tiles_kernel<TIn, TOut><<<1, kScanThreads, 0, s>>>(in, n, nullptr, out, total);
        return hipGetLastError();
    }
    uint64_t *partial = (uint64_t *)temp;
    uint64_t *poffs = partial + nb + 1;
    void *rest = poffs + nb + 1;
    scan_partials_kernel<TIn><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan<uint64_t, uint64_t>(partial, nb, poffs, (uint64_t *)nullptr, rest, s);
    if (e != hipSuccess) return e;
    scan_tiles_kernel<TIn, TOut><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, poffs, out, total);
    return hipGetLastError();
}
template hipError_t exclusive_scan<uint32_t, uint64_t>(const uint32_t *, int64_t, uint64_t *, uint64_t *, void *,
                                                       hipStream_t);
template hipError_t exclusive_scan<uint32_t, uint32_t>(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *,
                                                       hipStream_t);
template hipError_t exclusive_scan<uint64_t, uint64_t>(const uint64_t *, int64_t, uint64_t *, uint64_t *, void *,
                                                       hipStream_t);
template hipError_t exclusive_scan<int, int64_t>(const int *, int64_t, int64_t *, int64_t *, void *, hipStream_t);
template hipError_t exclusive_scan<uint8_t, uint32_t>(const uint8_t *, int64_t, uint32_t *, uint32_t *, void *,
                                                      hipStream_t);

size_t radix_temp_bytes(int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t h = 256 * (nb > 0 ? nb : 1);
    return sizeof(uint32_t) * (size_t)h + sizeof(uint64_t) * (size_t)h + scan_temp_bytes(h) + 256;
}

hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, int64_t n, int bits,
                      void *temp, hipStream_t s, bool *result_in_alt) {
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    uint32_t *hist = (uint32_t *)temp;
    uint64_t *offs = (uint64_t *)(hist + 256 * nb);
    void *stemp = offs + 256 * nb;
    uint64_t *k0 = keys, *k1 = keys_alt;
    uint32_t *v0 = vals, *v1 = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_hist_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(k0, n, shift, (int)nb, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan<uint32_t, uint64_t>(hist, 256 * nb, offs, (uint64_t *)nullptr, stemp, s);
        if (e != hipSuccess) return e;
        radix_scatter_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(k0, v0, n, shift, (int)nb, offs, k1, v1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        uint64_t *tk = k0;
        k0 = k1;
        k1 = tk;
        uint32_t *tv = v0;
        v0 = v1;
        v1 = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

}  // namespace pastis
