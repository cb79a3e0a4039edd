// Device-side binning of work items: bin ids -> per-bin index lists, with no
// host round trip (the consumer kernels read the bin bounds from device
// memory), so a whole alignment stage can be enqueued, or captured, at once.
#include "internal.hpp"

namespace pastis {
namespace {

constexpr int kMaxBins = 32;

__global__ void bin_zero_kernel(int *counts, int nbins) {
    int t = threadIdx.x;
    if (t < nbins) counts[t] = 0;
}

// Per-block histogram in LDS, then one global atomic per (block, bin).
__global__ void bin_count_kernel(const int8_t *__restrict__ bin_of, int64_t n, int nbins, int *__restrict__ counts) {
    __shared__ int local[kMaxBins];
    if (threadIdx.x < kMaxBins) local[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        int b = bin_of[q];
        if (b >= 0) atomicAdd(&local[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < nbins && local[threadIdx.x]) atomicAdd(&counts[threadIdx.x], local[threadIdx.x]);
}

__global__ void bin_scan_kernel(const int *__restrict__ counts, int nbins, int *__restrict__ starts,
                                int *__restrict__ cursor) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < nbins; ++b) {
            starts[b] = acc;
            cursor[b] = acc;
            acc += counts[b];
        }
        starts[nbins] = acc;
    }
}

// Each block reserves its slots per bin with one atomic, then places its
// items in index order inside that range.
__global__ void bin_scatter_kernel(const int8_t *__restrict__ bin_of, int64_t n, int nbins, int *__restrict__ cursor,
                                   int *__restrict__ idx) {
    __shared__ int local[kMaxBins];
    __shared__ int base[kMaxBins];
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x;
    for (int64_t chunk = q0; chunk < n; chunk += (int64_t)gridDim.x * blockDim.x) {
        if (threadIdx.x < kMaxBins) local[threadIdx.x] = 0;
        __syncthreads();
        const int64_t q = chunk + threadIdx.x;
        int b = (q < n) ? bin_of[q] : -1;
        int slot = (b >= 0) ? atomicAdd(&local[b], 1) : 0;
        __syncthreads();
        if (threadIdx.x < nbins && local[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], local[threadIdx.x]);
        __syncthreads();
        if (b >= 0) idx[base[b] + slot] = (int)q;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_bins(const int8_t *bin_of, int64_t n, int nbins, int *counts, int *starts, int *cursor, int *idx,
                       hipStream_t s) {
    if (nbins > kMaxBins) return hipErrorInvalidValue;
    bin_zero_kernel<<<1, 64, 0, s>>>(counts, nbins);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    bin_count_kernel<<<(unsigned)blocks, 256, 0, s>>>(bin_of, n, nbins, counts);
    bin_scan_kernel<<<1, 64, 0, s>>>(counts, nbins, starts, cursor);
    bin_scatter_kernel<<<(unsigned)blocks, 256, 0, s>>>(bin_of, n, nbins, cursor, idx);
    return hipGetLastError();
}

}  // namespace pastis
