// Residue encoding and pair orientation kernels.
#include "internal.hpp"

namespace pastis {

// BLOSUM62 (Henikoff & Henikoff 1992), rows/columns in the residue order
// A R N D C Q E G H I L K M F P S T W Y V B Z X *.
const int8_t kBlosum62[kAlpha * kAlpha] = {
    4,  -1, -2, -2, 0,  -1, -1, 0,  -2, -1, -1, -1, -1, -2, -1, 1,  0,  -3, -2, 0,  -2, -1, 0,  -4,  // A
    -1, 5,  0,  -2, -3, 1,  0,  -2, 0,  -3, -2, 2,  -1, -3, -2, -1, -1, -3, -2, -3, -1, 0,  -1, -4,  // R
    -2, 0,  6,  1,  -3, 0,  0,  0,  1,  -3, -3, 0,  -2, -3, -2, 1,  0,  -4, -2, -3, 3,  0,  -1, -4,  // N
    -2, -2, 1,  6,  -3, 0,  2,  -1, -1, -3, -4, -1, -3, -3, -1, 0,  -1, -4, -3, -3, 4,  1,  -1, -4,  // D
    0,  -3, -3, -3, 9,  -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4,  // C
    -1, 1,  0,  0,  -3, 5,  2,  -2, 0,  -3, -2, 1,  0,  -3, -1, 0,  -1, -2, -1, -2, 0,  3,  -1, -4,  // Q
    -1, 0,  0,  2,  -4, 2,  5,  -2, 0,  -3, -3, 1,  -2, -3, -1, 0,  -1, -3, -2, -2, 1,  4,  -1, -4,  // E
    0,  -2, 0,  -1, -3, -2, -2, 6,  -2, -4, -4, -2, -3, -3, -2, 0,  -2, -2, -3, -3, -1, -2, -1, -4,  // G
    -2, 0,  1,  -1, -3, 0,  0,  -2, 8,  -3, -3, -1, -2, -1, -2, -1, -2, -2, 2,  -3, 0,  0,  -1, -4,  // H
    -1, -3, -3, -3, -1, -3, -3, -4, -3, 4,  2,  -3, 1,  0,  -3, -2, -1, -3, -1, 3,  -3, -3, -1, -4,  // I
    -1, -2, -3, -4, -1, -2, -3, -4, -3, 2,  4,  -2, 2,  0,  -3, -2, -1, -2, -1, 1,  -4, -3, -1, -4,  // L
    -1, 2,  0,  -1, -3, 1,  1,  -2, -1, -3, -2, 5,  -1, -3, -1, 0,  -1, -3, -2, -2, 0,  1,  -1, -4,  // K
    -1, -1, -2, -3, -1, 0,  -2, -3, -2, 1,  2,  -1, 5,  0,  -2, -1, -1, -1, -1, 1,  -3, -1, -1, -4,  // M
    -2, -3, -3, -3, -2, -3, -3, -3, -1, 0,  0,  -3, 0,  6,  -4, -2, -2, 1,  3,  -1, -3, -3, -1, -4,  // F
    -1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7,  -1, -1, -4, -3, -2, -2, -1, -2, -4,  // P
    1,  -1, 1,  0,  -1, 0,  0,  0,  -1, -2, -2, 0,  -1, -2, -1, 4,  1,  -3, -2, -2, 0,  0,  0,  -4,  // S
    0,  -1, 0,  -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1,  5,  -2, -2, 0,  -1, -1, 0,  -4,  // T
    -3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1,  -4, -3, -2, 11, 2,  -3, -4, -3, -2, -4,  // W
    -2, -2, -2, -3, -2, -1, -2, -3, 2,  -1, -1, -2, -1, 3,  -3, -2, -2, 2,  7,  -1, -3, -2, -1, -4,  // Y
    0,  -3, -3, -3, -1, -2, -2, -3, -3, 3,  1,  -2, 1,  -1, -2, -2, 0,  -3, -1, 4,  -3, -2, -1, -4,  // V
    -2, -1, 3,  4,  -3, 0,  1,  -1, 0,  -3, -4, 0,  -3, -3, -2, 0,  -1, -4, -3, -3, 4,  1,  -1, -4,  // B
    -1, 0,  0,  1,  -3, 3,  4,  -2, 0,  -3, -3, 1,  -1, -3, -1, 0,  -1, -3, -2, -2, 1,  4,  -1, -4,  // Z
    0,  -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2, 0,  0,  -2, -1, -1, -1, -1, -1, -4,  // X
    -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, 1,   // *
};

namespace {

__constant__ uint8_t kAsciiToCode[256];

// One thread per byte; the smallest offending index is kept with atomicMin.
__global__ void encode_kernel(const uint8_t *__restrict__ ascii, int64_t n, uint8_t *__restrict__ codes,
                              unsigned long long *__restrict__ bad) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride) {
        uint8_t c = kAsciiToCode[ascii[t]];
        codes[t] = c;
        if (c == 0xFF) atomicMin(bad, (unsigned long long)t);
    }
}

bool g_table_ready[64] = {false};

hipError_t upload_ascii_table() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 64 && g_table_ready[dev]) return hipSuccess;
    static const char kLetters[] = "ARNDCQEGHILKMFPSTWYVBZX*";
    uint8_t table[256];
    memset(table, 0xFF, sizeof(table));
    for (int c = 0; c < kAlpha; ++c) table[(uint8_t)kLetters[c]] = (uint8_t)c;
    e = hipMemcpyToSymbol(HIP_SYMBOL(kAsciiToCode), table, sizeof(table));
    if (e == hipSuccess && dev < 64) g_table_ready[dev] = true;
    return e;
}

// Orientation: rows a = the shorter sequence, the first of the pair on equal
// length.  Seeds arrive as (pos in min(i,j) << 16 | pos in max(i,j)).
__global__ void orient_kernel(const int64_t *__restrict__ offsets, int64_t n, const uint32_t *__restrict__ pi,
                              const uint32_t *__restrict__ pj, const uint32_t *__restrict__ seed1,
                              const uint32_t *__restrict__ seed2, int64_t npairs, int k, PairDesc *__restrict__ out,
                              unsigned long long *__restrict__ bad) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    uint32_t i = pi[q], j = pj[q];
    PairDesc d;
    if (i >= (uint64_t)n || j >= (uint64_t)n || i == j) {
        atomicOr(bad, 1ull);
        memset(&d, 0, sizeof(d));
        d.pa1 = d.pb1 = d.pa2 = d.pb2 = -1;
        out[q] = d;
        return;
    }
    int64_t li = offsets[i + 1] - offsets[i], lj = offsets[j + 1] - offsets[j];
    if (li > kMaxLen || lj > kMaxLen) atomicOr(bad, 2ull);
    const bool swapped = !(li < lj || (li == lj && i < j));
    d.a_off = swapped ? offsets[j] : offsets[i];
    d.b_off = swapped ? offsets[i] : offsets[j];
    d.la = (int32_t)(swapped ? lj : li);
    d.lb = (int32_t)(swapped ? li : lj);
    d.swapped = swapped ? 1 : 0;
    d.a_seq = (int32_t)(swapped ? j : i);
    int32_t pa[2] = {-1, -1}, pb[2] = {-1, -1};
    for (int s = 0; s < 2; ++s) {
        const uint32_t *src = s == 0 ? seed1 : seed2;
        uint32_t key = src ? src[q] : kNoSeed;
        if (key == kNoSeed) continue;
        int32_t plo = (int32_t)(key >> 16), phi = (int32_t)(key & 0xFFFF);
        int32_t p_i = (i < j) ? plo : phi, p_j = (i < j) ? phi : plo;
        int32_t a = swapped ? p_j : p_i, b = swapped ? p_i : p_j;
        if (a + k > d.la || b + k > d.lb) continue;  // not a k-mer of these sequences
        pa[s] = a;
        pb[s] = b;
    }
    d.pa1 = pa[0];
    d.pb1 = pb[0];
    d.pa2 = pa[1];
    d.pb2 = pb[1];
    out[q] = d;
}

}  // namespace

hipError_t launch_encode(const uint8_t *ascii, int64_t n, uint8_t *codes, unsigned long long *bad, hipStream_t s) {
    hipError_t e = upload_ascii_table();
    if (e != hipSuccess) return e;
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    encode_kernel<<<(unsigned)blocks, 256, 0, s>>>(ascii, n, codes, bad);
    return hipGetLastError();
}

hipError_t launch_orient_pairs(const int64_t *offsets, int64_t n, const uint32_t *pi, const uint32_t *pj,
                               const uint32_t *seed1, const uint32_t *seed2, int64_t npairs, int k, PairDesc *out,
                               unsigned long long *bad, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    orient_kernel<<<(unsigned)((npairs + 255) / 256), 256, 0, s>>>(offsets, n, pi, pj, seed1, seed2, npairs, k, out,
                                                                   bad);
    return hipGetLastError();
}

}  // namespace pastis
