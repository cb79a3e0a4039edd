// Learned pre-alignment filter: per-pair features and a 16-128-128-1 MLP
// with bf16 weights and activations, fp32 accumulation on MFMA (not part of
// the paper: it predicts whether a candidate pair will pass the identity /
// coverage cut of Section IV-F, so that predicted failures skip alignment).
//
// Features of a pair (a = the shorter sequence): shared-k-mer count; seed-1
// diagonal (pos_b - pos_a) / Lb; |diag2 - diag1| / Lb; ln La; ln Lb; La / Lb;
// and |comp_a - comp_b| over 10 residue groups {AG}{ST}{DE}{NQ}{KRH}{IV}{LM}
// {FYW}{C}{P}.  They are z-scored with training statistics and cast to bf16.
//
// Layout.  A wave handles 16 pairs and computes each layer transposed,
// H^T = W X^T, with v_mfma_f32_16x16x16bf16: the 16x16 accumulator of an
// output-feature tile (lane l: features 4*(l/16)..+3 of pair l%16) is exactly
// the B operand of the next layer's K tile, so layers chain in registers.
// Training stores activations and gradients by tile of 16 pairs, feature by
// feature inside a tile ([pair / 16][feature][pair % 16], bf16): a wave's
// stores of one array share one address with immediate offsets, and both
// operands of the weight-gradient GEMMs (reductions over the batch) load 4
// consecutive pairs of a feature per lane, 512 contiguous bytes per wave.
#include <cmath>

#include "internal.hpp"
#include "mlp.hpp"
#include "prim.hpp"

namespace pastis {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = kMlpIn, kH = kMlpHidden;

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 load4(const uint16_t *p) {
    const uint2 v = *(const uint2 *)p;  // 4 bf16, 8-byte aligned
    bf16x4 r;
    r[0] = (short)(v.x & 0xFFFF);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFF);
    r[3] = (short)(v.y >> 16);
    return r;
}

// group of residue code c (0..23), or -1
__device__ __forceinline__ int group_of(int c) {
    // A R N D C Q E G H I L K M F P S T W Y V B Z X *
    const int8_t g[24] = {0, 4, 3, 2, 8, 3, 2, 0, 4, 5, 6, 4, 6, 7, 9, 1, 1, 7, 7, 5, -1, -1, -1, -1};
    return g[c];
}

__global__ void comp_kernel(const uint8_t *__restrict__ codes, const int64_t *__restrict__ offsets, int64_t n,
                            float *__restrict__ comp) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int cnt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        const int64_t b = offsets[i], e = offsets[i + 1];
        for (int64_t x = b; x < e; ++x) {
            const int g = group_of(codes[x]);
            if (g >= 0) cnt[g]++;
        }
        const float L = (float)((e - b) > 0 ? (e - b) : 1);
        for (int g = 0; g < 10; ++g) comp[i * 10 + g] = (float)cnt[g] / L;
    }
}

__global__ void features_kernel(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                const uint32_t *__restrict__ count, const uint32_t *__restrict__ s1,
                                const uint32_t *__restrict__ s2, int64_t n, const int64_t *__restrict__ offsets,
                                const float *__restrict__ comp, float *__restrict__ F) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = lo[q], j = hi[q];
        const int64_t Li = offsets[i + 1] - offsets[i], Lj = offsets[j + 1] - offsets[j];
        const bool swap = !(Li < Lj || (Li == Lj && i < j));
        const float La = (float)(swap ? Lj : Li), Lb = (float)(swap ? Li : Lj);
        const uint32_t ia = swap ? j : i, ib = swap ? i : j;
        float *f = F + q * kIn;
        f[0] = (float)count[q];
        const uint32_t k1 = s1[q], k2 = s2[q];
        auto diag = [&](uint32_t key) {
            const int p_lo = (int)(key >> 16), p_hi = (int)(key & 0xFFFF);
            const int pa = swap ? p_hi : p_lo, pb = swap ? p_lo : p_hi;
            return (float)(pb - pa);
        };
        const float d1 = k1 != kNoSeed ? diag(k1) : 0.f;
        const float d2 = k2 != kNoSeed ? diag(k2) : 0.f;
        f[1] = k1 != kNoSeed ? d1 / Lb : 0.f;
        f[2] = (k1 != kNoSeed && k2 != kNoSeed) ? fabsf(d2 - d1) / Lb : 0.f;
        f[3] = logf(La);
        f[4] = logf(Lb);
        f[5] = La / Lb;
        for (int g = 0; g < 10; ++g) f[6 + g] = fabsf(comp[ia * 10 + g] - comp[ib * 10 + g]);
    }
}

struct Net {
    const uint16_t *W1b, *W2b, *W2Tb, *w3b;  // bf16 copies
    const float *b1, *b2, *b3;
    const float *mean, *stdv;
};

// B operand of layer 1 for this lane: features 4*kg..+3 of pair p, normalised
__device__ __forceinline__ bf16x4 input_operand(const float *X, int64_t p, bool valid, int kg, const Net &N,
                                                float zf[4]) {
    bf16x4 z;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int f = 4 * kg + i;
        const float v = valid ? (X[p * kIn + f] - N.mean[f]) / N.stdv[f] : 0.f;
        const uint16_t h = valid ? to_bf16(v) : (uint16_t)0;
        z[i] = (short)h;
        zf[i] = from_bf16(h);
    }
    return z;
}

struct Fwd {
    bf16x4 h1[8];        // B operands of layer 2
    float a1p[8][4];     // pre-activations of layer 1 (sign only is used)
    float h2[8][4];      // bf16-valued layer-2 activations
    float a2p[8][4];
    float y;             // logit of pair l % 16 (all four lane groups hold it)
};

__device__ __forceinline__ void forward_tile(bf16x4 zop, const Net &N, int lane, Fwd &o) {
    const int col = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const bf16x4 a = load4(N.W1b + (16 * t + col) * kIn + 4 * kg);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(a, zop, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float pre = acc[i] + N.b1[16 * t + 4 * kg + i];
            o.a1p[t][i] = pre;
            o.h1[t][i] = (short)to_bf16(pre > 0.f ? pre : 0.f);
        }
    }
    float part = 0.f;
#pragma unroll
    for (int t2 = 0; t2 < 8; ++t2) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = mfma(load4(N.W2b + (16 * t2 + col) * kH + 16 * t + 4 * kg), o.h1[t], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * t2 + 4 * kg + i;
            const float pre = acc[i] + N.b2[f];
            o.a2p[t2][i] = pre;
            const float h = from_bf16(to_bf16(pre > 0.f ? pre : 0.f));
            o.h2[t2][i] = h;
            part += from_bf16(N.w3b[f]) * h;
        }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    o.y = part + N.b3[0];
}

__global__ __launch_bounds__(256) void forward_kernel(const float *__restrict__ X, int64_t n, Net N,
                                                      float *__restrict__ logits) {
    const int lane = threadIdx.x & 63;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t p = tile * 16 + (lane & 15);
        float zf[4];
        const bf16x4 z = input_operand(X, p, p < n, lane >> 4, N, zf);
        Fwd o;
        forward_tile(z, N, lane, o);
        if (lane < 16 && p < n) logits[p] = o.y;
    }
}

// One Adam step of parameter x (Kingma & Ba, bias-corrected moments) when
// A.update, then its bf16 copies from the fp32 master.
struct AdamArgs {
    float *theta, *m, *v;
    uint16_t *W1b, *W2b, *W2Tb, *w3b;
    float lr, b1, b2, eps, c1, c2;
    int update;
};

__device__ __forceinline__ void adam_one(const AdamArgs &A, int x, float g) {
    float w = A.theta[x];
    if (A.update) {
        const float mm = A.b1 * A.m[x] + (1.f - A.b1) * g;
        const float vv = A.b2 * A.v[x] + (1.f - A.b2) * g * g;
        A.m[x] = mm;
        A.v[x] = vv;
        w -= A.lr * (mm / A.c1) / (sqrtf(vv / A.c2) + A.eps);
        A.theta[x] = w;
    }
    const uint16_t h = to_bf16(w);
    if (x < kMlpOffB1) {
        A.W1b[x] = h;
    } else if (x >= kMlpOffW2 && x < kMlpOffB2) {
        const int r = (x - kMlpOffW2) / kH, c = (x - kMlpOffW2) % kH;
        A.W2b[r * kH + c] = h;
        A.W2Tb[c * kH + r] = h;
    } else if (x >= kMlpOffW3 && x < kMlpOffB3) {
        A.w3b[x - kMlpOffW3] = h;
    }
}

// Forward + backward of 16 pairs per wave for one minibatch.  Pairs of the
// batch are examples order[off + p]; p >= count are padding (zero input and
// gradient).  Writes ZT, H1, DH2 and DH1 (bf16, [B / 16][feature][16]) and,
// per block, the sums of the loss and of the bias /
// w3 gradients over its pairs into part[block][kMlpPartN] (slot 0 the loss,
// then b1, b2, w3, b3), in a fixed order: no atomics, so a minibatch's
// gradient is the same on every run.
struct Train {
    const float *X;
    const uint8_t *labels;
    const int32_t *order;
    int64_t off, count;  // batch = examples order[off .. off + count)
    int B;               // padded batch size (multiple of 16)
    float pos_weight, inv_n;
    uint16_t *ZT, *H1, *DH2, *DH1;
    float *part;
};

// Part slots: the gradient of parameter x >= kMlpOffB2 (b2, w3, b3 are
// contiguous there) sits in slot kPartB2 + x - kMlpOffB2.
constexpr int kPartB1 = 1, kPartB2 = 1 + kH, kPartW3 = 1 + 2 * kH, kPartB3 = 1 + 3 * kH;

// Sums v[0..N) of every lane over the 16 lanes of its lane group (same
// lane >> 4), reduce-scatter style: after the four exchange steps lane col
// holds the group's totals of v[N/16 * col .. + N/16) in v[0 .. N/16).  Each
// step hands half of the remaining values to the partner lane, so the wave
// does N - N/16 exchanges instead of 4N.
template <int N>
__device__ __forceinline__ void group_reduce_scatter(float (&v)[N], int col) {
#pragma unroll
    for (int m = 8, half = N / 2; m >= 1; m >>= 1, half >>= 1) {
        const bool up = (col & m) != 0;
#pragma unroll
        for (int q = 0; q < half; ++q) {
            const float lo = v[q], hi = v[half + q];  // values, so the selects below are not on addresses
            const float keep = up ? hi : lo, give = up ? lo : hi;
            v[q] = keep + __shfl_xor(give, m, 64);
        }
    }
}

__global__ __launch_bounds__(64 * kMlpTrainWaves) void train_tile_kernel(Net N, Train T) {
    constexpr int W = kMlpTrainWaves;
    __shared__ float acc_lds[W][kMlpPartN];  // one row per wave
    const int lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4, w = threadIdx.x >> 6;
    for (int x = threadIdx.x; x < W * kMlpPartN; x += blockDim.x) (&acc_lds[0][0])[x] = 0.f;
    __syncthreads();
    float *my = acc_lds[w];
    const int tile = blockIdx.x * W + w;  // the grid holds one wave per tile
    if (tile < T.B / 16) {
        const int pb = tile * 16 + col;  // pair index within the batch
        const bool valid = pb < T.count;
        const int64_t ex = valid ? (int64_t)T.order[T.off + pb] : 0;
        float zf[4];
        const bf16x4 z = input_operand(T.X, ex, valid, kg, N, zf);
        uint16_t *const zt = T.ZT + (size_t)tile * kIn * 16 + col;
        uint16_t *const h1 = T.H1 + (size_t)tile * kH * 16 + col;
        uint16_t *const dh2 = T.DH2 + (size_t)tile * kH * 16 + col;
        uint16_t *const dh1 = T.DH1 + (size_t)tile * kH * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) zt[(4 * kg + i) * 16] = (uint16_t)z[i];
        Fwd o;
        forward_tile(z, N, lane, o);
        const float t = valid ? (float)T.labels[ex] : 0.f;
        const float s = 1.f / (1.f + expf(-o.y));
        const float dy = valid ? (T.pos_weight * t * (s - 1.f) + (1.f - t) * s) * T.inv_n : 0.f;
        // loss: softplus(-y) for positives, softplus(y) for negatives, computed stably
        const float sp = log1pf(expf(-fabsf(o.y)));
        float lo = valid ? (T.pos_weight * t * (fmaxf(-o.y, 0.f) + sp) + (1.f - t) * (fmaxf(o.y, 0.f) + sp)) * T.inv_n
                         : 0.f;
        float sdy = dy;
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) {
            lo += __shfl_xor(lo, m, 64);
            sdy += __shfl_xor(sdy, m, 64);
        }
        if (lane == 0) {
            my[0] += lo;
            my[kPartB3] += sdy;
        }
        // layer 3 / layer 2 backward, in the accumulator layout
        bf16x4 dh2op[8];
        float gw3[32], gb2[32];  // [4 * t2 + i]: feature 16 * t2 + 4 * kg + i
#pragma unroll
        for (int t2 = 0; t2 < 8; ++t2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * t2 + 4 * kg + i;
                gw3[4 * t2 + i] = dy * o.h2[t2][i];
                const float d = o.a2p[t2][i] > 0.f ? dy * from_bf16(N.w3b[f]) : 0.f;
                gb2[4 * t2 + i] = d;
                const uint16_t db = to_bf16(d);
                dh2op[t2][i] = (short)db;
                dh2[f * 16] = db;
                h1[f * 16] = (uint16_t)o.h1[t2][i];
            }
        }
        group_reduce_scatter(gw3, col);
        group_reduce_scatter(gb2, col);
        // lane col now holds j = 2 col, 2 col + 1: feature 16 (j / 4) + 4 kg + j % 4
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int j = 2 * col + r, f = 16 * (j >> 2) + 4 * kg + (j & 3);
            my[kPartW3 + f] += gw3[r];
            my[kPartB2 + f] += gb2[r];
        }
        // dH1 = W2^T dH2 (transposed weights as the A operand)
        float gb1[32];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t2 = 0; t2 < 8; ++t2)
                acc = mfma(load4(N.W2Tb + (16 * t + col) * kH + 16 * t2 + 4 * kg), dh2op[t2], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * t + 4 * kg + i;
                const float d = o.a1p[t][i] > 0.f ? acc[i] : 0.f;
                gb1[4 * t + i] = d;
                dh1[f * 16] = to_bf16(d);
            }
        }
        group_reduce_scatter(gb1, col);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int j = 2 * col + r;
            my[kPartB1 + 16 * (j >> 2) + 4 * kg + (j & 3)] += gb1[r];
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < kMlpPartN; x += blockDim.x) {
        float a = acc_lds[0][x];
#pragma unroll
        for (int i = 1; i < W; ++i) a += acc_lds[i][x];
        T.part[(size_t)blockIdx.x * kMlpPartN + x] = a;
    }
}

// Weight gradients over one minibatch, split over the pairs: dW2 = DH2 H1^T
// (64 tiles of 16x16) and dW1 = DH1 Z^T (8 tiles), each over chunks of
// kMlpSplitK pairs.  One wave per (tile, chunk); chunk c's partial products
// go to wp2 + c * 128 * 128 and wp1 + c * 128 * 16 ([row][col] as the
// parameters), to be summed in chunk order.
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t *__restrict__ DH2, const uint16_t *__restrict__ H1,
                                                    const uint16_t *__restrict__ DH1,
                                                    const uint16_t *__restrict__ ZT, int B, int chunks,
                                                    float *__restrict__ wp2, float *__restrict__ wp1) {
    constexpr int kTiles2 = (kH / 16) * (kH / 16), kTiles = kTiles2 + kH / 16;
    const int lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= kTiles * chunks) return;
    const int tile = wave % kTiles, c = wave / kTiles;
    const uint16_t *A, *Bm;
    float *C;
    int Nn, mt, nt;
    if (tile < kTiles2) {
        A = DH2, Bm = H1, Nn = kH, mt = tile / (kH / 16), nt = tile % (kH / 16), C = wp2 + (size_t)c * kH * kH;
    } else {
        A = DH1, Bm = ZT, Nn = kIn, mt = tile - kTiles2, nt = 0, C = wp1 + (size_t)c * kH * kIn;
    }
    // pair tiles [t0, t1) of this chunk; a tile of A holds kH features, of Bm Nn
    const int t0 = c * (kMlpSplitK / 16), t1 = min(B / 16, t0 + kMlpSplitK / 16);
    const uint16_t *ap = A + (size_t)t0 * kH * 16 + (16 * mt + col) * 16 + 4 * kg;
    const uint16_t *bp = Bm + (size_t)t0 * Nn * 16 + (16 * nt + col) * 16 + 4 * kg;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int t = t0; t < t1; ++t, ap += kH * 16, bp += Nn * 16) acc = mfma(load4(ap), load4(bp), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) C[(size_t)(16 * mt + 4 * kg + i) * Nn + 16 * nt + col] = acc[i];
}

// The minibatch gradient from the partials, summed in a fixed order, then
// (A.update) the Adam step of every parameter.  Threads [0, nW) take one
// weight of W1 or W2 each (sum over the chunks); then one wave per part slot
// sums the blocks' values (lane-strided, then a fixed shuffle tree) into the
// bias / w3 gradient, and slot 0 adds the batch loss to *loss.  The gradient
// is written to grad either way.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *__restrict__ part, int nblk,
                                                          const float *__restrict__ wp2,
                                                          const float *__restrict__ wp1, int chunks,
                                                          float *__restrict__ grad, float *__restrict__ loss,
                                                          AdamArgs A) {
    constexpr int nW1 = kH * kIn, nW2 = kH * kH, nW = nW1 + nW2;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nW) {
        const bool w1 = x < nW1;
        const float *src = w1 ? wp1 + x : wp2 + (x - nW1);
        const size_t stride = w1 ? nW1 : nW2;
        float a = 0.f;
#pragma unroll 8
        for (int c = 0; c < chunks; ++c) a += src[(size_t)c * stride];
        const int px = w1 ? kMlpOffW1 + x : kMlpOffW2 + x - nW1;
        grad[px] = a;
        if (A.update) adam_one(A, px, a);
        return;
    }
    const int wbase = (nW + 255) / 256 * 4;  // first wave of the slot sums
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6) - wbase, lane = threadIdx.x & 63;
    if (slot < 0 || slot >= kMlpPartN) return;
    float a = 0.f;
    for (int b = lane; b < nblk; b += 64) a += part[(size_t)b * kMlpPartN + slot];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m, 64);
    if (lane != 0) return;
    if (slot == 0) {
        *loss += a;
        return;
    }
    const int px = slot < kPartB2 ? kMlpOffB1 + slot - kPartB1 : kMlpOffB2 + slot - kPartB2;
    grad[px] = a;
    if (A.update) adam_one(A, px, a);
}

// bf16 copies of the fp32 masters (no update).
__global__ void refresh_kernel(AdamArgs A) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < kMlpParams; x += gridDim.x * blockDim.x)
        adam_one(A, x, 0.f);
}

// mean / std (population) of each feature column, fp64 accumulation
__global__ void moments_kernel(const float *__restrict__ X, int64_t n, double *__restrict__ acc) {
    __shared__ double s[2 * kIn];
    if (threadIdx.x < 2 * kIn) s[threadIdx.x] = 0.0;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n * kIn; q += (int64_t)gridDim.x * blockDim.x) {
        const int f = (int)(q % kIn);
        const double x = X[q];
        atomicAdd(&s[f], x);
        atomicAdd(&s[kIn + f], x * x);
    }
    __syncthreads();
    if (threadIdx.x < 2 * kIn) atomicAdd(&acc[threadIdx.x], s[threadIdx.x]);
}

__global__ void moments_finish_kernel(const double *__restrict__ acc, int64_t n, float *__restrict__ mean,
                                      float *__restrict__ stdv) {
    const int f = threadIdx.x;
    if (f < kIn) {
        const double mu = acc[f] / (double)n;
        const double var = acc[kIn + f] / (double)n - mu * mu;
        mean[f] = (float)mu;
        stdv[f] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
    }
}

__global__ void keep_kernel(const float *__restrict__ logits, int64_t n, float tau, uint8_t *__restrict__ keep) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        keep[q] = logits[q] >= tau ? 1 : 0;
}

__global__ void compact_kernel(const uint8_t *__restrict__ keep, const uint32_t *__restrict__ pos, int64_t n,
                               const uint32_t *__restrict__ in0, const uint32_t *__restrict__ in1,
                               const uint32_t *__restrict__ in2, const uint32_t *__restrict__ in3,
                               const uint32_t *__restrict__ in4, uint32_t *__restrict__ out0,
                               uint32_t *__restrict__ out1, uint32_t *__restrict__ out2, uint32_t *__restrict__ out3,
                               uint32_t *__restrict__ out4) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (!keep[q]) continue;
        const uint32_t p = pos[q];
        out0[p] = in0[q];
        out1[p] = in1[q];
        out2[p] = in2[q];
        out3[p] = in3[q];
        out4[p] = in4[q];
    }
}

// flag[0] = min position of an index outside [0, limit) (stays ~0 if none)
__global__ void check_order_kernel(const int32_t *__restrict__ order, int64_t n, int64_t limit,
                                   unsigned long long *__restrict__ flag) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = order[q];
        if (v < 0 || (int64_t)v >= limit) atomicMin(flag, (unsigned long long)q);
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

Net net_of(const MlpState &S) {
    Net N;
    N.W1b = S.W1b;
    N.W2b = S.W2b;
    N.W2Tb = S.W2Tb;
    N.w3b = S.w3b;
    N.b1 = S.theta + kMlpOffB1;
    N.b2 = S.theta + kMlpOffB2;
    N.b3 = S.theta + kMlpOffB3;
    N.mean = S.mean;
    N.stdv = S.stdv;
    return N;
}

AdamArgs adam_args(const MlpState &S, float lr, int step) {
    AdamArgs A;
    A.theta = S.theta;
    A.m = S.m;
    A.v = S.v;
    A.W1b = S.W1b;
    A.W2b = S.W2b;
    A.W2Tb = S.W2Tb;
    A.w3b = S.w3b;
    A.b1 = 0.9f;
    A.b2 = 0.999f;
    A.eps = 1e-8f;
    A.lr = lr;
    A.update = step > 0;
    A.c1 = step > 0 ? 1.f - powf(A.b1, (float)step) : 1.f;
    A.c2 = step > 0 ? 1.f - powf(A.b2, (float)step) : 1.f;
    return A;
}

}  // namespace

hipError_t mlp_refresh(const MlpState &S, hipStream_t s) {
    refresh_kernel<<<grid_for(kMlpParams), 256, 0, s>>>(adam_args(S, 0.f, 0));
    return hipGetLastError();
}

hipError_t mlp_features(const uint8_t *codes, const int64_t *offsets, int64_t n, const uint32_t *lo,
                        const uint32_t *hi, const uint32_t *count, const uint32_t *s1, const uint32_t *s2,
                        int64_t npairs, float *comp, float *F, hipStream_t s) {
    if (n > 0) {
        comp_kernel<<<grid_for(n), 256, 0, s>>>(codes, offsets, n, comp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (npairs <= 0) return hipSuccess;
    features_kernel<<<grid_for(npairs), 256, 0, s>>>(lo, hi, count, s1, s2, npairs, offsets, comp, F);
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpState &S, const float *X, int64_t n, float *logits, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    forward_kernel<<<(unsigned)blocks, 256, 0, s>>>(X, n, net_of(S), logits);
    return hipGetLastError();
}

hipError_t mlp_moments(const float *X, int64_t n, double *acc, float *mean, float *stdv, hipStream_t s) {
    hipError_t e = fill<uint64_t>((uint64_t *)acc, 2 * kIn, 0ull, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        moments_kernel<<<grid_for(n * kIn / 8 + 1), 256, 0, s>>>(X, n, acc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    moments_finish_kernel<<<1, 64, 0, s>>>(acc, n > 0 ? n : 1, mean, stdv);
    return hipGetLastError();
}

hipError_t mlp_batch_grad(const MlpState &S, const float *X, const uint8_t *labels, const int32_t *order, int64_t off,
                          int64_t count, int B, float pos_weight, float *loss, float lr, int step, hipStream_t s) {
    if (B <= 0 || B % 16 || B > S.batch_cap || count > B) return hipErrorInvalidValue;
    Train T;
    T.X = X;
    T.labels = labels;
    T.order = order;
    T.off = off;
    T.count = count;
    T.B = B;
    T.pos_weight = pos_weight;
    T.inv_n = 1.f / (float)(count > 0 ? count : 1);
    T.ZT = S.ZT;
    T.H1 = S.H1;
    T.DH2 = S.DH2;
    T.DH1 = S.DH1;
    T.part = S.part;
    const int tiles = B / 16, nblk = (tiles + kMlpTrainWaves - 1) / kMlpTrainWaves;  // rows of part
    train_tile_kernel<<<nblk, 64 * kMlpTrainWaves, 0, s>>>(net_of(S), T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int chunks = (B + kMlpSplitK - 1) / kMlpSplitK;  // <= batch_cap / kMlpSplitK
    float *wp2 = S.wpart, *wp1 = S.wpart + (size_t)chunks * kH * kH;
    const int waves = (kH / 16 * kH / 16 + kH / 16) * chunks;
    wgrad_kernel<<<(waves + 3) / 4, 256, 0, s>>>(S.DH2, S.H1, S.DH1, S.ZT, B, chunks, wp2, wp1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nW = kH * kIn + kH * kH;
    const int rblocks = (nW + 255) / 256 + (kMlpPartN + 3) / 4;
    grad_reduce_kernel<<<rblocks, 256, 0, s>>>(S.part, nblk, wp2, wp1, chunks, S.grad, loss,
                                                adam_args(S, lr, step));
    return hipGetLastError();
}


hipError_t mlp_keep(const float *logits, int64_t n, float tau, uint8_t *keep, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    keep_kernel<<<grid_for(n), 256, 0, s>>>(logits, n, tau, keep);
    return hipGetLastError();
}

hipError_t mlp_check_order(const int32_t *order, int64_t n, int64_t limit, unsigned long long *flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    check_order_kernel<<<grid_for(n), 256, 0, s>>>(order, n, limit, flag);
    return hipGetLastError();
}

hipError_t compact5(const uint8_t *keep, const uint32_t *pos, int64_t n, const uint32_t *const in[5],
                    uint32_t *const out[5], hipStream_t s) {
    if (n <= 0) return hipSuccess;
    compact_kernel<<<grid_for(n), 256, 0, s>>>(keep, pos, n, in[0], in[1], in[2], in[3], in[4], out[0], out[1],
                                                out[2], out[3], out[4]);
    return hipGetLastError();
}

}  // namespace pastis
