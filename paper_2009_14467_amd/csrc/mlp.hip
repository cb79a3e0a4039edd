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
// Training stores activations and gradients feature-major ([feature][pair],
// bf16) so both operands of the weight-gradient GEMMs (reductions over the
// batch) load 4 consecutive bf16 per lane.
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

// Forward + backward of 16 pairs per wave for one minibatch.  Pairs of the
// batch are examples order[off + p]; p >= count are padding (zero input and
// gradient).  Writes ZT [16][B], H1 [128][B], DH2 [128][B], DH1 [128][B]
// (bf16, feature-major) and accumulates bias / w3 gradients and the loss.
struct Train {
    const float *X;
    const uint8_t *labels;
    const int32_t *order;
    int64_t off, count;  // batch = examples order[off .. off + count)
    int B;               // padded batch size (multiple of 16)
    float pos_weight, inv_n;
    uint16_t *ZT, *H1, *DH2, *DH1;
    float *g_b1, *g_b2, *g_w3, *g_b3, *loss;
};

__global__ __launch_bounds__(256) void train_tile_kernel(Net N, Train T) {
    const int lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4;
    const int tiles = T.B / 16;
    for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += gridDim.x * 4) {
        const int pb = tile * 16 + col;  // pair index within the batch
        const bool valid = pb < T.count;
        const int64_t ex = valid ? (int64_t)T.order[T.off + pb] : 0;
        float zf[4];
        const bf16x4 z = input_operand(T.X, ex, valid, kg, N, zf);
#pragma unroll
        for (int i = 0; i < 4; ++i) T.ZT[(size_t)(4 * kg + i) * T.B + pb] = (uint16_t)z[i];
        Fwd o;
        forward_tile(z, N, lane, o);
        const float t = valid ? (float)T.labels[ex] : 0.f;
        const float s = 1.f / (1.f + expf(-o.y));
        const float dy = valid ? (T.pos_weight * t * (s - 1.f) + (1.f - t) * s) * T.inv_n : 0.f;
        if (lane < 16 && valid) {
            // softplus(-y) = -log(s), softplus(y) = y - log(s)... computed stably
            const float sp_neg = fmaxf(-o.y, 0.f) + log1pf(expf(-fabsf(o.y)));
            const float sp_pos = fmaxf(o.y, 0.f) + log1pf(expf(-fabsf(o.y)));
            atomicAdd(T.loss, (T.pos_weight * t * sp_neg + (1.f - t) * sp_pos) * T.inv_n);
        }
        float sdy = dy;  // sum over the 16 pairs of the lane group
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) sdy += __shfl_xor(sdy, m, 64);
        if (lane == 0) atomicAdd(T.g_b3, sdy);
        // layer 3 / layer 2 backward, in the accumulator layout
        bf16x4 dh2op[8];
#pragma unroll
        for (int t2 = 0; t2 < 8; ++t2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * t2 + 4 * kg + i;
                float gw3 = dy * o.h2[t2][i];
                const float d = o.a2p[t2][i] > 0.f ? dy * from_bf16(N.w3b[f]) : 0.f;
                float gb2 = d;
                const uint16_t db = to_bf16(d);
                dh2op[t2][i] = (short)db;
                T.DH2[(size_t)f * T.B + pb] = db;
                T.H1[(size_t)f * T.B + pb] = (uint16_t)o.h1[t2][i];
                // sum over the 16 pairs of this lane group
#pragma unroll
                for (int m = 1; m < 16; m <<= 1) {
                    gw3 += __shfl_xor(gw3, m, 64);
                    gb2 += __shfl_xor(gb2, m, 64);
                }
                if (col == 0) {
                    atomicAdd(&T.g_w3[f], gw3);
                    atomicAdd(&T.g_b2[f], gb2);
                }
            }
        }
        // dH1 = W2^T dH2 (transposed weights as the A operand)
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
                float gb1 = d;
                T.DH1[(size_t)f * T.B + pb] = to_bf16(d);
#pragma unroll
                for (int m = 1; m < 16; m <<= 1) gb1 += __shfl_xor(gb1, m, 64);
                if (col == 0) atomicAdd(&T.g_b1[f], gb1);
            }
        }
    }
}

// C[M][N] = sum_k A[m][k] * Bm[n][k] for bf16 A [M][K], Bm [N][K] (K contiguous,
// K a multiple of 16); one wave per 16x16 output tile.
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bm,
                                                      int M, int Nn, int K, float *__restrict__ C) {
    const int lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4;
    const int tiles_n = Nn / 16, tiles = (M / 16) * tiles_n;
    for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += gridDim.x * 4) {
        const int mt = tile / tiles_n, nt = tile % tiles_n;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const uint16_t *ap = A + (size_t)(16 * mt + col) * K + 4 * kg;
        const uint16_t *bp = Bm + (size_t)(16 * nt + col) * K + 4 * kg;
        for (int k0 = 0; k0 < K; k0 += 16) acc = mfma(load4(ap + k0), load4(bp + k0), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) C[(size_t)(16 * mt + 4 * kg + i) * Nn + 16 * nt + col] = acc[i];
    }
}

// Adam on the fp32 masters, then fresh bf16 copies; clears the atomically
// accumulated gradients.  grad layout = parameter layout.
__global__ void adam_kernel(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                            float *__restrict__ grad, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                            uint16_t *__restrict__ W1b, uint16_t *__restrict__ W2b, uint16_t *__restrict__ W2Tb,
                            uint16_t *__restrict__ w3b, int update) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        float w = theta[x];
        if (update) {
            const float g = grad[x];
            const float mm = b1 * m[x] + (1.f - b1) * g;
            const float vv = b2 * v[x] + (1.f - b2) * g * g;
            m[x] = mm;
            v[x] = vv;
            w -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
            theta[x] = w;
        }
        grad[x] = 0.f;
        const uint16_t h = to_bf16(w);
        if (x < kMlpOffB1) {
            W1b[x] = h;
        } else if (x >= kMlpOffW2 && x < kMlpOffB2) {
            const int r = (x - kMlpOffW2) / kH, c = (x - kMlpOffW2) % kH;
            W2b[r * kH + c] = h;
            W2Tb[c * kH + r] = h;
        } else if (x >= kMlpOffW3 && x < kMlpOffB3) {
            w3b[x - kMlpOffW3] = h;
        }
    }
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

}  // namespace

hipError_t mlp_refresh(const MlpState &S, hipStream_t s) {
    adam_kernel<<<grid_for(kMlpParams), 256, 0, s>>>(S.theta, S.m, S.v, S.grad, kMlpParams, 0.f, 0.f, 0.f, 0.f, 1.f,
                                                      1.f, S.W1b, S.W2b, S.W2Tb, S.w3b, 0);
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
                          int64_t count, int B, float pos_weight, float *loss, hipStream_t s) {
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
    T.g_b1 = S.grad + kMlpOffB1;
    T.g_b2 = S.grad + kMlpOffB2;
    T.g_w3 = S.grad + kMlpOffW3;
    T.g_b3 = S.grad + kMlpOffB3;
    T.loss = loss;
    const int tiles = B / 16;
    train_tile_kernel<<<(tiles + 3) / 4, 256, 0, s>>>(net_of(S), T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // dW2 = DH2 H1^T over the batch, dW1 = DH1 Z^T
    gemm_nt_kernel<<<16, 256, 0, s>>>(S.DH2, S.H1, kH, kH, B, S.grad + kMlpOffW2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    gemm_nt_kernel<<<2, 256, 0, s>>>(S.DH1, S.ZT, kH, kIn, B, S.grad + kMlpOffW1);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpState &S, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<grid_for(kMlpParams), 256, 0, s>>>(S.theta, S.m, S.v, S.grad, kMlpParams, lr, b1, b2, 1e-8f, c1, c2,
                                                      S.W1b, S.W2b, S.W2Tb, S.w3b, 1);
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
